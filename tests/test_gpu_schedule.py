"""Launch schedules of batched plans: every schedule gives bitwise the same
NLL and gradient (tiles write their own partials, summed in tile order), the
autotuner keeps one of its candidates, and bad schedules are refused."""
import sys

import numpy as np
import pytest

from paper_1706_01420_amd import toys
from paper_1706_01420_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def lib():
    from paper_1706_01420_amd import ipx
    return ipx


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.ipx_create(0)
    yield c
    lib.ipx_destroy(c)


@pytest.mark.parametrize("model", [2, 3])
def test_schedules_do_not_change_results(lib, ctx, model):
    sizes = [30000, 5000, 77777, 1, 12345, 0, 40000]
    th = np.array(W.THETA_GEN[model])
    say("schedules model", model, "segments", len(sizes))
    ds = [lib.ipx_dataset_create(ctx, model, *W.events(model, n, seed=100 + j)) if n else None
          for j, n in enumerate(sizes)]
    ds = [d for d in ds if d is not None]
    plan = lib.ipx_plan_create(ctx, ds)
    try:
        rng = np.random.default_rng(5)
        thb = np.tile(th, (len(ds), 1)) * (1.0 + 1e-3 * rng.standard_normal((len(ds), th.size)))
        ref_f, ref_g = lib.nll_eval_batch(ctx, plan, thb, grad=True)
        ref_e = lib.nll_eval_batch(ctx, plan, thb)
        variants = (0, 1) if model == 3 else (0,)
        for wg, order, graph, var in ([(w, o, 1, v) for w in (0, 1, 7, 256, 2048) for o in (0, 1) for v in variants]
                                      + [(0, 0, 0, 0), (7, 1, 0, variants[-1])]):
            lib.ipx_plan_set_schedule(plan, wg, order, graph, var)
            assert lib.ipx_plan_get_schedule(plan) == {"workgroups": wg, "order": order, "graph": graph,
                                                       "variant": var}
            for _ in range(2):   # the first call captures the graph (if any), the second replays it
                f, g = lib.nll_eval_batch(ctx, plan, thb, grad=True)
                assert np.array_equal(f, ref_f) and np.array_equal(g, ref_g), (wg, order, graph, var)
                assert np.array_equal(lib.nll_eval_batch(ctx, plan, thb), ref_e), (wg, order, graph, var)
        best, us, rows = lib.ipx_plan_autotune(ctx, plan, thb, grad=True, reps=2)
        say("autotune", best, round(us, 1), rows)
        assert best in [r[0] for r in rows] and us == min(r[1] for r in rows)
        assert lib.ipx_plan_get_schedule(plan) == best
        f, g = lib.nll_eval_batch(ctx, plan, thb, grad=True)
        assert np.array_equal(f, ref_f) and np.array_equal(g, ref_g)
        for bad in ((-1, 0, 1), (0, 2, 1), (0, 0, 2), (0, 0, 1, 2) if model == 3 else (0, 0, 1, 1)):
            with pytest.raises(lib.IpxError) as e:
                lib.ipx_plan_set_schedule(plan, *bad)
            assert e.value.status == lib.IPX_EINVAL
    finally:
        lib.ipx_plan_destroy(plan)
        for d in ds:
            lib.ipx_dataset_destroy(ctx, d)


def test_fit_batched_with_tuned_schedule(lib, ctx, tmp_path, monkeypatch):
    monkeypatch.setenv("IPX_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    th = np.array(W.THETA_GEN[1])
    ds = toys.generate(lib, ctx, 1, th, 31, [4000] * 8)
    try:
        steps = toys.steps_for(1, [4000] * 8)
        start = th[None, :] + 0.5 * steps
        a = toys.fit_batched(lib, ctx, 1, ds, start, steps)
        b = toys.fit_batched(lib, ctx, 1, ds, start, steps, tune=True)
        c = toys.fit_batched(lib, ctx, 1, ds, start, steps, tune=True)   # from the cache
        assert np.array_equal(a["theta"], b["theta"]) and np.array_equal(a["theta"], c["theta"])
        assert (tmp_path / "tune.json").exists()
    finally:
        for d in ds:
            lib.ipx_dataset_destroy(ctx, d)
