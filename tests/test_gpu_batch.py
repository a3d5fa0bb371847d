"""Batched evaluation: each dataset's NLL and gradient from nll_eval_batch must
be bitwise equal to nll_eval / nll_grad on that dataset alone, whatever else
is in the batch and whichever entries are active."""
import sys

import numpy as np
import pytest

from oracle import models as M
from oracle import nll as N
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


def _thetas(model, nb, seed):
    rng = np.random.default_rng(seed)
    base = np.array(M.THETA_GEN[model])
    out = []
    while len(out) < nb:
        th = base * (1.0 + 0.02 * rng.standard_normal(base.size))
        if M.theta_valid(model, th):
            out.append(th)
    return np.array(out)


@pytest.mark.parametrize("model", [1, 2, 3])
def test_batch_equals_plain_bitwise(lib, ctx, model):
    sizes = [0, 1, 1023, 1024, 5000, 13331, 777]
    ds, data = [], []
    try:
        for j, n in enumerate(sizes):
            cols, w = W.events(model, n, seed=100 + j)
            data.append((cols, w))
            ds.append(lib.ipx_dataset_create(ctx, model, cols, w))
        th = _thetas(model, len(ds), model)
        say("batch vs plain model", model)
        plan = lib.ipx_plan_create(ctx, ds)
        try:
            for rep in range(3):                       # first call captures, then replays
                f = lib.nll_eval_batch(ctx, plan, th)
                fg, g = lib.nll_eval_batch(ctx, plan, th, grad=True)
                for j, d in enumerate(ds):
                    assert f[j] == lib.nll_eval(ctx, d, th[j]), (rep, j)
                    fj, gj = lib.nll_grad(ctx, d, th[j])
                    assert fg[j] == fj and np.array_equal(g[j], gj), (rep, j)
            # and two entries directly against the oracle
            for j in (4, 5):
                cols, w = data[j]
                fref, gref = N.nll_grad(model, cols, th[j], w)
                assert abs(fg[j] - fref) <= 1e-10 * abs(fref), (j, fg[j], fref)
                scale = np.abs(N.event_grad(model, cols, th[j]) * (1.0 if w is None else w)).sum(axis=1)
                bound = 1e-6 * np.abs(gref) + 1e-9 * scale + 1e-13 * sizes[j]
                assert np.all(np.abs(g[j] - gref) <= bound), (j, g[j], gref)
            # masks: inactive entries are skipped, active ones unchanged
            act = np.array([j % 2 for j in range(len(ds))], dtype=np.uint8)
            th2 = th * (1 + 1e-3)
            f2, g2 = lib.nll_eval_batch(ctx, plan, th2, active=act, grad=True)
            for j, d in enumerate(ds):
                if act[j]:
                    fj, gj = lib.nll_grad(ctx, d, th2[j])
                    assert f2[j] == fj and np.array_equal(g2[j], gj)
                else:
                    assert np.isnan(f2[j])
            # an entry outside the domain does not disturb the others
            bad = th.copy()
            bad[2, 0] = -0.5
            f3 = lib.nll_eval_batch(ctx, plan, bad)
            assert f3[2] == np.inf
            assert all(f3[j] == f[j] for j in range(len(ds)) if j != 2)
        finally:
            lib.ipx_plan_destroy(plan)
    finally:
        for d in ds:
            lib.ipx_dataset_destroy(ctx, d)


def test_plan_errors(lib, ctx):
    a = lib.ipx_dataset_create(ctx, 1, W.events(1, 10)[0])
    b = lib.ipx_dataset_create(ctx, 2, W.events(2, 10)[0])
    try:
        with pytest.raises(lib.IpxError):
            lib.ipx_plan_create(ctx, [a, b])
        with pytest.raises(lib.IpxError):
            lib.ipx_plan_create(ctx, [a, a])
    finally:
        lib.ipx_dataset_destroy(ctx, a)
        lib.ipx_dataset_destroy(ctx, b)
