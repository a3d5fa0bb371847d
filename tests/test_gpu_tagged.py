"""GPU parity of the tagged angular model (IPX_MODEL_ANGTIME_TAGGED), the
per-dataset angular constants (efficiency weights xi_k, C_SP) and the
simultaneous fit over categories (paper Example 2: per KK-mass bin and
flavour, each category normalised on its own), against the oracle.

Tolerances as tests/test_gpu_parity.py: NLL relative 1e-10; gradient
|g - g_ref| <= 1e-6 |g_ref| + 1e-9 sum_i |w_i d ln P_i/d theta_j| + 1e-13 n;
per-event terms |got - ref| <= 1e-12 max(1, |ref|); whatever the GPU computes
twice (plain, batched, served, simultaneous) agrees bitwise.
"""
import math
import sys

import numpy as np
import pytest

import pins
from storage_order import band_order

from oracle import models as M
from oracle import nll as N
from oracle import sim as S
from paper_1706_01420_amd import workloads as W

pytestmark = pytest.mark.gpu

SMALL_N = 9 * 1024 + 301
THETAS = [M.THETA_GEN[4],
          (0.45, 0.3, 0.2, 2.5, 0.4, -1.0, 0.7, 0.12, 17.0, 0.4, 5370.0, 12.0),
          (0.6, 0.1, 0.1, 3.0, 3.0, 0.5, 0.6, -0.05, 18.5, -0.7, 5360.0, 18.0)]


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


def xi_of_acceptance():
    ck, cl, ph, w = pins.angular_grid(8, 16)
    e = pins.acceptance(ck, cl, ph)
    return np.array([np.sum(w * e * f) for f in M.angular_functions(ck, cl, ph)])


def check_nll(got, ref):
    assert math.isfinite(got) and abs(got - ref) <= 1e-10 * abs(ref), (got, ref)


def check_grad(model, cols, w, theta, g, gref, settings=None):
    scale = np.abs(N.event_grad(model, cols, theta, settings) * (1.0 if w is None else w)).sum(axis=1)
    bound = 1e-6 * np.abs(gref) + 1e-9 * scale + 1e-13 * cols[0].shape[0]
    assert np.all(np.abs(g - gref) <= bound), (g, gref, np.abs(g - gref) / bound)


@pytest.mark.parametrize("weighted", [True, False])
def test_tagged_nll_and_gradient_match_oracle(lib, ctx, weighted):
    cols, w = W.events(4, SMALL_N, seed=61, weights=weighted)
    ds = lib.ipx_dataset_create(ctx, 4, cols, w)
    try:
        for i, th in enumerate(THETAS):
            say("tagged model theta", i, "weighted", weighted)
            check_nll(lib.nll_eval(ctx, ds, th), N.nll(4, cols, th, w))
            f, g = lib.nll_grad(ctx, ds, th)
            fref, gref = N.nll_grad(4, cols, th, w)
            check_nll(f, fref)
            check_grad(4, cols, w, th, g, gref)
    finally:
        lib.ipx_dataset_destroy(ctx, ds)


@pytest.mark.parametrize("q,omega", [(1.0, 0.0), (-1.0, 0.0), (1.0, 0.5)])
def test_pure_flavours_and_untagged(lib, ctx, q, omega):
    """qd = +1 everywhere is model 3 (bitwise: the same constants, the cos
    and sin terms scaled by exactly 1); qd = -1 is the anti-B_s PDF; qd = 0
    (omega = 1/2) the untagged one."""
    cols, w = W.events(4, 4 * 1024 + 17, seed=62, q=q, omega=omega)
    ds4 = lib.ipx_dataset_create(ctx, 4, cols, w)
    ds3 = lib.ipx_dataset_create(ctx, 3, cols[:6], w)
    try:
        th = THETAS[1]
        f4, g4 = lib.nll_grad(ctx, ds4, th)
        fref, gref = N.nll_grad(4, cols, th, w)
        check_nll(f4, fref)
        check_grad(4, cols, w, th, g4, gref)
        if q == 1.0 and omega == 0.0:
            f3, g3 = lib.nll_grad(ctx, ds3, th)
            assert f3 == f4 and np.array_equal(g3, g4)
    finally:
        lib.ipx_dataset_destroy(ctx, ds4)
        lib.ipx_dataset_destroy(ctx, ds3)


def test_tagged_per_event_terms_at_one_million(lib, ctx):
    n = 1_000_000
    cols, w = W.events(4, n, seed=63)
    ds = lib.ipx_dataset_create(ctx, 4, cols, w)
    try:
        order = band_order(cols[3], cols[4])
        sc = [c[order] for c in cols]
        sw = w[order]
        for c in range(7):
            assert np.array_equal(lib.ipx_dataset_read(ctx, ds, c), sc[c])
        for th in THETAS[:2]:
            say("tagged per-event terms n", n)
            got = lib.ipx_event_logp(ctx, ds, th).cpu().numpy()
            ref = N.log_pdf(4, sc, th) * sw
            err = np.abs(got - ref)
            assert np.all(err <= 1e-12 * np.maximum(1.0, np.abs(ref))), float(err.max())
            f = lib.nll_eval(ctx, ds, th)
            assert abs(-math.fsum(got.tolist()) - f) <= 1e-12 * abs(f)
            check_nll(f, -math.fsum(ref.tolist()))
    finally:
        lib.ipx_dataset_destroy(ctx, ds)


@pytest.mark.parametrize("model", [3, 4])
def test_efficiency_weights_and_csp(lib, ctx, model):
    cols, w = W.events(model, SMALL_N, seed=64)
    settings = {"xi": xi_of_acceptance(), "c_sp": 0.72}
    ds = lib.ipx_dataset_create(ctx, model, cols, w)
    try:
        th = THETAS[1]
        plain = lib.nll_grad(ctx, ds, th)
        lib.ipx_dataset_set_angular(ctx, ds, settings["xi"], settings["c_sp"])
        say("angular settings model", model)
        f, g = lib.nll_grad(ctx, ds, th)
        fref, gref = N.nll_grad(model, cols, th, w, settings)
        check_nll(f, fref)
        check_grad(model, cols, w, th, g, gref, settings)
        assert abs(f - plain[0]) > 1e-6 * abs(f)      # the settings change the likelihood
        got = lib.ipx_event_logp(ctx, ds, th).cpu().numpy()
        sc = [lib.ipx_dataset_read(ctx, ds, c) for c in range(M.NCOLS[model])]
        sw = lib.ipx_dataset_read(ctx, ds, M.NCOLS[model])
        ref = N.log_pdf(model, sc, th, settings) * sw
        assert np.all(np.abs(got - ref) <= 1e-12 * np.maximum(1.0, np.abs(ref)))
        # back to the defaults: bitwise the first evaluation
        lib.ipx_dataset_set_angular(ctx, ds, None, 1.0)
        f0, g0 = lib.nll_grad(ctx, ds, th)
        assert f0 == plain[0] and np.array_equal(g0, plain[1])
        with pytest.raises(lib.IpxError):
            lib.ipx_dataset_set_angular(ctx, ds, np.full(10, np.nan), 1.0)
    finally:
        lib.ipx_dataset_destroy(ctx, ds)


def test_settings_rejected_for_mass_models(lib, ctx):
    cols, w = W.events(1, 100, seed=1)
    ds = lib.ipx_dataset_create(ctx, 1, cols, w)
    try:
        with pytest.raises(lib.IpxError) as e:
            lib.ipx_dataset_set_angular(ctx, ds, None, 0.5)
        assert e.value.status == lib.IPX_EINVAL
    finally:
        lib.ipx_dataset_destroy(ctx, ds)


def _sim_setup(lib, ctx, nbins, n_each, seed):
    cats, dss, bins = [], [], []
    csp = [0.95, 0.81, 0.64, 0.52, 0.46, 0.39]
    for b in range(nbins):
        for q in (1.0, -1.0):
            cols, w = W.events(4, n_each + 37 * b, seed=seed + 10 * b + (q > 0), q=q)
            settings = {"c_sp": csp[b]}
            ds = lib.ipx_dataset_create(ctx, 4, cols, w)
            lib.ipx_dataset_set_angular(ctx, ds, None, csp[b])
            cats.append((4, cols, w, b, settings))
            dss.append(ds)
            bins.append(b)
    return cats, dss, bins


def _sim_theta(nbins, seed=0):
    rng = np.random.default_rng(seed)
    g = M.THETA_GEN[4]
    shared = [g[0], g[1], g[3], g[4], g[6], g[7], g[8], g[9], g[10], g[11]]
    per = []
    for _ in range(nbins):
        per += [0.02 + 0.06 * rng.uniform(), -0.5 + 1.5 * rng.uniform()]
    return np.array(shared + per)


def test_simultaneous_fit_matches_oracle(lib, ctx):
    """Six KK-mass bins x two flavours, twelve categories in one launch."""
    nbins = 6
    cats, dss, bins = _sim_setup(lib, ctx, nbins, 3000, 700)
    sim = lib.ipx_sim_create(ctx, dss, bins, nbins)
    try:
        assert lib.ipx_sim_nparams(sim) == 10 + 2 * nbins
        for k in range(2):
            th = _sim_theta(nbins, seed=k)
            say("simultaneous fit, 12 categories, point", k)
            f = lib.nll_sim(ctx, sim, th)
            fg, g = lib.nll_sim(ctx, sim, th, grad=True)
            assert fg == f
            fref, gref = S.nll_grad(cats, th)
            check_nll(f, fref)
            scale = np.zeros(th.size)
            for model, cols, w, b, settings in cats:
                sc = np.abs(N.event_grad(model, cols, S.category_theta(th, b), settings) * w).sum(axis=1)
                for j, i in enumerate(S.category_index(b)):
                    scale[i] += sc[j]
            n = sum(c[1][0].size for c in cats)
            bound = 1e-6 * np.abs(gref) + 1e-9 * scale + 1e-13 * n
            assert np.all(np.abs(g - gref) <= bound), (g, gref)
            # the same categories evaluated one by one give the same terms
            per = [lib.nll_grad(ctx, d, S.category_theta(th, b)) for d, b in zip(dss, bins)]
            assert abs(sum(p[0] for p in per) - f) <= 1e-13 * abs(f)
        bad = _sim_theta(nbins)
        bad[10] = 1.5                                  # Fs of bin 0 outside [0, 1]
        assert lib.nll_sim(ctx, sim, bad) == math.inf
    finally:
        lib.ipx_sim_destroy(sim)
        for d in dss:
            lib.ipx_dataset_destroy(ctx, d)


def test_tagged_batched_and_served_equal_plain(lib, ctx):
    dss, ths = [], []
    for j, n in enumerate([1, 700, 5000, 23000]):
        cols, w = W.events(4, n, seed=80 + j)
        dss.append(lib.ipx_dataset_create(ctx, 4, cols, w))
        ths.append(np.array(THETAS[j % 3]))
    lib.ipx_dataset_set_angular(ctx, dss[2], xi_of_acceptance(), 0.6)
    try:
        plan = lib.ipx_plan_create(ctx, dss)
        try:
            say("tagged batched")
            nll, g = lib.nll_eval_batch(ctx, plan, np.array(ths), grad=True)
        finally:
            lib.ipx_plan_destroy(plan)
        srv = lib.ipx_server_start(ctx, slots=8)
        try:
            say("tagged served")
            tickets = [lib.ipx_submit(srv, d, th, True) for d, th in zip(dss, ths)]
            res = [lib.ipx_wait(srv, t, 60.0) for t in tickets]
        finally:
            lib.ipx_server_stop(srv)
        for j, (d, th) in enumerate(zip(dss, ths)):
            f, gg = lib.nll_grad(ctx, d, th)
            assert nll[j] == f and np.array_equal(g[j], gg)
            assert res[j]["nll"] == f and np.array_equal(res[j]["grad"], gg)
    finally:
        for d in dss:
            lib.ipx_dataset_destroy(ctx, d)
