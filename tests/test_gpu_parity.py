"""GPU parity: libipx (through its C ABI) against the FP64 oracle.

Tolerances
  * NLL: relative 1e-10 (both sides are FP64; only the summation order and the
    special-function implementations differ, ~1e-14 expected).
  * gradient: |g - g_ref| <= 1e-6 |g_ref| + 1e-9 sum_i |w_i d ln P_i / d theta_j|
    + 1e-13 n (the second term bounds cancellation in sums whose total is near
    0; the third covers per-event derivatives that are themselves exact
    cancellations, e.g. d/ds where the resolution enters F and its integral
    alike and the difference is rounding noise of ~1e-17 per event).
  * anything the GPU computes twice (repeat calls, eval vs grad NLL, borrowed vs
    copied columns) must agree bitwise.
"""
import math
import sys

import numpy as np
import pytest

import theta_sweep
from storage_order import band_order

from oracle import models as M
from oracle import nll as N
from paper_1706_01420_amd import workloads as W

pytestmark = pytest.mark.gpu

MODELS = [1, 2, 3]
SMALL_N = 10 * 1024 + 517          # several tiles and a ragged tail


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


def thetas(model, k=4):
    """The generation point, then the first k - 1 random points of the parity
    sweep (drawn over each parameter's whole range, tests/theta_sweep.py)."""
    pts = [np.array(th) for lab, th, _ in theta_sweep.points(model) if lab.startswith("random")]
    return [np.array(M.THETA_GEN[model])] + pts[:k - 1]


def small_data(model, n=SMALL_N, seed=7):
    cols, w = W.events(model, n, seed=seed)
    return cols, w


def check_nll(got, ref, tol=1e-10):
    assert math.isfinite(got)
    assert abs(got - ref) <= tol * abs(ref), (got, ref, (got - ref) / ref)


def check_grad(model, cols, w, theta, g, gref):
    scale = np.abs(N.event_grad(model, cols, theta) * (1.0 if w is None else w)).sum(axis=1)
    bound = 1e-6 * np.abs(gref) + 1e-9 * scale + 1e-13 * cols[0].shape[0]
    assert np.all(np.abs(g - gref) <= bound), (g, gref, np.abs(g - gref) / np.maximum(bound, 1e-300))


@pytest.mark.parametrize("model", MODELS)
def test_nll_matches_oracle(lib, ctx, model):
    cols, w = small_data(model)
    ds = lib.ipx_dataset_create(ctx, model, cols, w)
    try:
        for i, th in enumerate(thetas(model)):
            say("nll_eval model", model, "n", SMALL_N, "theta", i)
            check_nll(lib.nll_eval(ctx, ds, th), N.nll(model, cols, th, w))
    finally:
        lib.ipx_dataset_destroy(ctx, ds)


@pytest.mark.parametrize("model", MODELS)
def test_grad_matches_oracle(lib, ctx, model):
    cols, w = small_data(model)
    ds = lib.ipx_dataset_create(ctx, model, cols, w)
    try:
        for i, th in enumerate(thetas(model, 3)):
            say("nll_grad model", model, "theta", i)
            f, g = lib.nll_grad(ctx, ds, th)
            fref, gref = N.nll_grad(model, cols, th, w)
            check_nll(f, fref)
            check_grad(model, cols, w, th, g, gref)
    finally:
        lib.ipx_dataset_destroy(ctx, ds)


@pytest.mark.parametrize("model", MODELS)
def test_eval_and_grad_nll_are_bitwise_equal_and_repeatable(lib, ctx, model):
    cols, w = small_data(model, seed=9)
    ds = lib.ipx_dataset_create(ctx, model, cols, w)
    try:
        th = thetas(model, 2)[1]
        say("determinism model", model)
        a = lib.nll_eval(ctx, ds, th)
        b = lib.nll_eval(ctx, ds, th)
        f1, g1 = lib.nll_grad(ctx, ds, th)
        f2, g2 = lib.nll_grad(ctx, ds, th)
        assert a == b == f1 == f2
        assert np.array_equal(g1, g2)
    finally:
        lib.ipx_dataset_destroy(ctx, ds)


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("n", [1, 31, 1024, 1025, 4097])
def test_small_and_ragged_sizes(lib, ctx, model, n):
    cols, w = small_data(model, n=n, seed=n)
    ds = lib.ipx_dataset_create(ctx, model, cols, w)
    try:
        th = thetas(model, 2)[1]
        say("size", n, "model", model)
        check_nll(lib.nll_eval(ctx, ds, th), N.nll(model, cols, th, w))
        f, g = lib.nll_grad(ctx, ds, th)
        fref, gref = N.nll_grad(model, cols, th, w)
        check_grad(model, cols, w, th, g, gref)
    finally:
        lib.ipx_dataset_destroy(ctx, ds)


@pytest.mark.parametrize("model", MODELS)
def test_empty_dataset(lib, ctx, model):
    say("empty model", model)
    ds = lib.ipx_dataset_create(ctx, model, [np.empty(0)] * M.NCOLS[model])
    try:
        assert lib.nll_eval(ctx, ds, M.THETA_GEN[model]) == 0.0
        f, g = lib.nll_grad(ctx, ds, M.THETA_GEN[model])
        assert f == 0.0 and np.all(g == 0.0)
    finally:
        lib.ipx_dataset_destroy(ctx, ds)


@pytest.mark.parametrize("model", MODELS)
def test_weights_on_every_model(lib, ctx, model):
    cols, _ = small_data(model, n=3000, seed=3)
    w = np.random.default_rng(4).uniform(0.5, 1.5, 3000)
    ds = lib.ipx_dataset_create(ctx, model, cols, w)
    dsu = lib.ipx_dataset_create(ctx, model, cols, None)
    try:
        th = M.THETA_GEN[model]
        say("weights model", model)
        check_nll(lib.nll_eval(ctx, ds, th), N.nll(model, cols, th, w))
        check_nll(lib.nll_eval(ctx, dsu, th), N.nll(model, cols, th, None))
    finally:
        lib.ipx_dataset_destroy(ctx, ds)
        lib.ipx_dataset_destroy(ctx, dsu)


def test_domain_errors(lib, ctx):
    cols, w = small_data(1, n=100)
    ds = lib.ipx_dataset_create(ctx, 1, cols, w)
    try:
        say("domain errors")
        assert lib.nll_eval(ctx, ds, (1.5, 5367.0, 15.0, 0.002)) == math.inf
        assert lib.nll_eval(ctx, ds, (0.3, 5367.0, 0.0, 0.002)) == math.inf
        f, g = lib.nll_grad(ctx, ds, (0.3, math.nan, 15.0, 0.002))
        assert f == math.inf and np.all(np.isnan(g))
        with pytest.raises(lib.IpxError):
            lib.nll_eval(ctx, ds, (0.3, 5367.0, 15.0))       # wrong parameter count
    finally:
        lib.ipx_dataset_destroy(ctx, ds)
    # an event with P = 0: pure Gaussian, event 40 sigma away
    ds = lib.ipx_dataset_create(ctx, 1, [np.array([5367.0, 5499.0])])
    try:
        assert lib.nll_eval(ctx, ds, (1.0, 5200.0, 3.0, 0.0)) == math.inf
    finally:
        lib.ipx_dataset_destroy(ctx, ds)


@pytest.mark.parametrize("model", MODELS)
def test_borrowed_device_columns_and_torch_stream(lib, ctx, model):
    import torch
    cols, w = small_data(model, n=5000, seed=5)
    dev = [torch.from_numpy(c).cuda() for c in cols]
    wd = None if w is None else torch.from_numpy(w).cuda()
    ds_copy = lib.ipx_dataset_create(ctx, model, cols, w, flags=lib.IPX_COPY_HOST | lib.IPX_KEEP_ORDER)
    ds_borrow = lib.ipx_dataset_create(ctx, model, dev, wd, flags=lib.IPX_BORROW_DEVICE)
    ds_dcopy = lib.ipx_dataset_create(ctx, model, dev, wd, flags=lib.IPX_COPY_DEVICE | lib.IPX_KEEP_ORDER)
    try:
        th = thetas(model, 2)[1]
        say("borrow/stream model", model)
        ref = lib.nll_eval(ctx, ds_copy, th)
        s = torch.cuda.Stream()
        assert lib.nll_eval(ctx, ds_borrow, th, stream=s) == ref
        assert lib.nll_eval(ctx, ds_dcopy, th) == ref
        assert lib.ipx_dataset_size(ds_borrow) == 5000
    finally:
        for d in (ds_copy, ds_borrow, ds_dcopy):
            lib.ipx_dataset_destroy(ctx, d)


@pytest.mark.parametrize("model", [2, 3])
def test_band_ordered_store_is_the_documented_permutation(lib, ctx, model):
    cols, w = small_data(model, n=6000, seed=12)
    ds = lib.ipx_dataset_create(ctx, model, cols, w)                      # resolution-band order
    dk = lib.ipx_dataset_create(ctx, model, cols, w, flags=lib.IPX_COPY_HOST | lib.IPX_KEEP_ORDER)
    try:
        say("band-ordered store model", model)
        tcol, scol = (1, 2) if model == 2 else (3, 4)
        got = [lib.ipx_dataset_read(ctx, ds, c) for c in range(len(cols))]
        order = band_order(cols[tcol], cols[scol])
        for c in range(len(cols)):
            assert np.array_equal(np.sort(got[c]), np.sort(cols[c]))
            assert np.array_equal(got[c], cols[c][order])
        if w is not None:
            assert np.array_equal(lib.ipx_dataset_read(ctx, ds, len(cols)), w[order])
        th = thetas(model, 2)[1]
        a, b = lib.nll_eval(ctx, ds, th), lib.nll_eval(ctx, dk, th)
        assert abs(a - b) <= 1e-13 * abs(b)
        fa, ga = lib.nll_grad(ctx, ds, th)
        fb, gb = lib.nll_grad(ctx, dk, th)
        assert np.allclose(ga, gb, rtol=1e-10, atol=1e-10 * np.abs(gb).max())
    finally:
        lib.ipx_dataset_destroy(ctx, ds)
        lib.ipx_dataset_destroy(ctx, dk)


def test_timing_counters(lib, ctx):
    cols, w = small_data(3, n=20000)
    ds = lib.ipx_dataset_create(ctx, 3, cols, w)
    try:
        say("timing")
        lib.ipx_timing_read(ctx, reset=True)
        lib.ipx_timing_enable(ctx, True)
        for _ in range(5):
            lib.nll_grad(ctx, ds, M.THETA_GEN[3])
        ms, n = lib.ipx_timing_read(ctx, reset=True)
        lib.ipx_timing_enable(ctx, False)
        assert n == 5 and ms > 0.0
    finally:
        lib.ipx_dataset_destroy(ctx, ds)


# ---------------------------------------------------------------------------
# Full workload sizes, in the launch configuration the benchmark times
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("model", MODELS)
def test_full_size_nll_matches_oracle(lib, ctx, model):
    n = W.WORKLOAD_SIZES[model]
    cols, w = W.events(model, n)
    ds = lib.ipx_dataset_create(ctx, model, cols, w)
    try:
        th = thetas(model, 2)[1]
        say("full-size nll model", model, "n", n)
        got = lib.nll_eval(ctx, ds, th)
        f, g = lib.nll_grad(ctx, ds, th)
        assert got == f
        check_nll(got, N.nll(model, cols, th, w))
        # gradient at full size: central differences of the (pinned) NLL
        for j in range(len(th)):
            h = 1e-5 * max(1.0, abs(th[j]))
            tp, tm = th.copy(), th.copy()
            tp[j] += h
            tm[j] -= h
            fd = (lib.nll_eval(ctx, ds, tp) - lib.nll_eval(ctx, ds, tm)) / (2 * h)
            # truncation O(h^2 f''') and rounding 1e-16 |NLL| / h
            tol = 1e-5 * abs(g[j]) + 1e-14 * abs(f) / h + 1e-6 * math.sqrt(n)
            assert abs(g[j] - fd) <= tol, (j, g[j], fd)
    finally:
        lib.ipx_dataset_destroy(ctx, ds)


def test_full_size_gradient_on_subsample(lib, ctx):
    """The full angular workload's gradient equals the sum of the gradients of
    a partition of its events; one part is checked against the oracle."""
    n = W.WORKLOAD_SIZES[3]
    cols, w = W.events(3, n)
    th = thetas(3, 2)[1]
    ds = lib.ipx_dataset_create(ctx, 3, cols, w)
    cut = 60_000
    da = lib.ipx_dataset_create(ctx, 3, [c[:cut] for c in cols], w[:cut])
    db = lib.ipx_dataset_create(ctx, 3, [c[cut:] for c in cols], w[cut:])
    try:
        say("full-size gradient partition")
        f, g = lib.nll_grad(ctx, ds, th)
        fa, ga = lib.nll_grad(ctx, da, th)
        fb, gb = lib.nll_grad(ctx, db, th)
        assert abs(f - (fa + fb)) <= 1e-12 * abs(f)
        assert np.allclose(g, ga + gb, rtol=1e-9, atol=1e-9 * np.abs(g).max())
        fref, gref = N.nll_grad(3, [c[:cut] for c in cols], th, w[:cut])
        check_nll(fa, fref)
        check_grad(3, [c[:cut] for c in cols], w[:cut], th, ga, gref)
    finally:
        for d in (ds, da, db):
            lib.ipx_dataset_destroy(ctx, d)


def test_torch_autograd_mirror(lib, ctx):
    import torch
    cols, w = small_data(3, n=3000, seed=21)
    ds = lib.ipx_dataset_create(ctx, 3, cols, w)
    try:
        say("torch autograd mirror")
        th = thetas(3, 2)[1]
        f, g = lib.nll_grad(ctx, ds, th)
        t = torch.tensor(th, dtype=torch.float64, requires_grad=True)
        out = lib.nll(ctx, ds, t)
        assert out.item() == f
        (2.5 * out).backward()
        assert np.array_equal(t.grad.numpy(), 2.5 * g)
    finally:
        lib.ipx_dataset_destroy(ctx, ds)


@pytest.mark.parametrize("model", [2, 3])
def test_resolution_extremes_match_oracle(lib, ctx, model):
    # sigma_t log-uniform over [0.002, 0.5] ps: corrections skipped, every
    # continued-fraction depth, the full depth, the rational-series branch
    # (Im u < 3.4) and, for the complex rate, |u| >= 6 with E < 0
    cols, w = small_data(model, n=20000, seed=31)
    scol = 2 if model == 2 else 4
    rng = np.random.default_rng(32)
    cols = [c.copy() for c in cols]
    cols[scol] = np.exp(rng.uniform(np.log(0.002), np.log(0.5), cols[0].shape[0]))
    ds = lib.ipx_dataset_create(ctx, model, cols, w)
    try:
        for i, th in enumerate(thetas(model, 2)):
            say("resolution extremes model", model, "theta", i)
            f, g = lib.nll_grad(ctx, ds, th)
            fref, gref = N.nll_grad(model, cols, th, w)
            check_nll(f, fref)
            check_nll(lib.nll_eval(ctx, ds, th), fref)
            check_grad(model, cols, w, th, g, gref)
    finally:
        lib.ipx_dataset_destroy(ctx, ds)
