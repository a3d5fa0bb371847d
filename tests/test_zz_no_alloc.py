"""The allocation-free entry point (nll_eval_noalloc) against the existing one.

nll_eval_noalloc evaluates caller-owned device columns with the library's
fixed device scratch; nll_eval / nll_grad on a dataset that borrows the same
columns (IPX_BORROW_DEVICE, events in the given order) run the same tile
kernels and reduction, so the two must agree bitwise.  Each case makes two
calls in a row, the second on a smaller input (the scratch keeps the first
call's contents), and checks both against the oracle at the parity
tolerances of the other GPU tests.
"""
import math
import sys

import numpy as np
import pytest

from oracle import models as M
from oracle import nll as N
from paper_1706_01420_amd import workloads as W

pytestmark = pytest.mark.gpu

MAX_EVENTS = 1 << 24


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


def device_cols(cols, w):
    import torch
    dc = [torch.from_numpy(np.ascontiguousarray(c)).to("cuda") for c in cols]
    dw = None if w is None else torch.from_numpy(np.ascontiguousarray(w)).to("cuda")
    torch.cuda.synchronize()
    return dc, dw


def check_oracle(model, cols, w, theta, f, g):
    fref = N.nll(model, cols, theta, w) if g is None else None
    if g is None:
        assert math.isfinite(f) and abs(f - fref) <= 1e-10 * abs(fref), (f, fref)
        return
    fref, gref = N.nll_grad(model, cols, theta, w)
    assert abs(f - fref) <= 1e-10 * abs(fref), (f, fref)
    scale = np.abs(N.event_grad(model, cols, theta) * (1.0 if w is None else w)).sum(axis=1)
    bound = 1e-6 * np.abs(gref) + 1e-9 * scale + 1e-13 * cols[0].shape[0]
    assert np.all(np.abs(g - gref) <= bound), (g, gref)


@pytest.mark.parametrize("model", [1, 2, 3, 4])
@pytest.mark.parametrize("grad", [False, True])
def test_noalloc_equals_borrowed_dataset(lib, ctx, model, grad):
    theta = np.array(M.THETA_GEN[model]) * (1.0 + 0.01 * np.arange(1, len(M.THETA_GEN[model]) + 1) / 12.0)
    # two calls in a row, the second smaller (several tiles and a ragged tail,
    # then fewer tiles than the first call left in the scratch)
    for n, seed in ((9 * 1024 + 333, 31), (2 * 1024 + 45, 32)):
        cols, w = W.events(model, n, seed=seed)
        if model not in (3, 4):
            w = None if seed == 31 else w
        dc, dw = device_cols(cols, w)
        say("nll_eval_noalloc model", model, "grad", grad, "n", n)
        got = lib.nll_eval_noalloc(ctx, model, dc, dw, theta, grad=grad)
        ds = lib.ipx_dataset_create(ctx, model, dc, dw, flags=lib.IPX_BORROW_DEVICE)
        try:
            ref = lib.nll_grad(ctx, ds, theta) if grad else lib.nll_eval(ctx, ds, theta)
        finally:
            lib.ipx_dataset_destroy(ctx, ds)
        if grad:
            assert got[0] == ref[0] and np.array_equal(got[1], ref[1]), (got, ref)
            check_oracle(model, cols, w, theta, got[0], got[1])
        else:
            assert got == ref, (got, ref)
            check_oracle(model, cols, w, theta, got, None)


def test_noalloc_empty_and_limits(lib, ctx):
    import torch
    theta = np.array(M.THETA_GEN[1])
    empty = [torch.empty(0, dtype=torch.float64, device="cuda")]
    say("nll_eval_noalloc empty")
    assert lib.nll_eval_noalloc(ctx, 1, empty, None, theta) == 0.0
    # beyond the fixed scratch: rejected before anything runs (the columns are
    # only checked for length on the host, so a 2^24 + 1 event view of a
    # small buffer is never read)
    big = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.IpxError) as e:
        lib._check(lib._lib.nll_eval_noalloc(ctx, 1, MAX_EVENTS + 1,
                                             (lib.ctypes.c_void_p * 1)(big.data_ptr()), 1, None,
                                             lib._buffers(theta)[0].th_p, 4, lib._buffers(theta)[0].out_p,
                                             None, None))
    assert e.value.status == lib.IPX_EINVAL and "maximum" in str(e.value)
    # parameters outside the domain: +inf, nothing launched
    cols, _ = W.events(1, 100, seed=3)
    dc, _ = device_cols(cols, None)
    bad = theta.copy()
    bad[2] = -1.0
    assert lib.nll_eval_noalloc(ctx, 1, dc, None, bad) == float("inf")
