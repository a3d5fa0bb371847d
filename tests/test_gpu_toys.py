"""GPU toy generation (toy_generate) against the oracle generator.

Bitwise: the candidate sequence (which candidates are accepted, hence
n_candidates and every column computed from uniforms with +, -, x only:
m of the mass model, sigma_t, the angles, the weights).  The columns that go
through log / sqrt / sin / cos (decay times, Box-Muller masses) are compared at
relative 1e-13: both sides use correctly rounded-to-1-ulp library functions.
The oracle also reports the smallest relative gap |u M - R| / R over all
candidates examined; the decisions can only differ if that gap is below the
last-bit differences of the two sides' transcendental functions (1e-15), so
the test asserts the gap exceeds 1e-12 on these seeds.
"""
import sys

import numpy as np
import pytest

from storage_order import band_order

from oracle import generate as G
from oracle import models as M

pytestmark = pytest.mark.gpu

EXACT_COLS = {1: [0], 2: [2], 3: [0, 1, 2, 4]}


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


def _read_all(lib, ctx, ds, model):
    cols = [lib.ipx_dataset_read(ctx, ds, c) for c in range(M.NCOLS[model])]
    w = lib.ipx_dataset_read(ctx, ds, M.NCOLS[model]) if model == 3 else None
    return cols, w


@pytest.mark.parametrize("model", [1, 2, 3])
@pytest.mark.parametrize("n,toy", [(20000, 3), (1, 0), (4099, 77)])
def test_toy_generate_matches_oracle(lib, ctx, model, n, toy):
    seed = 170601420 + model
    theta = M.THETA_GEN[model]
    ref = G.generate(model, theta, seed, toy, n)
    assert ref["violations"] == 0
    assert ref["min_margin"] > 1e-12
    say("toy_generate model", model, "n", n, "toy", toy)
    ds, st = lib.toy_generate(ctx, model, theta, seed, toy, n, flags=lib.IPX_KEEP_ORDER)
    try:
        assert st["n_violations"] == 0
        assert st["n_candidates"] == ref["n_candidates"]
        cols, w = _read_all(lib, ctx, ds, model)
        for c in range(M.NCOLS[model]):
            if c in EXACT_COLS[model]:
                assert np.array_equal(cols[c], ref["cols"][c]), c
            else:
                assert np.allclose(cols[c], ref["cols"][c], rtol=1e-13, atol=0), c
        if model == 3:
            assert np.array_equal(w, ref["w"])
    finally:
        lib.ipx_dataset_destroy(ctx, ds)


@pytest.mark.parametrize("model", [2, 3])
def test_toy_generate_sorted_output_is_the_same_sample(lib, ctx, model):
    seed, toy, n = 99, 5, 30000
    theta = M.THETA_GEN[model]
    say("toy_generate sorted model", model)
    a, _ = lib.toy_generate(ctx, model, theta, seed, toy, n, flags=lib.IPX_KEEP_ORDER)
    b, _ = lib.toy_generate(ctx, model, theta, seed, toy, n)
    try:
        ca, wa = _read_all(lib, ctx, a, model)
        cb, wb = _read_all(lib, ctx, b, model)
        tcol, scol = (1, 2) if model == 2 else (3, 4)
        order = band_order(ca[tcol], ca[scol])
        for c in range(M.NCOLS[model]):
            assert np.array_equal(cb[c], ca[c][order])
        # the NLL of both layouts agrees to rounding
        th = np.array(theta)
        fa, fb = lib.nll_eval(ctx, a, th), lib.nll_eval(ctx, b, th)
        assert abs(fa - fb) <= 1e-12 * abs(fa)
    finally:
        lib.ipx_dataset_destroy(ctx, a)
        lib.ipx_dataset_destroy(ctx, b)


def test_toy_generate_errors(lib, ctx):
    say("toy_generate errors")
    with pytest.raises(lib.IpxError):
        lib.toy_generate(ctx, 4, (0.3,), 1, 0, 10)
    with pytest.raises(lib.IpxError):
        lib.toy_generate(ctx, 1, (1.3, 5367.0, 15.0, 0.002), 1, 0, 10)
    ds, st = lib.toy_generate(ctx, 1, M.THETA_GEN[1], 1, 0, 0)
    try:
        assert lib.ipx_dataset_size(ds) == 0 and st["n_candidates"] == 0
    finally:
        lib.ipx_dataset_destroy(ctx, ds)


@pytest.mark.parametrize("model", [1, 2, 3])
def test_toy_generate_batch_equals_single_toys(lib, ctx, model):
    seed = 77
    theta = M.THETA_GEN[model]
    ids = [3, 0, 11, 5, 9]
    sizes = [5000, 0, 1, 12345, 777]
    for flags in (lib.IPX_KEEP_ORDER, 0):
        say("toy_generate_batch model", model, "flags", flags)
        batch, bstats = lib.toy_generate_batch(ctx, model, theta, seed, ids, sizes, flags)
        try:
            for j, (tid, n) in enumerate(zip(ids, sizes)):
                d, st = lib.toy_generate(ctx, model, theta, seed, tid, n, flags)
                try:
                    assert lib.ipx_dataset_size(batch[j]) == n
                    assert bstats[j]["n_candidates"] == st["n_candidates"]
                    assert bstats[j]["n_violations"] == 0 and st["n_violations"] == 0
                    if n:
                        a, wa = _read_all(lib, ctx, batch[j], model)
                        b, wb = _read_all(lib, ctx, d, model)
                        for c in range(M.NCOLS[model]):
                            assert np.array_equal(a[c], b[c])
                        assert (wa is None and wb is None) or np.array_equal(wa, wb)
                finally:
                    lib.ipx_dataset_destroy(ctx, d)
        finally:
            for d in batch:
                lib.ipx_dataset_destroy(ctx, d)


def test_toy_generate_batch_errors(lib, ctx):
    say("toy_generate_batch errors")
    th = M.THETA_GEN[1]
    with pytest.raises(lib.IpxError):
        lib.toy_generate_batch(ctx, 1, th, 1, [0, 1], [10, -1])
    with pytest.raises(lib.IpxError):
        lib.toy_generate_batch(ctx, 4, th, 1, [0], [10])
    ds, st = lib.toy_generate_batch(ctx, 1, th, 1, [], [])
    assert ds == [] and st == []
