"""GPU parity of the binned path (Examples 3-5, binned side) against the oracle
(oracle/binned.py):

  * smearing and the signal template: element by element, |got - ref| <=
    1e-12 max|ref| (sums of up to 2 x 10^4 products in another order);
  * binned NLL (relative 1e-12) and gradient (1e-9 relative, or the size of
    the terms it cancels from);
  * toy counts: bit-exact, per bin, for several toys of both hypotheses (an
    integer decided in FP64 on both sides; a difference is allowed only
    where u is within 1e-12 of a CDF step, and there must be none here);
  * q of every toy (relative 1e-11) and the CL counts: equal, except for
    toys whose q is within 1e-10 of q_obs (none expected), at the workload
    of 10^4 bins with 10^4 toys per hypothesis;
  * binned fits (the lockstep BFGS on nll_binned) of toys generated at a
    known point: convergence, pulls, and stationarity of the oracle's
    likelihood at the fitted point.
"""
import math
import sys

import numpy as np
import pytest

from oracle import binned as B

pytestmark = pytest.mark.gpu

LO, HI = 5179.0, 5379.0
MU, SCORE, SSMEAR = 5279.0, 3.0, 2.0


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


@pytest.mark.parametrize("n,sigma", [(1, 0.5), (255, 1.0), (3001, 2.0), (10000, 0.7)])
def test_smear_matches_oracle(lib, ctx, n, sigma):
    import torch
    rng = np.random.default_rng(n)
    h = rng.uniform(0.0, 1.0, n) * (rng.uniform(size=n) < 0.3)
    dx = (HI - LO) / n
    say("smear n", n)
    got = lib.ipx_smear(ctx, torch.from_numpy(h).to("cuda"), dx, sigma).cpu().numpy()
    ref = B.gauss_smear(h, dx, sigma)
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(np.max(np.abs(ref)), 1e-300)


def _oracle_template(n):
    x, dx = B.bin_centres(LO, HI, n)
    return x, dx, B.signal_template(x, dx, MU, SCORE, SSMEAR)


@pytest.mark.parametrize("n", [100, 2048, 10000])
def test_template_and_nll_match_oracle(lib, ctx, n):
    x, dx, sig = _oracle_template(n)
    th0 = (70.0, 50_000.0 * n / 10000, 0.004)
    counts = B.toy_counts(17, 1, 0, B.expected(sig, th0[0], th0[1], th0[2], x)).astype(float)
    H = lib.ipx_hist_create(ctx, n, LO, HI, MU, SCORE, SSMEAR, counts)
    try:
        got = lib.ipx_hist_read(ctx, H, 0)
        assert np.max(np.abs(got - sig)) <= 1e-12 * sig.max()
        assert np.array_equal(lib.ipx_hist_read(ctx, H, 1), counts)
        for th in (th0, (90.0, th0[1] * 1.02, 0.0), (10.0, th0[1] * 0.9, -0.003)):
            say("binned nll n", n, "theta", th)
            f, g = lib.nll_binned(ctx, H, th, grad=True)
            fr, gr = B.nll_grad(counts, sig, x, th)
            assert abs(f - fr) <= 1e-12 * abs(fr), (f, fr)
            # the sums the gradient cancels from
            nu = B.expected(sig, th[0], th[1], th[2], x)
            r = np.abs(1.0 - counts / nu)
            scale = np.array([np.sum(r * sig), np.sum(r), np.sum(r) * th[1] * (HI - LO)])
            assert np.all(np.abs(g - gr) <= 1e-9 * np.abs(gr) + 1e-12 * scale), (g, gr)
            assert lib.nll_binned(ctx, H, th) == f
        assert lib.nll_binned(ctx, H, (-1.0, 10.0, 0.0)) == math.inf
    finally:
        lib.ipx_hist_destroy(ctx, H)


def test_toy_counts_bit_exact(lib, ctx):
    n = 2000
    x, dx, sig = _oracle_template(n)
    H = lib.ipx_hist_create(ctx, n, LO, HI, MU, SCORE, SSMEAR)
    try:
        for th in ((70.0, 10_000.0, 0.004), (400.0, 300.0, -0.002), (5.0, 2e5, 0.0)):
            for hyp in (0, 1):
                nu = th[1] * B.background_template(x, th[2]) + (th[0] * sig if hyp else 0.0)
                for toy in (0, 1, 12345):
                    say("binned toy", th, "hyp", hyp, "toy", toy)
                    got = lib.ipx_binned_toy(ctx, H, th, 99, hyp, toy)
                    ref = B.toy_counts(99, hyp, toy, nu)
                    assert np.array_equal(got, ref), np.flatnonzero(got != ref)[:10]
        # the inversion needs e^{-nu} > 0: expected counts of 700 or more are refused
        with pytest.raises(lib.IpxError) as e:
            lib.ipx_binned_toy(ctx, H, (5.0, 2e6, 0.0), 99, 0, 0)
        assert e.value.status == lib.IPX_EDOMAIN
    finally:
        lib.ipx_hist_destroy(ctx, H)


def test_cls_matches_oracle_at_the_workload(lib, ctx):
    """10^4 bins, 10^4 toys per hypothesis: q of every toy and the CL
    counts; the oracle evaluates every toy (CPU, a few minutes) only at
    2 x 200 toys and is compared element-wise there; at 10^4 toys the GPU's
    background-only and signal+background q are checked against the oracle's
    on a sample of 50 toys each."""
    n, ntoys, seed = 10_000, 10_000, 2024
    x, dx, sig = _oracle_template(n)
    ns, nb, k = 70.0, 50_000.0, 0.004
    obs = B.toy_counts(7, B.HYP_B, 0, nb * B.background_template(x, k)).astype(float)
    H = lib.ipx_hist_create(ctx, n, LO, HI, MU, SCORE, SSMEAR, obs)
    try:
        say("cls 200 toys")
        small = lib.cls_toys(ctx, H, (ns, nb, k), seed, 200, want_q=True)
        cl_sb, cl_b, cl_s, q_obs, qb, qsb = B.cls(obs, sig, x, ns, nb, k, seed, 200)
        assert abs(small["q_obs"] - q_obs) <= 1e-11 * max(1.0, abs(q_obs))
        assert np.all(np.abs(small["q_b"] - qb) <= 1e-11 * np.maximum(1.0, np.abs(qb)))
        assert np.all(np.abs(small["q_sb"] - qsb) <= 1e-11 * np.maximum(1.0, np.abs(qsb)))
        near = lambda q: np.abs(q - q_obs) <= 1e-10 * max(1.0, abs(q_obs))  # noqa: E731
        assert not near(qb).any() and not near(qsb).any()
        assert small["n_b"] == int(np.sum(qb >= q_obs)) and small["n_sb"] == int(np.sum(qsb >= q_obs))
        say("cls 10^4 toys")
        big = lib.cls_toys(ctx, H, (ns, nb, k), seed, ntoys, want_q=True)
        # the first 200 toys of the large run are the small run's
        assert np.array_equal(big["q_b"][:200], small["q_b"]) and np.array_equal(big["q_sb"][:200], small["q_sb"])
        rng = np.random.default_rng(5)
        s = ns * sig
        b = nb * B.background_template(x, k)
        for t in rng.choice(np.arange(200, ntoys), 50, replace=False):
            for hyp, qv, nu in ((B.HYP_B, big["q_b"], b), (B.HYP_SB, big["q_sb"], s + b)):
                qr = B.q_statistic(B.toy_counts(seed, hyp, int(t), nu), s, b)
                assert abs(qv[t] - qr) <= 1e-11 * max(1.0, abs(qr)), (t, hyp)
        assert big["n_b"] == int(np.sum(big["q_b"] >= big["q_obs"]))
        assert big["n_sb"] == int(np.sum(big["q_sb"] >= big["q_obs"]))
        assert big["cl_s"] == pytest.approx(big["cl_sb"] / big["cl_b"])
        say("CL_b %.4f CL_s+b %.4f CL_s %.4f" % (big["cl_b"], big["cl_sb"], big["cl_s"]))
    finally:
        lib.ipx_hist_destroy(ctx, H)


def test_binned_fits_recover_the_generation_point(lib, ctx):
    """The binned fit of Examples 3-4: 20 signal + background toys of 10^3
    bins generated at theta_gen (ipx_binned_toy), each fitted with the
    lockstep BFGS on nll_binned and its gradient, errors from the inverse
    finite-difference Hessian; every fit converges to a stationary point and
    the pulls of the three parameters have mean within 4/sqrt(k) of 0 and
    width within 4/sqrt(2k) of 1."""
    from paper_1706_01420_amd import fit
    n, ntoys = 1000, 20
    th0 = np.array([400.0, 20_000.0, 0.004])
    H = lib.ipx_hist_create(ctx, n, LO, HI, MU, SCORE, SSMEAR)
    hs = []
    try:
        say("binned fits", ntoys)
        for j in range(ntoys):
            c = lib.ipx_binned_toy(ctx, H, th0, 77, 1, j)
            hs.append(lib.ipx_hist_create(ctx, n, LO, HI, MU, SCORE, SSMEAR, c))

        def evaluate(theta, active):
            f = np.full(theta.shape[0], np.inf)
            g = np.full(theta.shape, np.nan)
            for j in np.flatnonzero(active):
                f[j], g[j] = lib.nll_binned(ctx, hs[j], theta[j], grad=True)
            return f, g
        steps = np.array([30.0, 150.0, 2e-4])
        start = np.tile(th0 + 2.0 * steps * np.array([1.0, -1.0, 1.0]), (ntoys, 1))
        res = fit.bfgs(evaluate, start, steps)
        assert res["converged"].all(), res["converged"]
        err = fit.errors(evaluate, res["theta"], steps)
        pulls = (res["theta"] - th0) / err
        assert np.all(np.isfinite(pulls))
        k = ntoys
        assert np.all(np.abs(pulls.mean(axis=0)) < 4.0 / np.sqrt(k)), pulls.mean(axis=0)
        assert np.all(np.abs(pulls.std(axis=0, ddof=1) - 1.0) < 4.0 / np.sqrt(2 * k)), pulls.std(axis=0, ddof=1)
        for j in range(ntoys):       # a stationary point of the oracle's likelihood too
            x, dx, sig = _oracle_template(n)
            counts = lib.ipx_hist_read(ctx, hs[j], 1)
            _, gr = B.nll_grad(counts, sig, x, res["theta"][j])
            assert np.all(np.abs(gr) * steps < 1e-2), (j, gr)
    finally:
        for h in hs:
            lib.ipx_hist_destroy(ctx, h)
        lib.ipx_hist_destroy(ctx, H)
