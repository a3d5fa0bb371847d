"""Pins of the oracle's binned path (paper Examples 3-5, binned side):

  * smearing: a Gaussian smeared by a Gaussian is the Gaussian of the summed
    variances (closed form) at the bin centres; a single bin smears into the
    kernel itself; the total is kept away from the range ends;
  * Poisson inversion: the inverse CDF equals scipy's Poisson quantile away
    from exact ties; a million draws follow the Poisson pmf (chi-squared);
  * likelihood: the NLL equals minus scipy's summed Poisson log-pmf up to the
    constant sum ln n_b!; its gradient matches central differences;
  * q: equals -2 ln [L(s+b)/L(b)] from scipy's log-pmf; CL_b at the median
    background-only q is about one half; toy counts have the expected means.
"""
import math

import numpy as np
import pytest
from scipy import stats
from scipy.special import gammaln

from oracle import binned as B

LO, HI, NB = 5179.0, 5379.0, 2000


def test_smear_gaussian_by_gaussian_is_the_closed_form():
    x, dx = B.bin_centres(LO, HI, NB)
    for s1, s2 in ((3.0, 2.0), (6.0, 4.5), (1.2, 0.5)):
        h = np.exp(-(x - 5280.0) ** 2 / (2 * s1 * s1)) / (math.sqrt(2 * math.pi) * s1) * dx
        got = B.gauss_smear(h, dx, s2)
        st = math.hypot(s1, s2)
        ref = np.exp(-(x - 5280.0) ** 2 / (2 * st * st)) / (math.sqrt(2 * math.pi) * st) * dx
        assert np.max(np.abs(got - ref)) <= 1e-12 * ref.max(), (s1, s2)


def test_smear_delta_is_the_kernel_and_keeps_the_total():
    x, dx = B.bin_centres(LO, HI, NB)
    h = np.zeros(NB)
    h[777] = 1.0
    got = B.gauss_smear(h, dx, 2.5)
    d = (np.arange(NB) - 777) * dx       # the centre differences, without the rounding of x
    ref = np.exp(-d ** 2 / (2 * 2.5 ** 2)) / (math.sqrt(2 * math.pi) * 2.5) * dx
    assert np.max(np.abs(got - ref)) <= 1e-15 * ref.max()
    assert abs(got.sum() - 1.0) < 1e-13


@pytest.mark.parametrize("nu", [0.02, 0.7, 3.0, 11.5, 60.0, 400.0])
def test_poisson_inverse_is_the_quantile(nu):
    rng = np.random.default_rng(int(nu * 100))
    u = rng.uniform(size=4000)
    em = math.exp(-nu)
    got = np.array([B.poisson_inverse(float(v), nu, em) for v in u])
    ref = stats.poisson.ppf(u, nu).astype(int)
    diff = got != ref
    if diff.any():
        # only where u sits on a CDF step to within rounding
        F = stats.poisson.cdf(np.minimum(got, ref), nu)
        assert np.all(np.abs(u[diff] - F[diff]) < 1e-12), (u[diff], got[diff], ref[diff])
    assert diff.sum() <= 2


@pytest.mark.parametrize("nu", [0.3, 5.0, 42.0])
def test_poisson_draws_follow_the_pmf(nu):
    u = B.toy_uniforms(7, 0, 3, 200_000)
    em = math.exp(-nu)
    k = np.array([B.poisson_inverse(float(v), nu, em) for v in u])
    kmax = int(nu + 6 * math.sqrt(nu) + 6)
    obs = np.bincount(np.minimum(k, kmax), minlength=kmax + 1)
    p = stats.poisson.pmf(np.arange(kmax + 1), nu)
    p[-1] = stats.poisson.sf(kmax - 1, nu)
    exp = p * k.size
    keep = exp > 5
    chi2 = np.sum((obs[keep] - exp[keep]) ** 2 / exp[keep])
    assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-4, chi2
    assert abs(k.mean() - nu) < 5 * math.sqrt(nu / k.size)


def _setup(ns=70.0, nb=50_000.0, k=0.004, nbins=NB):
    x, dx = B.bin_centres(LO, HI, nbins)
    sig = B.signal_template(x, dx, 5279.0, 3.0, 2.0)
    return x, dx, sig, ns, nb, k


def test_nll_is_the_poisson_log_likelihood():
    x, dx, sig, ns, nb, k = _setup()
    nu = B.expected(sig, ns, nb, k, x)
    counts = B.toy_counts(11, 1, 0, nu)
    f = B.nll(counts, sig, x, (ns, nb, k))
    ref = -np.sum(stats.poisson.logpmf(counts, nu)) - np.sum(gammaln(counts + 1.0))
    assert abs(f - ref) <= 1e-12 * abs(ref)


def test_nll_gradient_matches_central_differences():
    x, dx, sig, ns, nb, k = _setup(nbins=400)
    nu = B.expected(sig, ns, nb, k, x)
    counts = B.toy_counts(5, 1, 2, nu)
    th = np.array([ns * 1.1, nb * 0.97, k * 1.2])
    f, g = B.nll_grad(counts, sig, x, th)
    for i in range(3):
        h = 1e-5 * max(1e-3, abs(th[i]))
        v = []
        for s in (-2, -1, 1, 2):
            t = th.copy()
            t[i] += s * h
            v.append(B.nll(counts, sig, x, t))
        fd = (v[0] - 8 * v[1] + 8 * v[2] - v[3]) / (12 * h)
        assert abs(g[i] - fd) <= 1e-6 * max(1.0, abs(fd)), (i, g[i], fd)


def test_q_is_minus_two_log_likelihood_ratio():
    x, dx, sig, ns, nb, k = _setup()
    s, b = ns * sig, nb * B.background_template(x, k)
    for toy in range(3):
        n = B.toy_counts(3, toy % 2, toy, s + b)
        q = B.q_statistic(n, s, b)
        ref = -2.0 * (np.sum(stats.poisson.logpmf(n, s + b)) - np.sum(stats.poisson.logpmf(n, b)))
        assert abs(q - ref) <= 1e-9 * max(1.0, abs(ref))


def test_cls_medians_and_toy_means():
    x, dx, sig, ns, nb, k = _setup(nbins=300, nb=3000.0, ns=40.0)
    s, b = ns * sig, nb * B.background_template(x, k)
    counts = [B.toy_counts(21, B.HYP_B, t, b) for t in range(400)]
    mean = np.mean(counts, axis=0)
    z = (mean - b) / np.sqrt(b / 400)
    assert abs(z.mean()) < 0.2 and abs(z.std() - 1.0) < 0.15
    cl_sb, cl_b, cl_s, q_obs, qb, qsb = B.cls(B.toy_counts(99, B.HYP_B, 0, b), sig, x, ns, nb, k, 21, 400)
    # data drawn from the background: signal-like toys rarely look as background-like
    assert qsb.mean() < qb.mean() and 0.0 <= cl_s <= 1.0
    med = float(np.median(qb))
    frac = np.mean(qb >= med)
    assert 0.45 <= frac <= 0.56


# -- planted mistakes (each must fail one of the pins above) --------------------
def _smear_no_width(h, width, sigma):
    n = len(h)
    d = np.arange(-(n - 1), n) * width
    kern = np.exp(-d * d / (2.0 * sigma * sigma)) / (math.sqrt(2.0 * math.pi) * sigma)   # dx dropped
    return np.convolve(h, kern)[n - 1:2 * n - 1]


def _smear_shifted(h, width, sigma):
    n = len(h)
    d = np.arange(-(n - 1), n) * width
    kern = np.exp(-d * d / (2.0 * sigma * sigma)) / (math.sqrt(2.0 * math.pi) * sigma) * width
    return np.convolve(h, kern)[n:2 * n]            # off by one bin


def _poisson_off_by_one(u, nu, em):
    k, p, F = 0, em, em
    while u > F and k < B.poisson_kmax(nu):
        k += 1
        p = p * nu / (k + 1)                         # wrong recurrence
        F = F + p
    return k


def _q_no_factor_two(counts, s, b):
    L = np.log1p(s / b)
    return math.fsum(s.tolist()) - math.fsum((np.asarray(counts, np.float64) * L).tolist())


@pytest.mark.parametrize("attr,fake,check", [
    ("gauss_smear", _smear_no_width, test_smear_delta_is_the_kernel_and_keeps_the_total),
    ("gauss_smear", _smear_shifted, test_smear_gaussian_by_gaussian_is_the_closed_form),
    ("poisson_inverse", _poisson_off_by_one, lambda: test_poisson_inverse_is_the_quantile(3.0)),
    ("q_statistic", _q_no_factor_two, test_q_is_minus_two_log_likelihood_ratio),
], ids=["smear without the bin width", "smear off by one bin", "Poisson recurrence", "q without the 2"])
def test_planted_binned_mistake_is_caught(attr, fake, check, monkeypatch):
    monkeypatch.setattr(B, attr, fake)
    with pytest.raises(AssertionError):
        check()


def test_array_inversion_is_the_scalar_one():
    rng = np.random.default_rng(4)
    nu = rng.uniform(0.0, 80.0, 3000)
    u = rng.uniform(size=3000)
    got = B.poisson_inverse_array(u, nu, np.exp(-nu))
    ref = [B.poisson_inverse(float(a), float(b), float(np.exp(-b))) for a, b in zip(u, nu)]
    assert np.array_equal(got, ref)
