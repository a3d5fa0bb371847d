"""Binned path: histogram templates, Gaussian smearing of a binned shape, the
binned Poisson likelihood, binned Poisson toys and the CL_s construction
(oracle test infrastructure).

Paper (Ipanema-beta, arXiv:1706.01420) passages followed:
  * Example 3: binned maximum-likelihood fit of a mass spectrum (the data set
    as counts per bin, the model as expected counts per bin);
  * Example 4 (CL_s): a signal shape filled per bin and convolved with a
    Gaussian, an exponential background per bin, both normalised to unit sum,
    expected counts ns * signal + nb * background, pseudo-data drawn per bin,
    CL_b, CL_s+b and CL_s from 10^4 toys per hypothesis;
  * Example 5: binned toys (a Poisson count per bin).
Readings where the paper gives no formula (listed in the design notes):
  * smearing: S_b = sum_j h_j g(x_b - x_j) dx with g the unit Gaussian density
    of width sigma and x the bin centres (the rectangle rule of the
    convolution integral, no wrap-around at the range ends);
  * the signal template before smearing is a Gaussian core of mean mu and
    width sigma_core at the bin centres (the paper's Ipatia shape is the next
    step); the background is exp(-k x) at the bin centres;
  * likelihood: NLL = sum_b [nu_b - n_b ln nu_b] (the constant sum ln n_b!
    dropped), parameters (ns, nb, k);
  * test statistic q = -2 ln [L(s+b) / L(b)] = 2 sum_b [s_b - n_b ln(1 + s_b/b_b)],
    CL_x = fraction of the hypothesis-x toys with q >= q_obs, CL_s = CL_s+b / CL_b;
  * toys: n_b = the smallest k with u <= F(k) (inversion of the Poisson CDF
    summed from k = 0: p_0 = e^{-nu}, p_k = p_{k-1} nu / k, F(k) = F(k-1) + p_k,
    evaluated in that order), u from Philox4x64-10 with key (seed, 0xB1),
    counter (b >> 2, toy, hypothesis, 0), word b & 3; the search stops at
    k_max = floor(nu + 30 sqrt(nu + 1) + 30) (probability beyond: < 1e-100).
"""
import math

import numpy as np

from . import philox as P

BINNED_KEY = 0xB1
HYP_B, HYP_SB = 0, 1


def bin_centres(lo, hi, nbins):
    width = (hi - lo) / nbins
    return lo + (np.arange(nbins) + 0.5) * width, width


def gauss_smear(h, width, sigma):
    """S_b = sum_j h_j g(x_b - x_j) width, g the unit Gaussian density."""
    h = np.asarray(h, dtype=np.float64)
    n = h.size
    d = np.arange(-(n - 1), n) * width
    kern = np.exp(-d * d / (2.0 * sigma * sigma)) / (math.sqrt(2.0 * math.pi) * sigma) * width
    return np.convolve(h, kern)[n - 1:2 * n - 1]


def signal_template(x, width, mu, sigma_core, sigma_smear):
    """Gaussian core at the bin centres, smeared, normalised to unit sum."""
    core = np.exp(-(x - mu) ** 2 / (2.0 * sigma_core * sigma_core))
    s = gauss_smear(core, width, sigma_smear)
    return s / math.fsum(s.tolist())


def background_template(x, k):
    """exp(-k x) at the bin centres, normalised to unit sum (x shifted to the
    first centre for conditioning: the shift cancels in the normalisation)."""
    e = np.exp(-k * (x - x[0]))
    return e / math.fsum(e.tolist())


def expected(sig, ns, nb, k, x):
    return ns * sig + nb * background_template(x, k)


def nll(counts, sig, x, theta):
    """sum_b [nu_b - n_b ln nu_b] at theta = (ns, nb, k); +inf if any nu_b <= 0
    where n_b > 0."""
    ns, nb, k = theta
    nu = expected(sig, ns, nb, k, x)
    n = np.asarray(counts, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = nu - np.where(n > 0, n * np.log(nu), 0.0)
    if not np.all(np.isfinite(t)):
        return math.inf
    return math.fsum(t.tolist())


def nll_grad(counts, sig, x, theta):
    """(NLL, gradient in (ns, nb, k)): dNLL/dnu_b = 1 - n_b/nu_b, with
    dnu_b/dns = s_b, dnu_b/dnb = e_b and dnu_b/dk = nb e_b (<x>_e - x_b),
    e the normalised background template."""
    ns, nb, k = theta
    e = background_template(x, k)
    nu = ns * sig + nb * e
    n = np.asarray(counts, dtype=np.float64)
    f = nll(counts, sig, x, theta)
    if not math.isfinite(f):
        return math.inf, np.full(3, np.nan)
    r = 1.0 - n / nu
    xm = math.fsum((e * x).tolist())
    g = np.array([math.fsum((r * sig).tolist()), math.fsum((r * e).tolist()),
                  math.fsum((r * nb * e * (xm - x)).tolist())])
    return f, g


# ---------------------------------------------------------------------------
# Toys and CL_s
# ---------------------------------------------------------------------------
def toy_uniforms(seed, hyp, toy, nbins):
    """u[b] for bins 0 .. nbins-1 of one toy of hypothesis hyp."""
    nblk = (nbins + 3) // 4
    ctr = np.stack([np.arange(nblk, dtype=np.uint64), np.full(nblk, toy, np.uint64),
                    np.full(nblk, hyp, np.uint64), np.zeros(nblk, np.uint64)], axis=1)
    key = np.array([seed, BINNED_KEY], dtype=np.uint64)
    return P.to_uniform(P.philox(ctr, key)).reshape(-1)[:nbins]


def poisson_kmax(nu):
    return math.floor(nu + 30.0 * math.sqrt(nu + 1.0) + 30.0)


def poisson_inverse(u, nu, exp_minus_nu):
    """Smallest k with u <= F(k), F summed from k = 0 in the order stated in
    the module notes; exp_minus_nu = e^{-nu} (computed once per bin)."""
    k = 0
    p = exp_minus_nu
    F = p
    kmax = poisson_kmax(nu)
    while u > F and k < kmax:
        k += 1
        p = p * nu / k
        F = F + p
    return k


def poisson_inverse_array(u, nu, exp_minus_nu):
    """poisson_inverse element by element, the bins stepped together (the same
    operations in the same order on each element)."""
    u = np.asarray(u, np.float64)
    nu = np.asarray(nu, np.float64)
    k = np.zeros(u.size)
    p = np.array(exp_minus_nu, np.float64)
    F = p.copy()
    kmax = np.floor(nu + 30.0 * np.sqrt(nu + 1.0) + 30.0)
    go = (u > F) & (k < kmax)
    while go.any():
        k = np.where(go, k + 1.0, k)
        p = np.where(go, p * nu / np.where(go, k, 1.0), p)
        F = np.where(go, F + p, F)
        go = go & (u > F) & (k < kmax)
    return k.astype(np.int64)


def toy_counts(seed, hyp, toy, nu):
    nu = np.asarray(nu, np.float64)
    u = toy_uniforms(seed, hyp, toy, nu.size)
    return poisson_inverse_array(u, nu, np.exp(-nu))


def q_statistic(counts, s, b):
    """q = 2 sum_b [s_b - n_b ln(1 + s_b / b_b)] (exactly summed)."""
    L = np.log1p(s / b)
    return 2.0 * (math.fsum(s.tolist()) - math.fsum((np.asarray(counts, np.float64) * L).tolist()))


def cls(counts_obs, sig, x, ns, nb, k, seed, ntoys):
    """(CL_s+b, CL_b, CL_s, q_obs, q_b[ntoys], q_sb[ntoys])."""
    s = ns * sig
    b = nb * background_template(x, k)
    q_obs = q_statistic(counts_obs, s, b)
    qs = {}
    for hyp, nu in ((HYP_B, b), (HYP_SB, s + b)):
        qs[hyp] = np.array([q_statistic(toy_counts(seed, hyp, t, nu), s, b) for t in range(ntoys)])
    cl_sb = float(np.mean(qs[HYP_SB] >= q_obs))
    cl_b = float(np.mean(qs[HYP_B] >= q_obs))
    return cl_sb, cl_b, (cl_sb / cl_b if cl_b > 0 else math.nan), q_obs, qs[HYP_B], qs[HYP_SB]
