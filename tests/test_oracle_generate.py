"""Pins of the oracle's toy generator (accept-reject from the Philox stream).

The device generator is compared with ``oracle.generate`` bit for bit, so a
recipe mistake made on both sides would pass that comparison; these CPU tests
pin the oracle generator itself against what the PDFs fix (the paper's
Example 5: accept-reject generation whose samples follow the fitted PDF):

  * binned marginals and joint distributions of ~2e5 generated events per
    model against the oracle PDF integrated over each bin by Gauss-Legendre
    quadrature (Pearson chi-squared, fixed seeds);
  * zero bound violations (acceptance ratio above the envelope) over a grid
    of parameter points that includes DeltaGamma < 0, lambda < 0, lambda = 0,
    Fs = 0 and a resolution scale s != 1;
  * planted mistakes in the sampling recipes (each must fail one of the
    above).

What the distributions are, derived from the recipes:
  model 1  m ~ P1(m).
  model 2  sigma_t uniform on [0.03, 0.06] and, given sigma_t, (m, t) ~ P2:
           every component is accepted with probability 1/M2 at every
           sigma_t, so neither the sigma_t density nor the fractions change.
  model 3  (Omega, t_true) ~ the unconvolved density, then t is smeared and
           kept in [0.3, 15]: the kept (Omega, t, sigma_t) have density
           proportional to sum_k f_k sum_j C_kj T_j(t | sigma_t) with sigma_t
           proposed uniformly, i.e. sigma_t ~ den(sigma_t) = sum_j D_j I_j and
           (Omega, t) | sigma_t ~ P3; m is an independent truncated Gaussian
           and w uniform on [0.8, 1].

A rotation of the Box-Muller angle (e.g. off by pi) maps two independent unit
Gaussians to two independent unit Gaussians: the sample's distribution does
not change, so no distribution pin can (or needs to) see it; the exact recipe
is fixed by the bit-exact comparison with the device generator.
"""
import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss
from scipy import stats

from oracle import generate as G
from oracle import models as M

N_EVENTS = 200_000
SEED = 20170605
P_MIN = 1e-3          # unmodified oracle, fixed seeds (deterministic)
P_FAIL = 1e-8         # a planted mistake must push some pin below this


# ---------------------------------------------------------------------------
# Helpers
# ---------------------------------------------------------------------------
def gl_bins(edges, order):
    """Nodes and weights of an order-point Gauss-Legendre rule on every bin;
    returns (nodes, weights, bin index of each node)."""
    x, w = leggauss(order)
    xs, ws, ids = [], [], []
    for b, (lo, hi) in enumerate(zip(edges[:-1], edges[1:])):
        xs.append(0.5 * (hi - lo) * x + 0.5 * (hi + lo))
        ws.append(0.5 * (hi - lo) * w)
        ids.append(np.full(order, b))
    return np.concatenate(xs), np.concatenate(ws), np.concatenate(ids)


def angle_bins(cos_edges, order):
    """Bins in cos(theta) integrated over theta (smooth integrand; the
    Jacobian sin(theta) folded into the weights): nodes are cos values."""
    th_edges = np.arccos(np.clip(cos_edges, -1.0, 1.0))[::-1]     # increasing theta
    th, w, ids = gl_bins(th_edges, order)
    nb = len(cos_edges) - 1
    return np.cos(th), w * np.sin(th), (nb - 1) - ids


def chi2_p(obs, prob):
    obs = np.asarray(obs, np.float64).ravel()
    prob = np.asarray(prob, np.float64).ravel()
    assert abs(prob.sum() - 1.0) < 1e-8, prob.sum()
    exp = obs.sum() * prob
    # cells expecting fewer than 20 events are pooled into one cell
    small = exp < 20.0
    if np.any(small):
        obs = np.append(obs[~small], obs[small].sum())
        exp = np.append(exp[~small], exp[small].sum())
    assert exp.min() >= 5.0, exp.min()
    x2 = np.sum((obs - exp) ** 2 / exp)
    return float(stats.chi2.sf(x2, obs.size - 1))


def counts(x, edges):
    return np.histogram(x, bins=edges)[0]


def counts2(x, y, ex, ey):
    return np.histogram2d(x, y, bins=[ex, ey])[0]


def counts3(x, y, z, ex, ey, ez):
    return np.histogramdd(np.stack([x, y, z], axis=1), bins=[ex, ey, ez])[0]


M_EDGES = np.linspace(M.M_LO, M.M_HI, 31)
M_EDGES2 = np.array([M.M_LO, 5330.0, 5360.0, 5374.0, 5404.0, M.M_HI])
T_EDGES = np.array([M.T_LO, 0.4, 0.55, 0.8, 1.2, 1.8, 2.7, 4.0, 6.0, M.T_HI])
T_EDGES5 = np.array([M.T_LO, 0.6, 1.2, 2.5, 5.0, M.T_HI])
S_EDGES3 = np.linspace(0.03, 0.06, 4)
S_EDGES10 = np.linspace(0.03, 0.06, 11)
C_EDGES = np.linspace(-1.0, 1.0, 11)
C_EDGES5 = np.linspace(-1.0, 1.0, 6)
P_EDGES = np.linspace(-np.pi, np.pi, 13)
P_EDGES6 = np.linspace(-np.pi, np.pi, 7)


# ---------------------------------------------------------------------------
# Expected bin probabilities from the oracle PDFs
# ---------------------------------------------------------------------------
def prob_mass(theta):
    m, w, b = gl_bins(M_EDGES, 16)
    return np.bincount(b, w * M.pdf(1, [m], theta), minlength=len(M_EDGES) - 1)


def prob_masstime(theta):
    """(sigma_t bin, m bin, t bin) cells; sigma_t uniform on [0.03, 0.06]."""
    s, ws, bs = gl_bins(S_EDGES3, 6)
    m, wm, bm = gl_bins(M_EDGES2, 12)
    t, wt, bt = gl_bins(T_EDGES, 12)
    S, MM, T = np.meshgrid(s, m, t, indexing="ij")
    W = (ws[:, None, None] / 0.03) * wm[None, :, None] * wt[None, None, :]
    p = W * M.pdf(2, [MM.ravel(), T.ravel(), S.ravel()], theta).reshape(S.shape)
    out = np.zeros((len(S_EDGES3) - 1, len(M_EDGES2) - 1, len(T_EDGES) - 1))
    np.add.at(out, (bs[:, None, None], bm[None, :, None], bt[None, None, :]), p)
    return out


def _ang_coeffs(theta):
    fL, fpe, Fs, dpa, dpe, dS, g, dg, dm, phis = theta[:10]
    return np.array(M.time_coefficients(fL, fpe, Fs, dpa, dpe, dS, phis), np.float64)


def _sigma_rule():
    return gl_bins(S_EDGES10, 6)


def _time_int_over_sigma(theta, s, ws):
    """I_bar_j = integral over sigma_t of I_j(sigma_t) (j = 0..3)."""
    g, dg, dm = theta[6:9]
    return np.array([np.sum(ws * np.asarray(Ij)) for Ij in M.time_integrals(g, dg, dm, s)])


def _den_norm(theta):
    s, ws, _ = _sigma_rule()
    C = _ang_coeffs(theta)
    return float(M.ANGULAR_INTEGRALS @ C @ _time_int_over_sigma(theta, s, ws))


def prob_ang_sigma(theta):
    s, ws, bs = _sigma_rule()
    C = _ang_coeffs(theta)
    Dj = M.ANGULAR_INTEGRALS @ C
    g, dg, dm = theta[6:9]
    den = sum(Dj[j] * np.asarray(Ij) for j, Ij in enumerate(M.time_integrals(g, dg, dm, s)))
    return np.bincount(bs, ws * den, minlength=len(S_EDGES10) - 1) / _den_norm(theta)


def gl_fine(edges, width, order=8):
    """Composite rule: every bin split into panels no wider than `width`
    (the oscillating terms cos, sin(Delta m t) need ~20 nodes per period)."""
    xs, ws, ids = [], [], []
    for b, (lo, hi) in enumerate(zip(edges[:-1], edges[1:])):
        k = int(np.ceil((hi - lo) / width))
        x, w, _ = gl_bins(np.linspace(lo, hi, k + 1), order)
        xs.append(x)
        ws.append(w)
        ids.append(np.full(x.size, b))
    return np.concatenate(xs), np.concatenate(ws), np.concatenate(ids)


def _time_bins_over_sigma(theta, s_edges, t_edges):
    """TB[sbin, tbin, j] = integral over the sigma bin and the t bin of T_j."""
    s, ws, bs = gl_bins(s_edges, 6)
    t, wt, bt = gl_fine(t_edges, 0.05)
    g, dg, dm = theta[6:9]
    S, T = np.meshgrid(s, t, indexing="ij")
    Tj = M.time_functions(T.ravel(), g, dg, dm, S.ravel())
    out = np.zeros((len(s_edges) - 1, len(t_edges) - 1, 4))
    W = ws[:, None] * wt[None, :]
    for j in range(4):
        np.add.at(out[:, :, j], (bs[:, None], bt[None, :]), W * np.asarray(Tj[j]).reshape(S.shape))
    return out


def prob_ang_time_sigma(theta):
    C = _ang_coeffs(theta)
    Dj = M.ANGULAR_INTEGRALS @ C
    TB = _time_bins_over_sigma(theta, S_EDGES3, T_EDGES)
    return (TB @ Dj) / _den_norm(theta)


def _angular_bin_integrals(which, edges):
    """F[bin, k] = integral of f_k over the bin of one angle, the other two
    angles over their full ranges."""
    order = 10
    full_c, full_wc, _ = angle_bins(np.array([-1.0, 1.0]), 24)
    full_p, full_wp, _ = gl_bins(np.array([-np.pi, np.pi]), 24)
    if which == "phi":
        x, wx, bx = gl_bins(edges, order)
    else:
        x, wx, bx = angle_bins(edges, order)
    if which == "ck":
        ck, cl, ph = np.meshgrid(x, full_c, full_p, indexing="ij")
        W = wx[:, None, None] * full_wc[None, :, None] * full_wp[None, None, :]
    elif which == "cl":
        cl, ck, ph = np.meshgrid(x, full_c, full_p, indexing="ij")
        W = wx[:, None, None] * full_wc[None, :, None] * full_wp[None, None, :]
    else:
        ph, ck, cl = np.meshgrid(x, full_c, full_c, indexing="ij")
        W = wx[:, None, None] * full_wc[None, :, None] * full_wc[None, None, :]
    fk = M.angular_functions(ck.ravel(), cl.ravel(), ph.ravel())
    nb = len(edges) - 1
    out = np.zeros((nb, 10))
    node_bin = np.repeat(bx, W[0].size)
    for k in range(10):
        out[:, k] = np.bincount(node_bin, (W * fk[k].reshape(W.shape)).ravel(), minlength=nb)
    return out


def prob_ang_angle(theta, which, edges):
    s, ws, _ = _sigma_rule()
    A = _ang_coeffs(theta) @ _time_int_over_sigma(theta, s, ws)
    return _angular_bin_integrals(which, edges) @ A / _den_norm(theta)


def prob_ang_angle_time(theta, which, edges):
    TB = _time_bins_over_sigma(theta, np.array([0.03, 0.06]), T_EDGES5)[0]   # (t bin, j)
    F = _angular_bin_integrals(which, edges)                                   # (a bin, k)
    return F @ _ang_coeffs(theta) @ TB.T / _den_norm(theta)


def prob_trunc_gauss(mu, sig):
    m, w, b = gl_bins(M_EDGES, 16)
    g = np.exp(-(m - mu) ** 2 / (2 * sig * sig))
    p = np.bincount(b, w * g, minlength=len(M_EDGES) - 1)
    return p / p.sum()


# ---------------------------------------------------------------------------
# Samples (cached per module run: the unmodified generator is deterministic)
# ---------------------------------------------------------------------------
THETA_ALT = {
    1: (0.6, 5300.0, 22.0, -0.003),
    2: (0.5, 5340.0, 20.0, -0.003, 1.2, 0.5, 1.3),
    3: (0.45, 0.3, 0.2, 2.5, 0.4, -1.0, 0.7, -0.12, 17.0, 0.4, 5370.0, 12.0),
}
_CACHE = {}


def sample(model, theta, n=N_EVENTS, toy=0):
    key = (model, tuple(theta), n, toy)
    if key not in _CACHE:
        _CACHE[key] = G.generate(model, theta, SEED + model, toy, n)
    return _CACHE[key]


def pvalues(model, theta, r):
    """Every pin p-value of a generated sample."""
    c = r["cols"]
    th = [float(x) for x in theta]
    if model == 1:
        return {"m": chi2_p(counts(c[0], M_EDGES), prob_mass(th))}
    if model == 2:
        return {
            "sigma_t": chi2_p(counts(c[2], S_EDGES10), np.full(10, 0.1)),
            "sigma_t x m x t": chi2_p(counts3(c[2], c[0], c[1], S_EDGES3, M_EDGES2, T_EDGES),
                                      prob_masstime(th)),
        }
    ck, cl, ph, t, st, m = c
    return {
        "sigma_t": chi2_p(counts(st, S_EDGES10), prob_ang_sigma(th)),
        "t x sigma_t": chi2_p(counts2(st, t, S_EDGES3, T_EDGES), prob_ang_time_sigma(th)),
        "cos_k": chi2_p(counts(ck, C_EDGES), prob_ang_angle(th, "ck", C_EDGES)),
        "cos_l": chi2_p(counts(cl, C_EDGES), prob_ang_angle(th, "cl", C_EDGES)),
        "phi": chi2_p(counts(ph, P_EDGES), prob_ang_angle(th, "phi", P_EDGES)),
        "cos_k x t": chi2_p(counts2(ck, t, C_EDGES5, T_EDGES5), prob_ang_angle_time(th, "ck", C_EDGES5)),
        "phi x t": chi2_p(counts2(ph, t, P_EDGES6, T_EDGES5), prob_ang_angle_time(th, "phi", P_EDGES6)),
        "m": chi2_p(counts(m, M_EDGES), prob_trunc_gauss(th[10], th[11])),
        "w": chi2_p(counts(r["w"], np.linspace(0.8, 1.0, 11)), np.full(10, 0.1)),
    }


# ---------------------------------------------------------------------------
# The unmodified generator
# ---------------------------------------------------------------------------
def test_bin_probabilities_are_normalised():
    # the quadrature of the expected counts covers the whole phase space
    assert abs(prob_mass(M.THETA_GEN[1]).sum() - 1.0) < 1e-12
    assert abs(prob_masstime(M.THETA_GEN[2]).sum() - 1.0) < 1e-9
    th = M.THETA_GEN[3]
    assert abs(prob_ang_sigma(th).sum() - 1.0) < 1e-12
    assert abs(prob_ang_time_sigma(th).sum() - 1.0) < 1e-9
    for which, e in (("ck", C_EDGES), ("cl", C_EDGES), ("phi", P_EDGES)):
        assert abs(prob_ang_angle(th, which, e).sum() - 1.0) < 1e-12, which
    assert abs(prob_ang_angle_time(th, "phi", P_EDGES6).sum() - 1.0) < 1e-9


@pytest.mark.parametrize("model", [1, 2, 3])
@pytest.mark.parametrize("which", ["gen", "alt"])
def test_generated_marginals_follow_the_pdf(model, which):
    theta = M.THETA_GEN[model] if which == "gen" else THETA_ALT[model]
    r = sample(model, theta)
    assert r["violations"] == 0
    assert len(r["cols"][0]) == N_EVENTS
    ps = pvalues(model, theta, r)
    bad = {k: v for k, v in ps.items() if not v > P_MIN}
    assert not bad, bad


def test_pins_see_a_wrong_parameter_point():
    # the same pins reject a sample generated at another point: they are not
    # blind to the parameters they are meant to constrain
    for model in (1, 2, 3):
        r = sample(model, M.THETA_GEN[model])
        ps = pvalues(model, THETA_ALT[model], r)
        assert min(ps.values()) < P_FAIL, (model, ps)


THETA_GRID = {
    1: [M.THETA_GEN[1], (0.7, 5300.0, 25.0, -0.003), (0.1, 5450.0, 8.0, 0.0), (1.0, 5367.0, 15.0, 0.01),
        (0.0, 5367.0, 15.0, -0.01), (0.5, 5210.0, 40.0, 3e-6)],
    2: [M.THETA_GEN[2], (0.6, 5320.0, 20.0, 0.0, 2.0, 0.4, 1.6), (0.05, 5367.0, 15.0, -0.002, 1.2, 1.9, 0.7),
        (0.3, 5367.0, 15.0, 0.002, 1.5, 0.7, 1.3), (1.0, 5400.0, 10.0, 0.01, 0.4, 3.0, 2.0),
        (0.3, 5367.0, 15.0, 0.002, 1.5, 0.7, 4.0)],
    3: [M.THETA_GEN[3], THETA_ALT[3],
        (0.6, 0.1, 0.0, 3.0, 3.0, 0.0, 0.6, -0.05, 18.5, -0.7, 5360.0, 18.0),
        (0.3, 0.35, 0.6, -1.0, 2.0, 1.5, 0.9, 0.5, 0.5, 1.2, 5367.0, 15.0),
        (0.5, 0.25, 0.1, 3.26, 3.08, 0.35, 0.66, -0.3, 30.0, -0.03, 5367.0, 15.0)],
}


def violations(model, theta, n=1 << 17, toy=3):
    u = G.uniforms(model, SEED, toy, 0, n)
    th = [float(x) for x in theta]
    acc, out, w, marg, v = G.candidates(model, th, u, G.bound(model, th))
    return int(np.sum(v)), int(np.sum(acc))


@pytest.mark.parametrize("model", [1, 2, 3])
def test_no_bound_violations_over_a_parameter_grid(model):
    for theta in THETA_GRID[model]:
        nv, na = violations(model, theta)
        assert nv == 0, (model, theta, nv)
        assert na > 0, (model, theta)


def sup_ratio(model, theta):
    """Largest acceptance ratio over a dense grid of the proposal space (the
    bound must not be below it anywhere, not only on sampled candidates)."""
    th = [float(x) for x in theta]
    if model == 1:
        return float(np.max(M.pdf(1, [np.linspace(M.M_LO, M.M_HI, 100_001)], th)))
    if model == 2:
        s = th[6]
        rs, rb = G._masstime_ratios(th, s * np.linspace(0.03, 0.06, 4001))
        return float(max(rs.max(), rb.max()))
    C = _ang_coeffs(th)
    g, dg, dm = th[6:9]
    gmin = G._envelope_rate(g, dg)
    c = np.cos(np.linspace(0.0, np.pi, 25))
    ck, cl, ph = np.meshgrid(c, c, np.linspace(-np.pi, np.pi, 49), indexing="ij")
    fk = np.array(M.angular_functions(ck.ravel(), cl.ravel(), ph.ravel()))      # (10, n_omega)
    best = 0.0
    for t0 in np.linspace(0.0, 40.0, 801):
        e = np.exp((gmin - g) * t0)
        h = np.array([e * np.cosh(dg * t0 / 2), e * np.sinh(dg * t0 / 2), e * np.cos(dm * t0), e * np.sin(dm * t0)])
        best = max(best, float(np.max(fk.T @ (C @ h))))
    return best


@pytest.mark.parametrize("model", [1, 2, 3])
def test_bounds_cover_the_acceptance_ratio_everywhere(model):
    for theta in THETA_GRID[model]:
        sup = sup_ratio(model, theta)
        assert 0.0 < sup <= G.bound(model, [float(x) for x in theta]), (model, theta, sup)


# ---------------------------------------------------------------------------
# Planted mistakes in the sampling recipes
# ---------------------------------------------------------------------------
def _ratios_without_ng(orig):
    def f(theta, sigma):
        rs, rb = orig(theta, sigma)
        return rs * M.gauss_norm(theta[1], theta[2]), rb          # 1/N_G dropped from R_s
    return f


def _bound_mass_emax_one(theta):
    f, mu, sig, lam = theta
    return f / M.gauss_norm(mu, sig) + (1.0 - f) / M.exp_norm(lam)    # E_max = 1 also for lambda < 0


def _box_muller_no_two(ua, ub):
    r = np.sqrt(-np.log(ua))                                        # sqrt(-2 ln u) -> sqrt(-ln u)
    return r * np.cos(2.0 * np.pi * ub), r * np.sin(2.0 * np.pi * ub)


def _inverse_cdf_wrong_end(u, lam):
    L = M.M_HI - M.M_LO
    return M.M_HI + np.log1p(-u * (-np.expm1(-lam * L))) / lam       # measured from the upper end


def _phi_half_range(ua, ub, uc):
    return 2.0 * ua - 1.0, 2.0 * ub - 1.0, np.pi * uc                 # phi on [0, pi] only


def _bound_ang_without_oscillation(theta):
    """M3 missing S2, the bound of the cos / sin (Delta m) terms."""
    fL, fpe, Fs, dpa, dpe, dS, g, dg, dm, phis = [float(x) for x in theta[:10]]
    C = M.time_coefficients(fL, fpe, Fs, dpa, dpe, dS, phis)
    sg = -1.0 if dg < 0.0 else 1.0
    S0 = sum(float(G.ANG_MAX[k]) * abs(float(C[k][0])) for k in range(10))
    S1 = sum(float(G.ANG_MAX[k]) * abs(float(C[k][0]) + sg * float(C[k][1])) for k in range(10))
    return max(S0, 0.5 * S1)


def _sup_check(model, theta):
    def run():
        return 1.0, int(sup_ratio(model, theta) > G.bound(model, [float(x) for x in theta]))
    return run


def _gen_check(model, theta, n):
    def run():
        r = G.generate(model, theta, SEED + 100 + model, 0, n)
        return min(pvalues(model, theta, r).values()), r["violations"]
    return run


def _viol_check(model, theta):
    def run():
        nv, _ = violations(model, theta)
        return 1.0, nv
    return run


MUTATIONS = [
    ("R_s without 1/N_G", "_masstime_ratios", _ratios_without_ng, _gen_check(2, M.THETA_GEN[2], 60_000)),
    ("Box-Muller radius without the 2", "_box_muller", lambda o: _box_muller_no_two,
     _gen_check(2, M.THETA_GEN[2], 60_000)),
    ("exponential inverse CDF from the wrong end", "_exp_inverse_cdf", lambda o: _inverse_cdf_wrong_end,
     _gen_check(2, M.THETA_GEN[2], 60_000)),
    ("M1 with E_max = 1 for lambda < 0", "bound_mass", lambda o: _bound_mass_emax_one,
     _viol_check(1, (0.0, 5367.0, 15.0, -0.01))),
    ("Gamma_min = Gamma + |DeltaGamma|/2", "_envelope_rate", lambda o: (lambda g, dg: g + abs(dg) / 2.0),
     _viol_check(3, THETA_GRID[3][3])),
    ("Gamma_min without the absolute value", "_envelope_rate", lambda o: (lambda g, dg: g - dg / 2.0),
     _viol_check(3, THETA_GRID[3][4])),
    ("phi proposed on [0, pi]", "_angles", lambda o: _phi_half_range, _gen_check(3, M.THETA_GEN[3], 60_000)),
    ("M3 without the oscillating terms", "bound_angtime", lambda o: _bound_ang_without_oscillation,
     _sup_check(3, THETA_GRID[3][2])),
]


@pytest.mark.parametrize("label,attr,make,check", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_generator_mistake_is_caught(label, attr, make, check, monkeypatch):
    monkeypatch.setattr(G, attr, make(getattr(G, attr)))
    with np.errstate(all="ignore"):
        p, nv = check()
    assert p < P_FAIL or nv > 0, (label, p, nv)
