"""Planted mistakes in the oracle (on the CPU) must each fail at least one pin.

Every case monkeypatches one oracle function with a plausible error (dropped
term, wrong sign, swapped operand, wrong constant) and checks that the
corresponding independent reference detects it.  The unmodified oracle passes
the same checks in the other test files.
"""
import numpy as np
import pytest

import pins
from oracle import models as M

THETA3 = M.THETA_GEN[3]


# -- checks (return the deviation that the pin tolerances bound) --------------
def dev_conv_mpmath():
    worst = 0.0
    for z in [0.66 - 17.8j, 0.62 + 0j]:
        for s in [0.045, 0.06, 0.25]:
            for t in [0.0, 0.3, 0.45, 2.0]:
                g = M.conv_exp(np.array([t]), z, s)[0]
                r = pins.conv_exp_mpmath(t, z, s)
                worst = max(worst, abs(g - r) / abs(r))
    return worst                                   # pin: < 1e-12


def dev_time_integral():
    x, w = pins.gl_composite(M.T_LO, M.T_HI, 100, 16)
    worst = 0.0
    for z in [0.66 - 17.8j, 0.62 + 0j]:
        num = np.sum(w * M.conv_exp(x, z, 0.05))
        worst = max(worst, abs(M.conv_exp_integral(z, 0.05) - num) / abs(num))
    return worst                                   # pin: < 1e-12


def dev_mass_norm():
    m, w = pins.gl_composite(M.M_LO, M.M_HI, 10, 16)
    return max(abs(np.sum(w * M.pdf(1, [m], th)) - 1.0)
               for th in [M.THETA_GEN[1], (0.7, 5300.0, 25.0, -0.003)])   # pin: < 1e-13


def dev_helicity():
    fL, fpe, Fs, dpa, dpe, dS, G, DG, DM, phis, _, _ = (0.45, 0.3, 0.2, 2.5, 0.4, -1.0, 0.7, 0.12, 17.0, 0.4, 0, 0)
    rng = np.random.default_rng(5)
    n = 200
    ck, cl = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    ph, t = rng.uniform(-np.pi, np.pi, n), rng.uniform(0.0, 6.0, n)
    A = pins.mixing_amplitudes(fL, fpe, Fs, dpa, dpe, dS, G, DG, DM, phis, M.LAMBDA_ABS, t)
    lhs = pins.helicity_density(A["0"], A["pa"], A["pe"], A["S"], ck, cl, ph)
    Cm = M.time_coefficients(fL, fpe, Fs, dpa, dpe, dS, phis)
    fk = M.angular_functions(ck, cl, ph)
    e = np.exp(-G * t)
    h = [e * np.cosh(DG * t / 2), e * np.sinh(DG * t / 2), e * np.cos(DM * t), e * np.sin(DM * t)]
    rhs = sum(fk[k] * sum(Cm[k][j] * h[j] for j in range(4)) for k in range(10))
    return np.max(np.abs(lhs / rhs / ((1 + M.LAMBDA_ABS ** 2) / 4) - 1))   # pin: < 1e-12


def dev_angtime_norm():
    theta, sigma_t = THETA3, 0.045
    ck, cl, ph, wa = pins.angular_grid(4, 6)
    t, wt = pins.gl_composite(M.T_LO, M.T_HI, 60, 12)
    A = np.repeat(np.arange(ck.size), t.size)
    Tt = np.tile(t, ck.size)
    p = M.pdf(3, [ck[A], cl[A], ph[A], Tt, np.full(Tt.size, sigma_t), np.full(Tt.size, theta[10])], theta)
    i_ot = np.sum(wa[A] * np.tile(wt, ck.size) * p)
    m, wm = pins.gl_composite(M.M_LO, M.M_HI, 10, 16)
    g = np.exp(-(m - theta[10]) ** 2 / (2 * theta[11] ** 2))
    # divide out the mass factor at m0 = mu (its unnormalised value is 1)
    return abs(i_ot * np.sum(wm * g) - 1.0)       # pin: < 1e-11


def dev_time_functions_limit():
    t = np.linspace(M.T_LO, M.T_HI, 40)
    G, DG, DM = 0.66, 0.08, 17.8
    T = M.time_functions(t, G, DG, DM, 1e-6)
    e = np.exp(-G * t)
    ref = [e * np.cosh(DG * t / 2), e * np.sinh(DG * t / 2), e * np.cos(DM * t), e * np.sin(DM * t)]
    return max(np.max(np.abs(a - b)) for a, b in zip(T, ref)) / e.max()   # pin: < 1e-7


CHECKS = {
    "conv": (dev_conv_mpmath, 1e-12),
    "tint": (dev_time_integral, 1e-12),
    "mass": (dev_mass_norm, 1e-13),
    "heli": (dev_helicity, 1e-12),
    "norm3": (dev_angtime_norm, 1e-11),
    "tlim": (dev_time_functions_limit, 1e-7),
}


def test_unmodified_oracle_passes_all_checks():
    for name, (fn, tol) in CHECKS.items():
        assert fn() < tol, name


# -- mutations -----------------------------------------------------------------
def _conv_no_correction(t, z, sigma):
    from oracle import dual as D
    z = z + 0j
    u = 1j * (z * sigma * sigma - t) / (M.SQRT2 * sigma)
    upper = np.imag(D.value(u)) >= 0.0
    uu = D.where(upper, u, -u)
    gt = D.exp(-(t * t) / (2.0 * sigma * sigma))
    half_gw = 0.5 * gt * D.wofz(uu)
    main = D.exp(z * z * sigma * sigma / 2.0 - z * t)
    return D.where(upper, half_gw, main)          # correction term dropped


def _wrap_conv_sign(orig):
    def f(t, z, sigma):
        from oracle import dual as D
        z = z + 0j
        return orig(t, z, sigma) * D.exp(-z * z * sigma * sigma)   # exponent z^2 s^2/2 -> -z^2 s^2/2
    return f


def _integral_wrong_sign(z, sigma, a=M.T_LO, b=M.T_HI):
    z = z + 0j
    return (1.0 / z) * (M.gauss_cdf(b, sigma) - M.gauss_cdf(a, sigma) + M.conv_exp(b, z, sigma) + M.conv_exp(a, z, sigma))


def _wrap_table(orig, k, j, fn):
    def f(*a, **kw):
        Cm = orig(*a, **kw)
        Cm[k][j] = fn(Cm[k][j])
        return Cm
    return f


def _wrap_table_swap(orig, k, j1, j2):
    def f(*a, **kw):
        Cm = orig(*a, **kw)
        Cm[k][j1], Cm[k][j2] = Cm[k][j2], Cm[k][j1]
        return Cm
    return f


def _wrap_angular(orig, k, fn):
    def f(ck, cl, phi):
        fk = orig(ck, cl, phi)
        fk[k] = fn(fk[k], ck, cl, phi)
        return fk
    return f


def _wrap_time_functions(orig):
    def f(*a, **kw):
        T = orig(*a, **kw)
        return [T[0], -T[1], T[2], T[3]]           # sinh term with the wrong sign
    return f


MUTATIONS = [
    ("drop large-t/sigma correction", "conv_exp", lambda o: _conv_no_correction, "conv"),
    ("wrong sign of z^2 sigma^2/2", "conv_exp", _wrap_conv_sign, "conv"),
    ("wrong sign of F(b) in integral", "conv_exp_integral", lambda o: _integral_wrong_sign, "tint"),
    ("expm1 sign in exponential norm", "exp_norm",
     lambda o: (lambda lam: D_expm1_plus(lam)), "mass"),
    ("sqrt(pi) instead of sqrt(pi/2)", "gauss_norm",
     lambda o: (lambda mu, s: o(mu, s) * np.sqrt(2.0)), "mass"),
    ("sign of S in k=1 sin weight", "time_coefficients",
     lambda o: _wrap_table(o, 0, 3, lambda x: -x), "heli"),
    ("swap sinh/cos weights of k=4", "time_coefficients",
     lambda o: _wrap_table_swap(o, 3, 1, 2), "heli"),
    ("cos phi -> sin phi in f_5", "angular_functions",
     lambda o: _wrap_angular(o, 4, lambda fk, ck, cl, ph: fk * np.tan(ph)), "heli"),
    ("wrong constant in f_10", "angular_functions",
     lambda o: _wrap_angular(o, 9, lambda fk, ck, cl, ph: 0.5 * fk), "heli"),
    ("transposed indices: f_2 <-> f_3", "angular_functions",
     lambda o: (lambda ck, cl, ph: (lambda fk: fk[:1] + [fk[2], fk[1]] + fk[3:])(o(ck, cl, ph))), "heli"),
    ("sinh sign in time functions", "time_functions", _wrap_time_functions, "tlim"),
]


def D_expm1_plus(lam):
    L = M.M_HI - M.M_LO
    return np.expm1(lam * L) / lam


@pytest.mark.parametrize("label,attr,make,check", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(label, attr, make, check, monkeypatch):
    orig = getattr(M, attr)
    monkeypatch.setattr(M, attr, make(orig))
    fn, tol = CHECKS[check]
    with np.errstate(all="ignore"):
        dev = fn()
    assert not (dev < tol), (label, dev)


def test_wrong_angular_integral_is_caught(monkeypatch):
    xi = M.ANGULAR_INTEGRALS.copy()
    xi[1] *= 1.01
    monkeypatch.setattr(M, "ANGULAR_INTEGRALS", xi)
    assert not (dev_angtime_norm() < 1e-11)


# -- tagged angular model, efficiency weights, S-P factor (model 4) -------------
def _tag_ratio_dev(qd, theta=(0.45, 0.3, 0.2, 2.5, 0.4, -1.0, 0.7, 0.12, 17.0, 0.4, 5370.0, 12.0)):
    rng = np.random.default_rng(8)
    n = 150
    ck, cl, ph, t = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(-np.pi, np.pi, n), rng.uniform(0.3, 6, n)
    fL, fpe, Fs, dpa, dpe, dS, G, DG, DM, phis, _, _ = theta
    A = pins.mixing_amplitudes(fL, fpe, Fs, dpa, dpe, dS, G, DG, DM, phis, M.LAMBDA_ABS, t)
    B = pins.mixing_amplitudes_bar(fL, fpe, Fs, dpa, dpe, dS, G, DG, DM, phis, M.LAMBDA_ABS, t)
    om = (1 - qd) / 2
    ref = (1 - om) * pins.helicity_density(A["0"], A["pa"], A["pe"], A["S"], ck, cl, ph) + \
        om * pins.helicity_density(B["0"], B["pa"], B["pe"], B["S"], ck, cl, ph)
    p = M.pdf(4, [ck, cl, ph, t, np.full(n, 1e-8), np.full(n, theta[10]), np.full(n, qd)], theta)
    r = p / ref
    return np.max(np.abs(r / r[0] - 1))


def dev_flavour():
    return max(_tag_ratio_dev(-1.0), _tag_ratio_dev(0.46))          # pin: < 1e-12


def _ot_integral(qd, settings=None, eps=None, theta=THETA3, sigma_t=0.045):
    ck, cl, ph, wa = pins.angular_grid(8, 16) if eps is not None else pins.angular_grid(4, 6)
    t, wt = pins.gl_composite(M.T_LO, M.T_HI, 60, 12)
    A = np.repeat(np.arange(ck.size), t.size)
    Tt = np.tile(t, ck.size)
    n = Tt.size
    p = M.pdf(4, [ck[A], cl[A], ph[A], Tt, np.full(n, sigma_t), np.full(n, theta[10]), np.full(n, qd)],
              theta, settings)
    if eps is not None:
        p = p * eps(ck[A], cl[A], ph[A])
    m, wm = pins.gl_composite(M.M_LO, M.M_HI, 10, 16)
    g = np.exp(-(m - theta[10]) ** 2 / (2 * theta[11] ** 2))
    return np.sum(wa[A] * np.tile(wt, ck.size) * p) * np.sum(wm * g)


def dev_tag_norm():
    return max(abs(_ot_integral(qd) - 1.0) for qd in (-1.0, -0.35))   # pin: < 1e-11


def dev_xi_norm():
    ck, cl, ph, w = pins.angular_grid(8, 16)
    e = pins.acceptance(ck, cl, ph)
    xi = np.array([np.sum(w * e * f) for f in M.angular_functions(ck, cl, ph)])
    return abs(_ot_integral(0.7, {"xi": xi}, pins.acceptance) - 1.0)   # pin: < 1e-11


def dev_csp(c_sp=0.5, theta=(0.45, 0.3, 0.2, 2.5, 0.4, -1.0, 0.7, 0.12, 17.0, 0.4, 5370.0, 12.0)):
    rng = np.random.default_rng(12)
    n = 150
    ck, cl, ph, t = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(-np.pi, np.pi, n), rng.uniform(0.3, 6, n)
    fL, fpe, Fs, dpa, dpe, dS, G, DG, DM, phis, _, _ = theta
    A = pins.mixing_amplitudes(fL, fpe, Fs, dpa, dpe, dS, G, DG, DM, phis, M.LAMBDA_ABS, t)
    ref = pins.helicity_density_csp(A["0"], A["pa"], A["pe"], A["S"], ck, cl, ph, c_sp)
    p = M.pdf(4, [ck, cl, ph, t, np.full(n, 1e-8), np.full(n, theta[10]), np.ones(n)], theta, {"c_sp": c_sp})
    r = p / ref
    return np.max(np.abs(r / r[0] - 1))                               # pin: < 1e-12


CHECKS.update({
    "flav": (dev_flavour, 1e-12),
    "tagnorm": (dev_tag_norm, 1e-11),
    "xinorm": (dev_xi_norm, 1e-11),
    "csp": (dev_csp, 1e-12),
})


def _mutant_pdf_angtime(qd_num_only=False, flip_ab=False, ignore_xi=False):
    """pdf_angtime with one planted mistake in how the tag or the efficiency
    weights enter."""
    def f(cos_k, cos_l, phi, t, sigma_t, m, fL, fpe, Fs, dpa, dpe, dS, G, DG, DM, phis, mu_m, sigma_m,
          qd=1.0, xi=None, c_sp=None):
        Cm = M.time_coefficients(fL, fpe, Fs, dpa, dpe, dS, phis, c_sp)
        fk = M.angular_functions(cos_k, cos_l, phi)
        T = M.time_functions(t, G, DG, DM, sigma_t)
        I = M.time_integrals(G, DG, DM, sigma_t)
        if flip_ab:
            T = [qd * T[0], qd * T[1], T[2], T[3]]
            I = [qd * I[0], qd * I[1], I[2], I[3]]
        else:
            T = [T[0], T[1], qd * T[2], qd * T[3]]
            if not qd_num_only:
                I = [I[0], I[1], qd * I[2], qd * I[3]]
        xk = M.ANGULAR_INTEGRALS if (xi is None or ignore_xi) else xi
        num = sum(fk[k] * (Cm[k][j] * T[j]) for k in range(10) for j in range(4))
        den = sum(sum(xk[k] * Cm[k][j] for k in range(10)) * I[j] for j in range(4))
        return num / den * M.gauss_shape(m, mu_m, sigma_m) / M.gauss_norm(mu_m, sigma_m)
    return f


def _csp_on_swave_rate(orig):
    def f(fL, fpe, Fs, dpa, dpe, dS, phis, c_sp=None):
        Cm = orig(fL, fpe, Fs, dpa, dpe, dS, phis, c_sp)
        if c_sp is not None:
            Cm[6] = [c_sp * x for x in Cm[6]]       # C_SP also on |A_S|^2
        return Cm
    return f


TAG_MUTATIONS = [
    ("tag dilution left out of the normalisation", "pdf_angtime",
     lambda o: _mutant_pdf_angtime(qd_num_only=True), "tagnorm"),
    ("flavour flip on cosh/sinh instead of cos/sin", "pdf_angtime",
     lambda o: _mutant_pdf_angtime(flip_ab=True), "flav"),
    ("efficiency weights ignored", "pdf_angtime", lambda o: _mutant_pdf_angtime(ignore_xi=True), "xinorm"),
    ("C_SP applied to the S-wave rate", "time_coefficients", _csp_on_swave_rate, "csp"),
]


def test_unmodified_oracle_passes_tagged_checks():
    for name in ("flav", "tagnorm", "xinorm", "csp"):
        fn, tol = CHECKS[name]
        assert fn() < tol, name


@pytest.mark.parametrize("label,attr,make,check", TAG_MUTATIONS, ids=[m[0] for m in TAG_MUTATIONS])
def test_planted_tag_mistake_is_caught(label, attr, make, check, monkeypatch):
    orig = getattr(M, attr)
    monkeypatch.setattr(M, attr, make(orig))
    fn, tol = CHECKS[check]
    with np.errstate(all="ignore"):
        dev = fn()
    assert not (dev < tol), (label, dev)


def test_planted_sim_layout_mistake_is_caught(monkeypatch):
    """Fs and delta_S of a bin exchanged in the category mapping: the
    one-bin check of the layout fails."""
    from oracle import sim as S
    orig = S.category_index

    def swapped(b):
        ix = orig(b)
        ix[2], ix[5] = ix[5], ix[2]
        return ix
    monkeypatch.setattr(S, "category_index", swapped)
    th = np.arange(12, dtype=float)
    assert S.category_theta(th, 0) != [th[0], th[1], th[10], th[2], th[3], th[11]] + list(th[4:10])
