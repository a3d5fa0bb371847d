"""Plain FP64 definitions of the three unbinned PDFs (oracle test infrastructure).

Everything here is written from the definitions, one formula per function,
evaluated with numpy/scipy (scipy's ``erfc`` and ``wofz`` are the library
primitives).  The functions accept plain arrays or ``oracle.dual.Dual`` values
for the parameters, so the same code yields the NLL and its exact gradient.

Paper passages followed (Ipanema-beta, arXiv:1706.01420):
  * Example 1 ("Fit to a signal peak on top of an exponential background"):
    per-event mixture log-likelihood of separately normalised signal and
    background shapes, the analytic exponential integral with its k = 0 branch.
  * Example 2 ("Fit to the time and angular distribution in bins of the KK
    mass"): the B_s -> J/psi KK time-dependent angular PDF with P wave (three
    polarisations) and S wave, per-category analytic normalisation.
  * Software section and "Combining with symbolic programming": Gaussian
    resolution through the Faddeeva function and its large t/sigma limit.

Where the paper gives no formula the reading used is the standard one listed
with each function (mixture normalisation, exponential sign and shift,
convolution with a per-event Gaussian resolution, the angular/time table).
"""
import numpy as np

from . import dual as D

# Observable ranges.
M_LO, M_HI = 5200.0, 5500.0      # MeV
T_LO, T_HI = 0.3, 15.0           # ps

SQRT2 = np.sqrt(2.0)

NPARAMS = {1: 4, 2: 7, 3: 12, 4: 12}
NCOLS = {1: 1, 2: 3, 3: 6, 4: 7}
PARAM_NAMES = {
    1: ("f", "mu", "sigma", "lam"),
    2: ("f", "mu", "sigma_m", "lam", "tau_s", "tau_b", "s"),
    3: ("fL", "fpe", "Fs", "dpa", "dpe", "dS", "G", "DG", "DM", "phis", "mu_m", "sigma_m"),
}
PARAM_NAMES[4] = PARAM_NAMES[3]
COL_NAMES = {
    1: ("m",),
    2: ("m", "t", "sigma_t"),
    3: ("cos_k", "cos_l", "phi", "t", "sigma_t", "m"),
    # model 4: model 3 with a flavour tag per event, qd = q (1 - 2 omega):
    # q = +1 (B_s) / -1 (anti-B_s) the tag decision, omega its mistag probability
    4: ("cos_k", "cos_l", "phi", "t", "sigma_t", "m", "qd"),
}
THETA_GEN = {
    1: (0.3, 5367.0, 15.0, 0.002),
    2: (0.3, 5367.0, 15.0, 0.002, 1.5, 0.7, 1.0),
    3: (0.52, 0.25, 0.05, 3.26, 3.08, 0.35, 0.66, 0.08, 17.8, -0.03, 5367.0, 15.0),
}
THETA_GEN[4] = THETA_GEN[3]

# Fixed physics constants of the angular model: |lambda| = 1, C_SP = 1, delta_0 = 0.
LAMBDA_ABS = 1.0
C_SP = 1.0
DELTA_0 = 0.0


# ---------------------------------------------------------------------------
# Mass shapes (Example 1)
# ---------------------------------------------------------------------------
def gauss_shape(m, mu, sigma):
    """Unnormalised Gaussian exp(-(m-mu)^2 / (2 sigma^2))."""
    return D.exp(-((m - mu) ** 2) / (2.0 * sigma * sigma))


def gauss_norm(mu, sigma):
    """Integral of gauss_shape over [M_LO, M_HI]:
    sigma sqrt(pi/2) [erfc((M_LO-mu)/(sqrt2 sigma)) - erfc((M_HI-mu)/(sqrt2 sigma))]."""
    s2 = SQRT2 * sigma
    return sigma * np.sqrt(np.pi / 2.0) * (D.erfc((M_LO - mu) / s2) - D.erfc((M_HI - mu) / s2))


def exp_shape(m, lam):
    """Background exp(-lam (m - M_LO)); the shift to the range start only changes
    the constant that the normalisation removes (the paper uses exp(k m))."""
    return D.exp(-lam * (m - M_LO))


def exp_norm(lam):
    """Integral of exp_shape over the range, with the exact lam = 0 branch
    (Example 1 writes the k = 0 case separately)."""
    L = M_HI - M_LO
    if float(D.value(lam)) == 0.0:
        # value L, first derivative -L^2/2 (enough for the forward gradient)
        return L - lam * (L * L / 2.0)
    return -D.expm1(-lam * L) / lam


def pdf_mass(m, f, mu, sigma, lam):
    """Model 1: f G/N_G + (1-f) E/N_E, each shape normalised on the range."""
    return f * gauss_shape(m, mu, sigma) / gauss_norm(mu, sigma) + \
        (1.0 - f) * exp_shape(m, lam) / exp_norm(lam)


# ---------------------------------------------------------------------------
# Decay time with Gaussian resolution
# ---------------------------------------------------------------------------
def conv_exp(t, z, sigma):
    """F(t; z, sigma) = integral_0^inf e^{-z tau} g_sigma(t - tau) d tau, Re z > 0,
    with g_sigma the unit-area Gaussian of width sigma.

    Closed form: F = 1/2 exp(z^2 sigma^2/2 - z t) erfc((z sigma^2 - t)/(sqrt2 sigma))
               = 1/2 exp(-t^2/(2 sigma^2)) w(u),   u = i (z sigma^2 - t)/(sqrt2 sigma).
    For Im u < 0 the reflection w(u) = 2 exp(-u^2) - w(-u) gives
        F = exp(z^2 sigma^2/2 - z t) - 1/2 exp(-t^2/(2 sigma^2)) w(-u),
    whose second term is the large-t/sigma correction.  Returns a complex value."""
    z = z + 0j
    u = 1j * (z * sigma * sigma - t) / (SQRT2 * sigma)
    upper = np.imag(D.value(u)) >= 0.0
    uu = D.where(upper, u, -u)
    gt = D.exp(-(t * t) / (2.0 * sigma * sigma))
    half_gw = 0.5 * gt * D.wofz(uu)
    main = D.exp(z * z * sigma * sigma / 2.0 - z * t)
    return D.where(upper, half_gw, main - half_gw)


def gauss_cdf(t, sigma):
    """Phi(t) = integral_{-inf}^t g_sigma = 1/2 erfc(-t/(sqrt2 sigma))."""
    return 0.5 * D.erfc(-t / (SQRT2 * sigma))


def conv_exp_integral(z, sigma, a=T_LO, b=T_HI):
    """integral_a^b F(t; z, sigma) dt = (1/z) [Phi(b) - Phi(a) - F(b) + F(a)],
    from dF/dt = g_sigma(t) - z F(t)."""
    z = z + 0j
    return (1.0 / z) * (gauss_cdf(b, sigma) - gauss_cdf(a, sigma)
                        - conv_exp(b, z, sigma) + conv_exp(a, z, sigma))


def time_pdf(t, gamma, sigma):
    """Per-event normalised decay-time PDF F(t;gamma,sigma)/I(gamma,sigma) on [T_LO, T_HI]."""
    return D.real(conv_exp(t, gamma, sigma)) / D.real(conv_exp_integral(gamma, sigma))


def pdf_masstime(m, t, sigma_t, f, mu, sigma_m, lam, tau_s, tau_b, s):
    """Model 2: f [G/N_G][F_s/I_s] + (1-f) [E/N_E][F_b/I_b] with per-event
    resolution sigma_i = s sigma_t,i; conditional on sigma_t."""
    sig = s * sigma_t
    sig_part = gauss_shape(m, mu, sigma_m) / gauss_norm(mu, sigma_m) * time_pdf(t, 1.0 / tau_s, sig)
    bkg_part = exp_shape(m, lam) / exp_norm(lam) * time_pdf(t, 1.0 / tau_b, sig)
    return f * sig_part + (1.0 - f) * bkg_part


# ---------------------------------------------------------------------------
# Angular x decay-time model (Example 2, one flavour)
# ---------------------------------------------------------------------------
def angular_functions(cos_k, cos_l, phi):
    """The ten angular functions f_k(Omega) of the P + S wave decomposition
    (helicity angles theta_K, theta_l, phi)."""
    sk2 = 1.0 - cos_k * cos_k
    sl2 = 1.0 - cos_l * cos_l
    sk = np.sqrt(sk2)
    sl = np.sqrt(sl2)
    s2k = 2.0 * sk * cos_k          # sin 2 theta_K
    s2l = 2.0 * sl * cos_l          # sin 2 theta_l
    cp, sp_ = np.cos(phi), np.sin(phi)
    return [
        2.0 * cos_k * cos_k * sl2,
        sk2 * (1.0 - sl2 * cp * cp),
        sk2 * (1.0 - sl2 * sp_ * sp_),
        sk2 * sl2 * np.sin(2.0 * phi),
        -(np.sqrt(2.0) / 2.0) * s2k * s2l * cp,
        (np.sqrt(2.0) / 2.0) * s2k * s2l * sp_,
        (2.0 / 3.0) * sl2,
        -(np.sqrt(6.0) / 3.0) * sk * s2l * cp,
        (np.sqrt(6.0) / 3.0) * sk * s2l * sp_,
        (4.0 * np.sqrt(3.0) / 3.0) * cos_k * sl2,
    ]


# Integrals of f_k over cos_k, cos_l in [-1, 1] and phi in [-pi, pi].
ANGULAR_INTEGRALS = np.array([32.0 * np.pi / 9.0] * 3 + [0.0] * 3 + [32.0 * np.pi / 9.0] + [0.0] * 3)


def time_coefficients(fL, fpe, Fs, dpa, dpe, dS, phis, c_sp=None):
    """C[k][j] = N_k (a_k, b_k, c_k, d_k): the weights of the cosh, sinh, cos and
    sin time terms in term k, for a B_s at production.  c_sp: the S-P
    interference factor of the KK-mass bin (Example 2 fits one per bin; the
    module constant C_SP when None)."""
    if c_sp is None:
        c_sp = C_SP
    l2 = LAMBDA_ABS * LAMBDA_ABS
    C = (1.0 - l2) / (1.0 + l2)
    S = -2.0 * LAMBDA_ABS * D.sin(phis) / (1.0 + l2)
    Dd = -2.0 * LAMBDA_ABS * D.cos(phis) / (1.0 + l2)
    a0 = (1.0 - Fs) * fL
    ape = (1.0 - Fs) * fpe
    apa = (1.0 - Fs) * (1.0 - fL - fpe)
    aS = Fs
    r0, rpe, rpa, rS = D.sqrt(a0), D.sqrt(ape), D.sqrt(apa), D.sqrt(aS)
    d0 = DELTA_0
    s_pe_pa, c_pe_pa = D.sin(dpe - dpa), D.cos(dpe - dpa)
    c_pa_0 = D.cos(dpa - d0)
    s_pe_0, c_pe_0 = D.sin(dpe - d0), D.cos(dpe - d0)
    c_pa_S, s_pa_S = D.cos(dpa - dS), D.sin(dpa - dS)
    s_pe_S = D.sin(dpe - dS)
    c_0_S, s_0_S = D.cos(d0 - dS), D.sin(d0 - dS)
    rows = [
        (a0, (1.0, Dd, C, -S)),
        (apa, (1.0, Dd, C, -S)),
        (ape, (1.0, -Dd, C, S)),
        (rpa * rpe, (C * s_pe_pa, S * c_pe_pa, s_pe_pa, Dd * c_pe_pa)),
        (r0 * rpa, (c_pa_0, Dd * c_pa_0, C * c_pa_0, -S * c_pa_0)),
        (r0 * rpe, (C * s_pe_0, S * c_pe_0, s_pe_0, Dd * c_pe_0)),
        (aS, (1.0, -Dd, C, S)),
        (c_sp * rS * rpa, (C * c_pa_S, S * s_pa_S, c_pa_S, Dd * s_pa_S)),
        (c_sp * rS * rpe, (s_pe_S, -Dd * s_pe_S, C * s_pe_S, S * s_pe_S)),
        (c_sp * rS * r0, (C * c_0_S, S * s_0_S, c_0_S, Dd * s_0_S)),
    ]
    return [[nk * x for x in abcd] for nk, abcd in rows]


def time_functions(t, G, DG, DM, sigma):
    """T_1..T_4 = resolution-convolved e^{-G t} x (cosh(DG t/2), sinh(DG t/2),
    cos(DM t), sin(DM t)), through Gamma_H = G - DG/2, Gamma_L = G + DG/2 and
    z = G - i DM."""
    gH = G - DG / 2.0
    gL = G + DG / 2.0
    FH = D.real(conv_exp(t, gH, sigma))
    FL = D.real(conv_exp(t, gL, sigma))
    Fc = conv_exp(t, G - 1j * DM, sigma)
    return [0.5 * (FH + FL), 0.5 * (FH - FL), D.real(Fc), D.imag(Fc)]


def time_integrals(G, DG, DM, sigma):
    """I_1..I_4: the same combinations of integral_{T_LO}^{T_HI} F dt."""
    gH = G - DG / 2.0
    gL = G + DG / 2.0
    IH = D.real(conv_exp_integral(gH, sigma))
    IL = D.real(conv_exp_integral(gL, sigma))
    Ic = conv_exp_integral(G - 1j * DM, sigma)
    return [0.5 * (IH + IL), 0.5 * (IH - IL), D.real(Ic), D.imag(Ic)]


def pdf_angtime(cos_k, cos_l, phi, t, sigma_t, m,
                fL, fpe, Fs, dpa, dpe, dS, G, DG, DM, phis, mu_m, sigma_m,
                qd=1.0, xi=None, c_sp=None):
    """Model 3: [sum_k f_k(Omega) sum_j C_kj T_j(t|sigma)] / [sum_j D_j I_j(sigma)]
    x G(m)/N_G, with D_j = sum_k xi_k C_kj and xi_k = integral f_k dOmega.

    Model 4 (tagged) passes qd = q (1 - 2 omega) per event: an event tagged q
    with mistag probability omega is a B_s with probability 1 - omega when
    q = +1, and the anti-B_s PDF has the cos and sin weights (c_k, d_k) of
    the opposite sign, so the mixture (1 - omega) |A|^2 + omega |Abar|^2 has
    the cos and sin terms scaled by qd in the numerator and in the
    normalisation alike (qd = +1: B_s, qd = -1: anti-B_s, qd = 0: untagged).

    xi: the ten normalisation weights xi_k = integral eps(Omega) f_k dOmega of
    an angular efficiency eps (flat efficiency: the analytic integrals); the
    PDF is then normalised against eps, the efficiency itself being a
    constant factor per event that the likelihood drops."""
    Cm = time_coefficients(fL, fpe, Fs, dpa, dpe, dS, phis, c_sp)
    fk = angular_functions(cos_k, cos_l, phi)
    T = time_functions(t, G, DG, DM, sigma_t)
    I = time_integrals(G, DG, DM, sigma_t)
    T = [T[0], T[1], qd * T[2], qd * T[3]]
    I = [I[0], I[1], qd * I[2], qd * I[3]]
    xk = ANGULAR_INTEGRALS if xi is None else xi
    num = 0.0
    for k in range(10):
        for j in range(4):
            num = num + fk[k] * (Cm[k][j] * T[j])
    den = 0.0
    for j in range(4):
        Dj = 0.0
        for k in range(10):
            if xk[k] != 0.0:
                Dj = Dj + xk[k] * Cm[k][j]
        den = den + Dj * I[j]
    return num / den * gauss_shape(m, mu_m, sigma_m) / gauss_norm(mu_m, sigma_m)


# ---------------------------------------------------------------------------
# Parameter domain (values outside give +inf NLL)
# ---------------------------------------------------------------------------
def theta_valid(model, theta):
    th = [float(D.value(x)) for x in theta]
    if len(th) != NPARAMS[model] or not all(np.isfinite(th)):
        return False
    if model == 1:
        f, mu, sig, lam = th
        return 0.0 <= f <= 1.0 and sig > 0.0
    if model == 2:
        f, mu, sig, lam, ts, tb, s = th
        return 0.0 <= f <= 1.0 and sig > 0.0 and ts > 0.0 and tb > 0.0 and s > 0.0
    fL, fpe, Fs, dpa, dpe, dS, G, DG, DM, phis, mu, sig = th
    return (fL >= 0.0 and fpe >= 0.0 and fL + fpe <= 1.0 and 0.0 <= Fs <= 1.0
            and sig > 0.0 and G - abs(DG) / 2.0 > 0.0)


def pdf(model, cols, theta, settings=None):
    """Per-event PDF values; cols in COL_NAMES order, theta in PARAM_NAMES order.
    settings (models 3 and 4): a dict with the dataset's normalisation weights
    "xi" (ten values) and S-P factor "c_sp"; absent keys take the flat
    efficiency and the module's C_SP."""
    st = settings or {}
    if model == 1:
        return pdf_mass(cols[0], *theta)
    if model == 2:
        return pdf_masstime(cols[0], cols[1], cols[2], *theta)
    if model == 3:
        return pdf_angtime(*cols, *theta, xi=st.get("xi"), c_sp=st.get("c_sp"))
    if model == 4:
        return pdf_angtime(*cols[:6], *theta, qd=cols[6], xi=st.get("xi"), c_sp=st.get("c_sp"))
    raise ValueError("unknown model %r" % (model,))
