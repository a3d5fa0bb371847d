"""Unbinned toy generation by accept-reject (oracle test infrastructure).

Follows the paper's Example 5 (pseudo-experiments generated on the device by
accept-reject from a counter-based stream, Poisson-fluctuated sizes drawn on
the host).  The random stream is Philox4x64-10 (``oracle.philox``):

  key      = (seed, toy_id)
  counter  = (c, b, model, 0) for candidate c = 0, 1, 2, ... and block b
  uniforms u[4 b + j] = ((word_j >> 12) + 0.5) 2^-52, j = 0..3

Each candidate uses a fixed number of blocks (model 1: 1, model 2: 2,
model 3: 3).  A candidate is accepted or rejected on its own words only; the
output is the first n accepted candidates in increasing c.

Per model (every acceptance test is "u M < R" with a strict '<'):

  1  m = 5200 + 300 u0;  accept iff u1 M1 < P1(m), M1 = f/N_G + (1-f) E_max/N_E
     (E_max = 1 for lambda >= 0, e^{-300 lambda} otherwise).

  2  sigma_t = 0.03 + 0.03 u0 (sigma = s sigma_t); component signal iff u1 < f;
     Box-Muller r = sqrt(-2 ln u2), g1 = r cos(2 pi u3), g2 = r sin(2 pi u3);
     signal m = mu + sigma_m g1, background m by the inverse CDF of E on the
     range with u4; t = -tau_c ln u5 + sigma g2.  With both observables in
     range the ratio target/proposal is
         R_s = sigma_m sqrt(2 pi) / (N_G Gamma_s I_s(sigma)),
         R_b = 1 / (Gamma_b I_b(sigma)),
     and the candidate is accepted iff u6 M2 < R_c with one bound M2 common to
     both components (so the component fractions stay f, 1 - f at every
     sigma): M2 = (1 + 1e-3) max over 64 equally spaced sigma in
     [0.03 s, 0.06 s] (ends included) of max(R_s, R_b).

  3  sigma_t = 0.03 + 0.03 u0; true time t0 = -ln(u1)/Gamma_min with
     Gamma_min = Gamma - |DeltaGamma|/2; cos_k = 2 u2 - 1, cos_l = 2 u3 - 1,
     phi = pi (2 u4 - 1); accept iff
         u5 M3 < e^{Gamma_min t0} sum_k f_k(Omega) sum_j C_kj h_j(t0)
     (the unconvolved time-angular density; h = e^{-Gamma t}(cosh, sinh,
     cos, sin)), M3 of bound_angtime (about 15 % acceptance at the
     generation point); then Box-Muller with u6, u7:
     t = t0 + sigma_t g1 kept in [0.3, 15], m = mu_m + sigma_m g2 kept in
     [5200, 5500]; weight w = 0.8 + 0.2 u8.

Conditional on sigma_t every accepted sample follows the model's PDF exactly.
Candidates whose ratio exceeds the bound are counted ("violations"; must be 0).
"""
import numpy as np

from . import models as Mo
from . import philox as P

BLOCKS = {1: 1, 2: 2, 3: 3}
CHUNK = 1 << 15
SIGMA_GRID = 64
M2_SAFETY = 1e-3
ANG_MAX = np.array([2.0, 1.0, 1.0, 1.0, np.sqrt(2.0) / 2, np.sqrt(2.0) / 2, 2.0 / 3.0,
                    np.sqrt(6.0) / 3, np.sqrt(6.0) / 3, 4.0 * np.sqrt(3.0) / 3])


def uniforms(model, seed, toy_id, c0, count):
    """(count, 4 * blocks) uniforms of candidates c0 .. c0 + count - 1."""
    B = BLOCKS[model]
    c = np.arange(c0, c0 + count, dtype=np.uint64)
    out = np.empty((count, 4 * B))
    key = np.array([seed, toy_id], dtype=np.uint64)
    for b in range(B):
        ctr = np.stack([c, np.full(count, b, np.uint64), np.full(count, model, np.uint64),
                        np.zeros(count, np.uint64)], axis=1)
        out[:, 4 * b:4 * b + 4] = P.to_uniform(P.philox(ctr, key))
    return out


# ---------------------------------------------------------------------------
# Bounds
# ---------------------------------------------------------------------------
def bound_mass(theta):
    f, mu, sig, lam = theta
    L = Mo.M_HI - Mo.M_LO
    emax = 1.0 if lam >= 0 else np.exp(-lam * L)
    return f / Mo.gauss_norm(mu, sig) + (1.0 - f) * emax / Mo.exp_norm(lam)


def _masstime_ratios(theta, sigma):
    f, mu, sig_m, lam, tau_s, tau_b, s = theta
    gs, gb = 1.0 / tau_s, 1.0 / tau_b
    Is = np.real(Mo.conv_exp_integral(gs, sigma))
    Ib = np.real(Mo.conv_exp_integral(gb, sigma))
    rs = sig_m * np.sqrt(2.0 * np.pi) / Mo.gauss_norm(mu, sig_m) / (gs * Is)
    rb = 1.0 / (gb * Ib)
    return rs, rb


def bound_masstime(theta):
    s = theta[6]
    grid = s * (0.03 + 0.03 * np.arange(SIGMA_GRID) / (SIGMA_GRID - 1))
    rs, rb = _masstime_ratios(theta, grid)
    return (1.0 + M2_SAFETY) * max(np.max(rs), np.max(rb))


def bound_angtime(theta):
    """M3 = (1 + 1e-12) [max(S0, S1 / 2) + S2], over k = 0 .. 9 with
    m_k = max|f_k|:
        S0 = sum m_k |C_k0|,  S1 = sum m_k |C_k0 + s C_k1|  (s = sign of DeltaGamma, + for 0),
        S2 = sum m_k sqrt(C_k2^2 + C_k3^2).
    Why it bounds the ratio: with x = e^{-|DeltaGamma| t0} in (0, 1], the time
    functions times e^{Gamma_min t0} are h0 = (1 + x)/2, h1 = s (1 - x)/2 and
    (h2, h3) of length sqrt(x) <= 1; with A_j = sum_k f_k C_kj the ratio is
    [(A0 + s A1) + x (A0 - s A1)]/2 + A2 h2 + A3 h3, whose first part is linear
    in x (largest modulus at x = 0 or 1: |A0 + s A1|/2 or |A0|) and whose
    second part is at most |(A2, A3)|; then |A0| <= S0, |A0 + s A1| <= S1 and
    |(A2, A3)| <= S2 (triangle inequalities).  The factor covers the rounding
    of the sums.  Sums in increasing k."""
    fL, fpe, Fs, dpa, dpe, dS, G, DG, DM, phis = theta[:10]
    C = Mo.time_coefficients(fL, fpe, Fs, dpa, dpe, dS, phis)
    s = -1.0 if DG < 0.0 else 1.0
    S0 = S1 = S2 = 0.0
    for k in range(10):
        c0, c1, c2, c3 = (float(C[k][j]) for j in range(4))
        m = float(ANG_MAX[k])
        S0 += m * abs(c0)
        S1 += m * abs(c0 + s * c1)
        S2 += m * float(np.sqrt(c2 * c2 + c3 * c3))
    return (1.0 + 1e-12) * (max(S0, 0.5 * S1) + S2)


# ---------------------------------------------------------------------------
# Candidates
# ---------------------------------------------------------------------------
def _box_muller(ua, ub):
    """Two independent unit Gaussians from two uniforms (Box and Muller, 1958)."""
    r = np.sqrt(-2.0 * np.log(ua))
    return r * np.cos(2.0 * np.pi * ub), r * np.sin(2.0 * np.pi * ub)


def _exp_inverse_cdf(u, lam):
    """Mass of the exponential shape exp(-lam (m - M_LO)) truncated to the range,
    by inverting its CDF at u (uniform on the range when lam = 0)."""
    L = Mo.M_HI - Mo.M_LO
    if lam == 0.0:
        return Mo.M_LO + L * u
    return Mo.M_LO - np.log1p(-u * (-np.expm1(-lam * L))) / lam


def _envelope_rate(G, DG):
    """Rate of the exponential proposal of the true decay time: the slowest of
    the two mass eigenstates, Gamma - |DeltaGamma|/2, so that e^{rate t} times
    the unconvolved density stays bounded for every t >= 0."""
    return G - abs(DG) / 2.0


def _angles(ua, ub, uc):
    """cos(theta_K), cos(theta_l) uniform on [-1, 1] and phi uniform on [-pi, pi]."""
    return 2.0 * ua - 1.0, 2.0 * ub - 1.0, np.pi * (2.0 * uc - 1.0)


def candidates(model, theta, u, bound):
    """Accept flags, output columns, ratio/bound margins and violation flags."""
    if model == 1:
        m = Mo.M_LO + (Mo.M_HI - Mo.M_LO) * u[:, 0]
        R = Mo.pdf_mass(m, *theta)
        lhs = u[:, 1] * bound
        return lhs < R, [m], None, (R - lhs) / R, R > bound
    if model == 2:
        f, mu, sig_m, lam, tau_s, tau_b, s = theta
        st = 0.03 + 0.03 * u[:, 0]
        sig = u[:, 1] < f
        g1, g2 = _box_muller(u[:, 2], u[:, 3])
        mb = _exp_inverse_cdf(u[:, 4], lam)
        m = np.where(sig, mu + sig_m * g1, mb)
        t = -np.where(sig, tau_s, tau_b) * np.log(u[:, 5]) + s * st * g2
        inr = (m >= Mo.M_LO) & (m <= Mo.M_HI) & (t >= Mo.T_LO) & (t <= Mo.T_HI)
        rs, rb = _masstime_ratios(theta, s * st)
        R = np.where(sig, rs, rb)
        lhs = u[:, 6] * bound
        return inr & (lhs < R), [m, t, st], None, (R - lhs) / R, R > bound
    fL, fpe, Fs, dpa, dpe, dS, G, DG, DM, phis, mu_m, sig_m = theta
    st = 0.03 + 0.03 * u[:, 0]
    gmin = _envelope_rate(G, DG)
    t0 = -np.log(u[:, 1]) / gmin
    ck, cl, ph = _angles(u[:, 2], u[:, 3], u[:, 4])
    C = Mo.time_coefficients(fL, fpe, Fs, dpa, dpe, dS, phis)
    fk = Mo.angular_functions(ck, cl, ph)
    e = np.exp((gmin - G) * t0)
    h = [e * np.cosh(DG * t0 / 2.0), e * np.sinh(DG * t0 / 2.0), e * np.cos(DM * t0), e * np.sin(DM * t0)]
    R = sum(fk[k] * sum(C[k][j] * h[j] for j in range(4)) for k in range(10))
    lhs = u[:, 5] * bound
    g1, g2 = _box_muller(u[:, 6], u[:, 7])
    t = t0 + st * g1
    m = mu_m + sig_m * g2
    inr = (t >= Mo.T_LO) & (t <= Mo.T_HI) & (m >= Mo.M_LO) & (m <= Mo.M_HI)
    w = 0.8 + 0.2 * u[:, 8]
    return inr & (lhs < R), [ck, cl, ph, t, st, m], w, (R - lhs) / np.abs(R), R > bound


def bound(model, theta):
    return {1: bound_mass, 2: bound_masstime, 3: bound_angtime}[model](theta)


def generate(model, theta, seed, toy_id, n, max_candidates=None):
    """First n accepted events.  Returns dict with columns, weights (model 3),
    candidate indices, number of candidates examined (index of the n-th
    acceptance + 1), violations and the smallest relative margin |R - u M|/R
    over all examined candidates (near-ties would make the decision depend on
    the last bit)."""
    theta = [float(x) for x in theta]
    M = bound(model, theta)
    cols, ws, idx = [], [], []
    got = 0
    c0 = 0
    viol = 0
    margin = np.inf
    while got < n:
        if max_candidates is not None and c0 >= max_candidates:
            raise RuntimeError("candidate budget exhausted")
        u = uniforms(model, seed, toy_id, c0, CHUNK)
        acc, out, w, marg, v = candidates(model, theta, u, M)
        take = np.nonzero(acc)[0][: n - got]
        last = c0 + (take[-1] + 1 if got + take.size >= n else CHUNK)
        k = last - c0
        viol += int(np.sum(v[:k]))
        margin = min(margin, float(np.min(np.abs(marg[:k]))))
        cols.append([o[take] for o in out])
        if w is not None:
            ws.append(w[take])
        idx.append(c0 + take)
        got += take.size
        c0 += CHUNK
        if got >= n:
            c0 = last
    columns = [np.concatenate([c[i] for c in cols]) if cols else np.empty(0)
               for i in range(Mo.NCOLS[model])]
    return {"cols": columns, "w": np.concatenate(ws) if ws else (np.empty(0) if model == 3 else None),
            "index": np.concatenate(idx) if idx else np.empty(0, np.int64),
            "n_candidates": c0 if n > 0 else 0, "violations": viol, "bound": M, "min_margin": margin}
