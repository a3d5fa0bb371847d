"""Ipatia signal shape and the Example 1 mass model with a numerically
normalised signal (oracle test infrastructure).

Paper (Ipanema-beta, arXiv:1706.01420), Example 1: an Ipatia signal peak on
an exponential background, unbinned; the signal normalised numerically by
summing the shape over a fine grid of the mass range times the grid step,
the background analytically.  The Ipatia shape (Santos, Dupertuis, NIM A 764
(2014) 150) is not printed in the paper; it is taken here from its published
definition:

  core (generalised hyperbolic, scaled so that sigma is its standard
  deviation at beta = 0), d = m - mu:
      A^2 = zeta K_lambda(zeta) / K_{lambda+1}(zeta),
      q   = sqrt(1 + d^2 / (A^2 sigma^2)),
      G(d) = q^{lambda - 1/2} K_{lambda - 1/2}(zeta q) e^{beta d}      (zeta > 0)
      G(d) = q^{2 lambda - 1} e^{beta d},  A^2 = -2 (lambda + 1)        (zeta = 0, lambda < -1)
  (constant factors dropped: the normalisation removes them);
  tails, matching G and dG/dd at d = -a sigma and d = a2 sigma:
      d < -a sigma:  I = A_l (B_l - d)^{-n},   B_l = -a sigma + n G/G',   A_l = G (B_l + a sigma)^n
      d >  a2 sigma: I = A_r (B_r + d)^{-n2},  B_r = -a2 sigma - n2 G/G', A_r = G (B_r + a2 sigma)^{n2}
  with G, G' taken at the junction; otherwise I = G(d).

Model (parameters f, mu, sigma, lambda, zeta, beta, a, n, a2, n2, k; 11):
    P(m) = f I(m - mu) / N_I + (1 - f) e^{-k (m - 5200)} / N_E  on [5200, 5500] MeV,
    N_I = dm sum_g I(m_g - mu) over GRID midpoints m_g (step dm = 300 / GRID),
    N_E analytic (the k = 0 branch exact).
The modified Bessel function K_nu is scipy's ``kv`` (a library primitive,
pinned against mpmath).
"""
import math

import numpy as np
from scipy import special as sp

M_LO, M_HI = 5200.0, 5500.0
GRID = 1 << 14
NPARAMS = 11
PARAM_NAMES = ("f", "mu", "sigma", "lam", "zeta", "beta", "a", "n", "a2", "n2", "k")
THETA_GEN = (0.3, 5367.0, 15.0, -2.5, 0.01, 0.0, 2.0, 2.5, 2.5, 3.0, 0.002)


def a2_scale(lam, zeta):
    if zeta == 0.0:
        return -2.0 * (lam + 1.0)
    return zeta * sp.kv(lam, zeta) / sp.kv(lam + 1.0, zeta)


def core(d, sigma, lam, zeta, beta):
    d = np.asarray(d, np.float64)
    a2s2 = a2_scale(lam, zeta) * sigma * sigma
    q = np.sqrt(1.0 + d * d / a2s2)
    if zeta == 0.0:
        return q ** (2.0 * lam - 1.0) * np.exp(beta * d)
    nu = lam - 0.5
    return q ** nu * sp.kv(nu, zeta * q) * np.exp(beta * d)


def core_slope(d, sigma, lam, zeta, beta):
    """dG/dd: with d/dq [q^nu K_nu(zeta q)] = -zeta q^nu K_{nu-1}(zeta q) and
    dq/dd = d / (A^2 sigma^2 q)."""
    d = float(d)
    a2s2 = a2_scale(lam, zeta) * sigma * sigma
    q = math.sqrt(1.0 + d * d / a2s2)
    e = math.exp(beta * d)
    if zeta == 0.0:
        g = q ** (2.0 * lam - 1.0)
        return (2.0 * lam - 1.0) * q ** (2.0 * lam - 2.0) * (d / (a2s2 * q)) * e + beta * g * e
    nu = lam - 0.5
    g = q ** nu * sp.kv(nu, zeta * q)
    return -zeta * q ** nu * sp.kv(nu - 1.0, zeta * q) * (d / (a2s2 * q)) * e + beta * g * e


def tails(sigma, lam, zeta, beta, a, n, a2, n2):
    """(A_l, B_l, A_r, B_r) of the two power-law tails."""
    dl, dr = -a * sigma, a2 * sigma
    gl, sl = float(core(dl, sigma, lam, zeta, beta)), core_slope(dl, sigma, lam, zeta, beta)
    gr, sr = float(core(dr, sigma, lam, zeta, beta)), core_slope(dr, sigma, lam, zeta, beta)
    Bl = dl + n * gl / sl
    Br = -dr - n2 * gr / sr
    return gl * (Bl - dl) ** n, Bl, gr * (Br + dr) ** n2, Br


def ipatia(d, sigma, lam, zeta, beta, a, n, a2, n2):
    d = np.asarray(d, np.float64)
    Al, Bl, Ar, Br = tails(sigma, lam, zeta, beta, a, n, a2, n2)
    out = core(d, sigma, lam, zeta, beta)
    left, right = d < -a * sigma, d > a2 * sigma
    with np.errstate(invalid="ignore", divide="ignore"):
        out = np.where(left, Al * (Bl - d) ** (-n), out)
        out = np.where(right, Ar * (Br + d) ** (-n2), out)
    return out


def grid_norm(mu, sigma, lam, zeta, beta, a, n, a2, n2):
    dm = (M_HI - M_LO) / GRID
    mg = M_LO + (np.arange(GRID) + 0.5) * dm
    return dm * math.fsum(ipatia(mg - mu, sigma, lam, zeta, beta, a, n, a2, n2).tolist())


def exp_norm(k):
    L = M_HI - M_LO
    return L if k == 0.0 else -math.expm1(-k * L) / k


def theta_valid(theta):
    th = [float(x) for x in theta]
    if len(th) != NPARAMS or not all(np.isfinite(th)):
        return False
    f, mu, sigma, lam, zeta, beta, a, n, a2, n2, k = th
    if not (0.0 <= f <= 1.0 and sigma > 0.0 and zeta >= 0.0 and a > 0.0 and n > 0.0 and a2 > 0.0 and n2 > 0.0):
        return False
    if zeta == 0.0 and not lam < -1.0:
        return False
    # the tails must fall away from the core on both sides
    return (core_slope(-a * sigma, sigma, lam, zeta, beta) > 0.0 and
            core_slope(a2 * sigma, sigma, lam, zeta, beta) < 0.0)


def pdf(m, theta):
    f, mu, sigma, lam, zeta, beta, a, n, a2, n2, k = [float(x) for x in theta]
    m = np.asarray(m, np.float64)
    NI = grid_norm(mu, sigma, lam, zeta, beta, a, n, a2, n2)
    return (f * ipatia(m - mu, sigma, lam, zeta, beta, a, n, a2, n2) / NI +
            (1.0 - f) * np.exp(-k * (m - M_LO)) / exp_norm(k))


def nll(m, theta, w=None):
    if not theta_valid(theta):
        return math.inf
    lp = np.log(pdf(m, theta))
    if w is not None:
        lp = lp * np.asarray(w, np.float64)
    if not np.all(np.isfinite(lp)):
        return math.inf
    return -math.fsum(lp.tolist())
