"""Independent references that pin the oracle (no code shared with it).

Each helper computes a quantity the mathematics fixes, by a route that does not
go through the oracle's formula for it:
  * mpmath at 40 digits for the closed-form resolution convolution;
  * adaptive quadrature of the convolution integral itself;
  * Gauss-Legendre / uniform periodic grids for normalisation integrals;
  * the squared sum of helicity amplitudes with B_s mixing for the angular x
    time table.
"""
import mpmath as mp
import numpy as np
from numpy.polynomial.legendre import leggauss
from scipy import integrate

mp.mp.dps = 40


# ---------------------------------------------------------------------------
# Resolution-convolved exponential
# ---------------------------------------------------------------------------
def conv_exp_mpmath(t, z, sigma):
    """1/2 exp(z^2 s^2/2 - z t) erfc((z s^2 - t)/(sqrt2 s)) in 40-digit arithmetic."""
    t, s = mp.mpf(t), mp.mpf(sigma)
    z = mp.mpc(complex(z))
    v = 0.5 * mp.exp(z * z * s * s / 2 - z * t) * mp.erfc((z * s * s - t) / (mp.sqrt(2) * s))
    return complex(v)


def conv_exp_quad(t, z, sigma):
    """integral_0^inf e^{-z tau} N(t - tau; 0, sigma) d tau by adaptive quadrature."""
    z = complex(z)
    lo = max(0.0, t - 16.0 * sigma)
    hi = max(lo, t + 16.0 * sigma)
    norm = 1.0 / (np.sqrt(2.0 * np.pi) * sigma)

    def re(tau):
        return (np.exp(-z * tau) * norm * np.exp(-(t - tau) ** 2 / (2 * sigma * sigma))).real

    def im(tau):
        return (np.exp(-z * tau) * norm * np.exp(-(t - tau) ** 2 / (2 * sigma * sigma))).imag

    kw = dict(epsabs=0.0, epsrel=1e-13, limit=400, points=[min(max(t, lo), hi)])
    r = integrate.quad(re, lo, hi, **kw)[0]
    i = integrate.quad(im, lo, hi, **kw)[0]
    return complex(r, i)


# ---------------------------------------------------------------------------
# Quadrature grids
# ---------------------------------------------------------------------------
def gl_composite(a, b, panels, order):
    x, w = leggauss(order)
    edges = np.linspace(a, b, panels + 1)
    xs, ws = [], []
    for lo, hi in zip(edges[:-1], edges[1:]):
        xs.append(0.5 * (hi - lo) * x + 0.5 * (hi + lo))
        ws.append(0.5 * (hi - lo) * w)
    return np.concatenate(xs), np.concatenate(ws)


def angular_grid(n_cos=8, n_phi=16):
    """Tensor grid exact for the polynomial-in-cos and trigonometric-in-phi
    angular integrands used here."""
    c, wc = leggauss(n_cos)
    ph = -np.pi + (np.arange(n_phi) + 0.5) * (2 * np.pi / n_phi)
    wph = np.full(n_phi, 2 * np.pi / n_phi)
    CK, CL, PH = np.meshgrid(c, c, ph, indexing="ij")
    W = wc[:, None, None] * wc[None, :, None] * wph[None, None, :]
    return CK.ravel(), CL.ravel(), PH.ravel(), W.ravel()


# ---------------------------------------------------------------------------
# Helicity amplitudes with B_s mixing
# ---------------------------------------------------------------------------
def wigner_d1(j, m, c):
    s = np.sqrt(1.0 - c * c)
    r2 = np.sqrt(2.0)
    table = {(1, 1): (1 + c) / 2, (1, 0): -s / r2, (1, -1): (1 - c) / 2,
             (0, 1): s / r2, (0, 0): c, (0, -1): -s / r2,
             (-1, 1): (1 - c) / 2, (-1, 0): s / r2, (-1, -1): (1 + c) / 2}
    return table[(j, m)]


def helicity_density(A0, Apa, Ape, AS, cos_k, cos_l, phi):
    """sum over muon helicity difference D = +-1 of
    |sum_l H_l d1_{l,0}(theta_K) d1_{l,D}(theta_l) e^{i l phi} + A_S d1_{0,D}(theta_l)/sqrt3|^2,
    H_0 = A_0, H_+- = (A_par +- A_perp)/sqrt2."""
    H = {1: (Apa + Ape) / np.sqrt(2.0), 0: A0, -1: (Apa - Ape) / np.sqrt(2.0)}
    tot = 0.0
    for Dh in (1, -1):
        amp = sum(H[l] * wigner_d1(l, 0, cos_k) * wigner_d1(l, Dh, cos_l) * np.exp(1j * l * phi)
                  for l in (1, 0, -1))
        amp = amp + AS * wigner_d1(0, Dh, cos_l) / np.sqrt(3.0)
        tot = tot + np.abs(amp) ** 2
    return tot


def mixing_amplitudes(fL, fpe, Fs, dpa, dpe, dS, G, DG, DM, phis, lam_abs, t, delta0=0.0):
    """A_i(t) = A_i [g+(t) + eta_i lambda g-(t)] for a B_s at t = 0, with
    eta = (+1, +1, -1, -1) for (0, par, perp, S), lambda = |lambda| e^{-i phis},
    heavy state (mass +DM/2, width G - DG/2), light (-DM/2, G + DG/2)."""
    a = {"0": np.sqrt((1 - Fs) * fL) * np.exp(1j * delta0),
         "pa": np.sqrt((1 - Fs) * (1 - fL - fpe)) * np.exp(1j * dpa),
         "pe": np.sqrt((1 - Fs) * fpe) * np.exp(1j * dpe),
         "S": np.sqrt(Fs) * np.exp(1j * dS)}
    eta = {"0": 1.0, "pa": 1.0, "pe": -1.0, "S": -1.0}
    lam = lam_abs * np.exp(-1j * phis)
    eH = np.exp(-1j * (DM / 2) * t - (G - DG / 2) * t / 2)
    eL = np.exp(+1j * (DM / 2) * t - (G + DG / 2) * t / 2)
    gp, gm = (eL + eH) / 2, (eL - eH) / 2
    return {k: a[k] * (gp + eta[k] * lam * gm) for k in a}


def mixing_amplitudes_bar(fL, fpe, Fs, dpa, dpe, dS, G, DG, DM, phis, lam_abs, t, delta0=0.0):
    """The same amplitudes for an anti-B_s at t = 0:
    Abar_i(t) = A_i [eta_i lambda g+(t) + g-(t)] up to the common phase p/q
    (|p/q| = 1), from |Bbar(t)> = g+ |Bbar> + (p/q) g- |B> and
    Abar_f = (p/q) lambda_f A_f, lambda_f = eta_f lambda."""
    a = {"0": np.sqrt((1 - Fs) * fL) * np.exp(1j * delta0),
         "pa": np.sqrt((1 - Fs) * (1 - fL - fpe)) * np.exp(1j * dpa),
         "pe": np.sqrt((1 - Fs) * fpe) * np.exp(1j * dpe),
         "S": np.sqrt(Fs) * np.exp(1j * dS)}
    eta = {"0": 1.0, "pa": 1.0, "pe": -1.0, "S": -1.0}
    lam = lam_abs * np.exp(-1j * phis)
    eH = np.exp(-1j * (DM / 2) * t - (G - DG / 2) * t / 2)
    eL = np.exp(+1j * (DM / 2) * t - (G + DG / 2) * t / 2)
    gp, gm = (eL + eH) / 2, (eL - eH) / 2
    return {k: a[k] * (eta[k] * lam * gp + gm) for k in a}


def helicity_density_csp(A0, Apa, Ape, AS, cos_k, cos_l, phi, c_sp):
    """helicity_density with the S-P interference terms scaled by c_sp: the
    P-wave part, the S-wave part and c_sp times what the two add when summed
    coherently."""
    z = 0.0 * AS
    full = helicity_density(A0, Apa, Ape, AS, cos_k, cos_l, phi)
    p = helicity_density(A0, Apa, Ape, z, cos_k, cos_l, phi)
    s = helicity_density(z, z, z, AS, cos_k, cos_l, phi)
    return p + s + c_sp * (full - p - s)


def acceptance(cos_k, cos_l, phi):
    """A smooth, positive angular efficiency of the kind a detector imposes:
    polynomial in the cosines, trigonometric in phi (integrated exactly by
    angular_grid(8, 16))."""
    return (1.0 + 0.3 * cos_k ** 2 - 0.2 * cos_l + 0.15 * cos_l ** 2 * np.cos(2.0 * phi)
            - 0.1 * cos_k * np.sin(phi))
