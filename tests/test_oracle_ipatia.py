"""Pins of the oracle's Ipatia shape and Example 1 model (oracle/ipatia.py):

  * K_nu: scipy's kv against mpmath's besselk (30 digits);
  * scale: at beta = 0 the core's variance is sigma^2 (the defining property
    of A^2), by adaptive quadrature over the real line;
  * lambda = 1: the core is the hyperbolic density exp(-zeta q) (K_{1/2} in
    closed form);
  * zeta -> 0: the core tends to the Student-like (1 + d^2/(A^2 sigma^2))^{lambda - 1/2};
  * the analytic slope against central differences, and the tails continuous
    in value and slope at both junctions;
  * the grid normalisation against adaptive quadrature of the shape (the
    midpoint rule's error), and the model PDF integrating to 1 on the grid.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate
from scipy import special as sp

from oracle import ipatia as I

mp.mp.dps = 30
SHAPES = [(15.0, -2.5, 0.01, 0.0), (12.0, -1.6, 0.5, 0.002), (20.0, -3.2, 2.0, -0.004), (9.0, 1.0, 1.5, 0.0)]


@pytest.mark.parametrize("nu,x", [(0.3, 0.01), (-3.0, 0.02), (-1.7, 2.5), (2.2, 40.0), (-2.5, 7.3), (0.5, 1e-4)])
def test_kv_against_mpmath(nu, x):
    assert abs(sp.kv(nu, x) / float(mp.besselk(nu, x)) - 1.0) < 1e-14


@pytest.mark.parametrize("sigma,lam,zeta", [(15.0, -2.5, 0.01), (12.0, -1.6, 0.5), (20.0, -3.2, 2.0), (9.0, 1.0, 1.5),
                                            (10.0, -2.0, 0.0)])
def test_core_variance_is_sigma_squared(sigma, lam, zeta):
    def w(d):
        return float(I.core(np.array([d]), sigma, lam, zeta, 0.0)[0])
    kw = dict(limit=400, epsabs=0.0, epsrel=1e-12)
    z = integrate.quad(w, -np.inf, np.inf, **kw)[0]
    v = integrate.quad(lambda d: d * d * w(d), -np.inf, np.inf, **kw)[0]
    assert abs(v / z / sigma ** 2 - 1.0) < 1e-8


def test_lambda_one_is_the_hyperbolic_density():
    sigma, zeta, beta = 11.0, 1.3, 0.001
    d = np.linspace(-80, 80, 41)
    A2 = zeta * sp.kv(1.0, zeta) / sp.kv(2.0, zeta)
    q = np.sqrt(1 + d * d / (A2 * sigma * sigma))
    ref = np.exp(-zeta * q + beta * d)
    r = I.core(d, sigma, 1.0, zeta, beta) / ref
    assert np.max(np.abs(r / r[0] - 1)) < 1e-13


def test_small_zeta_limit():
    sigma, lam = 14.0, -2.3
    d = np.linspace(-90, 90, 31)
    A2 = -2 * (lam + 1)
    ref = (1 + d * d / (A2 * sigma * sigma)) ** (lam - 0.5)
    r = I.core(d, sigma, lam, 1e-9, 0.0) / ref
    assert np.max(np.abs(r / r[0] - 1)) < 1e-6
    r0 = I.core(d, sigma, lam, 0.0, 0.0) / ref
    assert np.max(np.abs(r0 / r0[0] - 1)) < 1e-14


@pytest.mark.parametrize("sigma,lam,zeta,beta", SHAPES)
def test_slope_and_tail_continuity(sigma, lam, zeta, beta):
    for d in (-3.0 * sigma, -0.7 * sigma, 0.4 * sigma, 2.2 * sigma):
        h = 1e-4 * sigma
        fd = (I.core(np.array([d + h]), sigma, lam, zeta, beta)[0] - I.core(np.array([d - h]), sigma, lam, zeta, beta)[0]) / (2 * h)
        assert abs(I.core_slope(d, sigma, lam, zeta, beta) / fd - 1) < 1e-7
    a, n, a2, n2 = 1.8, 2.2, 2.4, 3.5
    Al, Bl, Ar, Br = I.tails(sigma, lam, zeta, beta, a, n, a2, n2)
    left = lambda d: Al * (Bl - d) ** (-n)      # noqa: E731
    right = lambda d: Ar * (Br + d) ** (-n2)    # noqa: E731
    for dj, tail in ((-a * sigma, left), (a2 * sigma, right)):
        g = float(I.core(np.array([dj]), sigma, lam, zeta, beta)[0])
        assert abs(tail(dj) / g - 1) < 1e-13                       # value
        h = 1e-4 * sigma
        fd = (tail(dj + h) - tail(dj - h)) / (2 * h)
        assert abs(fd / I.core_slope(dj, sigma, lam, zeta, beta) - 1) < 1e-7   # slope
    # and the assembled shape takes the tails beyond the junctions
    assert I.ipatia(np.array([-a * sigma - 1.0]), sigma, lam, zeta, beta, a, n, a2, n2)[0] == left(-a * sigma - 1.0)
    assert I.ipatia(np.array([a2 * sigma + 1.0]), sigma, lam, zeta, beta, a, n, a2, n2)[0] == right(a2 * sigma + 1.0)


def test_grid_normalisation_and_unit_integral():
    th = list(I.THETA_GEN)
    f, mu, sigma, lam, zeta, beta, a, n, a2, n2, k = th
    NI = I.grid_norm(mu, sigma, lam, zeta, beta, a, n, a2, n2)

    def shape(m):
        return float(I.ipatia(np.array([m - mu]), sigma, lam, zeta, beta, a, n, a2, n2)[0])
    ref = integrate.quad(shape, I.M_LO, I.M_HI, points=[mu - a * sigma, mu, mu + a2 * sigma], limit=400,
                         epsabs=0.0, epsrel=1e-13)[0]
    assert abs(NI / ref - 1) < 1e-8            # midpoint rule, 16384 points
    dm = (I.M_HI - I.M_LO) / I.GRID
    mg = I.M_LO + (np.arange(I.GRID) + 0.5) * dm
    tot = math.fsum((I.pdf(mg, th) * dm).tolist())
    assert abs(tot - 1.0) < 1e-8


def test_domain():
    th = list(I.THETA_GEN)
    assert I.theta_valid(th)
    for i, v in ((0, 1.2), (2, -1.0), (4, -0.1), (6, 0.0), (9, -1.0)):
        t = list(th)
        t[i] = v
        assert not I.theta_valid(t)
    t = list(th)
    t[4], t[3] = 0.0, -0.5                    # zeta = 0 needs lambda < -1
    assert not I.theta_valid(t)
    t = list(th)
    t[5] = 0.5                                 # a steep asymmetry turns a tail's slope around
    assert not I.theta_valid(t)


# -- planted mistakes ------------------------------------------------------------
def _a2_inverted(lam, zeta):
    return zeta * sp.kv(lam + 1.0, zeta) / sp.kv(lam, zeta) if zeta > 0 else -2.0 * (lam + 1.0)


def _core_wrong_power(d, sigma, lam, zeta, beta):
    d = np.asarray(d, np.float64)
    a2s2 = I.a2_scale(lam, zeta) * sigma * sigma
    q = np.sqrt(1.0 + d * d / a2s2)
    if zeta == 0.0:
        return q ** (2.0 * lam - 1.0) * np.exp(beta * d)
    return q ** (lam + 0.5) * sp.kv(lam - 0.5, zeta * q) * np.exp(beta * d)


def _tails_wrong_sign(sigma, lam, zeta, beta, a, n, a2, n2):
    Al, Bl, Ar, Br = TAILS(sigma, lam, zeta, beta, a, n, a2, n2)
    dl = -a * sigma
    Bl2 = dl - (Bl - dl)                    # n G / G' with the wrong sign
    return Al * (Bl2 - dl) ** n / (Bl - dl) ** n, Bl2, Ar, Br


TAILS = I.tails


@pytest.mark.parametrize("attr,fake,check", [
    ("a2_scale", _a2_inverted, lambda: test_core_variance_is_sigma_squared(15.0, -2.5, 0.01)),
    ("core", _core_wrong_power, test_lambda_one_is_the_hyperbolic_density),
    ("tails", _tails_wrong_sign, lambda: test_slope_and_tail_continuity(*SHAPES[1])),
], ids=["A^2 ratio inverted", "core power", "tail slope sign"])
def test_planted_ipatia_mistake_is_caught(attr, fake, check, monkeypatch):
    monkeypatch.setattr(I, attr, fake)
    with pytest.raises(AssertionError):
        with np.errstate(all="ignore"):
            check()
