"""Pins of the oracle's special-function layer against independent references."""
import mpmath as mp
import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss

import pins
from oracle import dual as D
from oracle import models as M

# Complex decay constants that occur in the three models (Gamma - i Delta m, and
# real widths), plus a few outside the default workload.
Z_VALUES = [0.66 - 17.8j, 0.62 + 0j, 0.70 + 0j, 1 / 1.5 + 0j, 1 / 0.7 + 0j, 0.66 + 5.0j, 2.5 - 1.0j]
SIGMAS = [0.03, 0.045, 0.06, 0.25]
TIMES = [-0.1, 0.0, 0.01, 0.05, 0.3, 0.45, 1.0, 3.0, 14.99, 15.0]


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


@pytest.mark.parametrize("z", Z_VALUES)
@pytest.mark.parametrize("sigma", SIGMAS)
def test_conv_exp_matches_mpmath(z, sigma):
    got = M.conv_exp(np.array(TIMES), z, sigma)
    for t, g in zip(TIMES, got):
        ref = pins.conv_exp_mpmath(t, z, sigma)
        assert _rel(g, ref) < 1e-12, (t, z, sigma, g, ref)


@pytest.mark.parametrize("z", [0.66 - 17.8j, 0.62 + 0j, 1 / 0.7 + 0j])
@pytest.mark.parametrize("sigma", [0.03, 0.06])
def test_conv_exp_matches_numerical_convolution(z, sigma):
    ts = [0.0, 0.02, 0.3, 0.5, 2.0, 9.0]
    got = M.conv_exp(np.array(ts), z, sigma)
    for t, g in zip(ts, got):
        ref = pins.conv_exp_quad(t, z, sigma)
        # the convolution integral is smooth; quadrature reaches ~1e-13
        assert abs(g - ref) <= 1e-11 * abs(ref) + 1e-16, (t, z, sigma, g, ref)


def test_conv_exp_zero_resolution_limit():
    t = np.linspace(0.3, 15.0, 50)
    for z in Z_VALUES:
        got = M.conv_exp(t, z, 1e-5)
        assert np.allclose(got, np.exp(-z * t), rtol=1e-7, atol=0)


def test_conv_exp_integral_matches_quadrature():
    x, w = pins.gl_composite(M.T_LO, M.T_HI, 200, 20)
    for z in Z_VALUES:
        for sigma in SIGMAS:
            num = np.sum(w * M.conv_exp(x, z, sigma))
            got = M.conv_exp_integral(z, sigma)
            assert abs(got - num) < 1e-12 * abs(num), (z, sigma, got, num)


def test_gauss_cdf_matches_mpmath():
    for sigma in SIGMAS:
        for t in [-0.3, 0.0, 0.1, 0.3, 15.0]:
            ref = float(mp.ncdf(t, 0, sigma))
            assert _rel(M.gauss_cdf(t, sigma), ref) < 1e-14


@pytest.mark.parametrize("mu,sigma", [(5367.0, 15.0), (5250.0, 40.0), (5190.0, 12.0), (5490.0, 3.0)])
def test_gauss_norm_matches_mpmath_quad(mu, sigma):
    ref = mp.quad(lambda m: mp.exp(-(m - mu) ** 2 / (2 * mp.mpf(sigma) ** 2)),
                  [M.M_LO, mu, M.M_HI] if M.M_LO < mu < M.M_HI else [M.M_LO, M.M_HI])
    assert _rel(M.gauss_norm(mu, sigma), float(ref)) < 1e-13


@pytest.mark.parametrize("lam", [0.002, -0.004, 1e-9, 0.0, 0.05])
def test_exp_norm_matches_mpmath_quad(lam):
    ref = mp.quad(lambda m: mp.exp(-mp.mpf(lam) * (m - M.M_LO)), [M.M_LO, M.M_HI])
    assert _rel(M.exp_norm(lam), float(ref)) < 1e-14


def test_dual_derivatives_of_conv_exp_match_mpmath_diff():
    """d F/d Re z, d F/d Im z and dF/d sigma from the dual numbers vs 40-digit
    numerical differentiation of the mpmath closed form."""
    for z0 in [0.66 - 17.8j, 0.62 + 0j]:
        for s0 in [0.03, 0.06]:
            for t in [0.3, 0.4, 2.0]:
                zr, zi, s = D.seed([z0.real, z0.imag, s0])
                F = M.conv_exp(np.array([t]), zr + 1j * zi, s)
                for j, (name, fun) in enumerate([
                        ("re", lambda x: pins_mp(t, mp.mpc(x, z0.imag), s0)),
                        ("im", lambda x: pins_mp(t, mp.mpc(z0.real, x), s0)),
                        ("sigma", lambda x: pins_mp(t, mp.mpc(z0.real, z0.imag), x))]):
                    x0 = [z0.real, z0.imag, s0][j]
                    ref = complex(mp.diff(fun, mp.mpf(x0)))
                    got = complex(F.d[j][0])
                    assert abs(got - ref) <= 1e-11 * abs(ref) + 1e-14, (name, z0, s0, t, got, ref)


def pins_mp(t, z, s):
    t, s = mp.mpf(t), mp.mpf(s)
    return 0.5 * mp.exp(z * z * s * s / 2 - z * t) * mp.erfc((z * s * s - t) / (mp.sqrt(2) * s))


def test_gauss_legendre_grid_is_exact_for_polynomials():
    # the quadrature used by the normalisation pins integrates x^k exactly
    x, w = pins.gl_composite(-1.0, 1.0, 3, 8)
    for k in range(15):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 1e-14
    c, wc = leggauss(4)
    assert abs(np.sum(wc * c ** 6) - 2.0 / 7.0) < 1e-15
