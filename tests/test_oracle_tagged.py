"""Pins of the oracle's tagged angular model (model 4), its efficiency weights,
the S-P factor per KK-mass bin and the simultaneous categories (paper
Example 2: categories per KK-mass bin and flavour, each normalised on its own).

  * flavour: qd = -1 is the anti-B_s PDF, proportional at every (Omega, t) to
    the squared helicity amplitudes of an anti-B_s evolved with mixing
    (an independent construction from |Bbar(t)>);
  * dilution: qd = 1 - 2 omega is the normalised mixture (1 - omega) |A|^2 +
    omega |Abar|^2 of the two flavours' squared amplitudes;
  * every qd integrates to 1 over (Omega, t);
  * efficiency weights: with xi_k = integral eps f_k (by quadrature), eps x P
    integrates to 1;
  * C_SP: the table equals the helicity density with the S-P interference
    scaled by c_sp;
  * simultaneous fit: one bin equals the single-category NLL; the gradient
    matches central differences and lands on the right parameters.
"""
import math

import numpy as np
import pytest

import pins
from oracle import models as M
from oracle import nll as N
from oracle import sim as S

THETAS = [M.THETA_GEN[3],
          (0.45, 0.3, 0.2, 2.5, 0.4, -1.0, 0.7, 0.12, 17.0, 0.4, 5370.0, 12.0),
          (0.6, 0.1, 0.1, 3.0, 3.0, 0.5, 0.6, -0.05, 18.5, -0.7, 5360.0, 18.0)]
SIG0 = 1e-8      # resolution so small that the convolved terms are the bare exponentials


def _points(n=300, seed=11):
    rng = np.random.default_rng(seed)
    return (rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(-np.pi, np.pi, n),
            rng.uniform(M.T_LO, 6.0, n))


def _pdf4(theta, ck, cl, ph, t, qd, sig=SIG0, settings=None):
    n = ck.size
    m = np.full(n, theta[10])
    return M.pdf(4, [ck, cl, ph, t, np.full(n, sig), m, np.broadcast_to(qd, (n,)).astype(float)], theta, settings)


def _amps(theta, t, bar):
    fL, fpe, Fs, dpa, dpe, dS, G, DG, DM, phis, _, _ = theta
    f = pins.mixing_amplitudes_bar if bar else pins.mixing_amplitudes
    return f(fL, fpe, Fs, dpa, dpe, dS, G, DG, DM, phis, M.LAMBDA_ABS, t)


def _dens(A, ck, cl, ph):
    return pins.helicity_density(A["0"], A["pa"], A["pe"], A["S"], ck, cl, ph)


@pytest.mark.parametrize("theta", THETAS)
@pytest.mark.parametrize("qd", [1.0, -1.0, 0.0, 0.46, -0.8])
def test_tagged_pdf_is_the_flavour_mixture(theta, qd):
    """P(qd) / [(1 - omega)|A|^2 + omega |Abar|^2] is one constant over
    (Omega, t), omega = (1 - qd)/2 (qd = +1: B_s, -1: anti-B_s)."""
    ck, cl, ph, t = _points()
    om = (1.0 - qd) / 2.0
    ref = (1.0 - om) * _dens(_amps(theta, t, False), ck, cl, ph) + om * _dens(_amps(theta, t, True), ck, cl, ph)
    r = _pdf4(theta, ck, cl, ph, t, qd) / ref
    assert np.max(np.abs(r / r[0] - 1.0)) < 1e-12


def test_untagged_model_is_tag_plus_one():
    ck, cl, ph, t = _points(50)
    th = THETAS[1]
    sig = np.full(ck.size, 0.04)
    m = np.full(ck.size, 5360.0)
    a = M.pdf(3, [ck, cl, ph, t, sig, m], th)
    b = M.pdf(4, [ck, cl, ph, t, sig, m, np.ones(ck.size)], th)
    assert np.array_equal(a, b)


def _integral_ot(theta, sigma_t, qd, settings=None, eps=None):
    ck, cl, ph, wa = pins.angular_grid(8, 16) if eps is not None else pins.angular_grid(4, 6)
    t, wt = pins.gl_composite(M.T_LO, M.T_HI, 60, 12)
    A = np.repeat(np.arange(ck.size), t.size)
    Tt = np.tile(t, ck.size)
    n = Tt.size
    cols = [ck[A], cl[A], ph[A], Tt, np.full(n, sigma_t), np.full(n, theta[10]), np.full(n, qd)]
    p = M.pdf(4, cols, theta, settings)
    if eps is not None:
        p = p * eps(ck[A], cl[A], ph[A])
    m, wm = pins.gl_composite(M.M_LO, M.M_HI, 10, 16)
    g = np.exp(-(m - theta[10]) ** 2 / (2 * theta[11] ** 2))
    # the mass factor at m0 = mu has unnormalised value 1: multiply its integral back
    return np.sum(wa[A] * np.tile(wt, ck.size) * p) * np.sum(wm * g)


@pytest.mark.parametrize("theta", THETAS)
@pytest.mark.parametrize("qd", [1.0, -1.0, -0.35, 0.6])
def test_tagged_pdf_integrates_to_one(theta, qd):
    assert abs(_integral_ot(theta, 0.045, qd) - 1.0) < 1e-11


def _xi(eps):
    ck, cl, ph, w = pins.angular_grid(8, 16)
    e = eps(ck, cl, ph)
    return np.array([np.sum(w * e * f) for f in M.angular_functions(ck, cl, ph)])


@pytest.mark.parametrize("theta", THETAS)
@pytest.mark.parametrize("qd", [1.0, -0.5])
def test_efficiency_weights_normalise_against_the_efficiency(theta, qd):
    """With xi_k = integral eps f_k, the PDF is normalised against eps:
    integral eps(Omega) P dOmega dt = 1 (and not with the flat weights)."""
    xi = _xi(pins.acceptance)
    assert not np.allclose(xi, M.ANGULAR_INTEGRALS)
    got = _integral_ot(theta, 0.05, qd, {"xi": xi}, pins.acceptance)
    assert abs(got - 1.0) < 1e-11
    flat = _integral_ot(theta, 0.05, qd, None, pins.acceptance)
    assert abs(flat - 1.0) > 1e-4


@pytest.mark.parametrize("theta", THETAS)
@pytest.mark.parametrize("c_sp", [1.0, 0.83, 0.35])
def test_csp_scales_the_s_p_interference(theta, c_sp):
    ck, cl, ph, t = _points(200, seed=4)
    A = _amps(theta, t, False)
    ref = pins.helicity_density_csp(A["0"], A["pa"], A["pe"], A["S"], ck, cl, ph, c_sp)
    r = _pdf4(theta, ck, cl, ph, t, 1.0, settings={"c_sp": c_sp}) / ref
    assert np.max(np.abs(r / r[0] - 1.0)) < 1e-12


def _category(model, n, seed, qd_kind):
    from paper_1706_01420_amd import workloads as W
    cols, w = W.events(3, n, seed=seed)
    if model == 4:
        rng = np.random.default_rng(seed + 1)
        q = np.where(rng.uniform(size=n) < 0.5, 1.0, -1.0) if qd_kind == "mixed" else np.full(n, qd_kind)
        om = rng.uniform(0.0, 0.45, n)
        cols = list(cols) + [q * (1.0 - 2.0 * om)]
    return cols, w


def _sim_theta(nbins, seed=0):
    rng = np.random.default_rng(seed)
    g = M.THETA_GEN[3]
    shared = [g[0], g[1], g[3], g[4], g[6], g[7], g[8], g[9], g[10], g[11]]
    per = []
    for b in range(nbins):
        per += [0.03 + 0.04 * rng.uniform(), 0.2 + 0.5 * rng.uniform()]
    return np.array(shared + per)


def test_sim_one_bin_is_the_single_category():
    cols, w = _category(4, 700, 5, "mixed")
    th = _sim_theta(1)
    cats = [(4, cols, w, 0, {"c_sp": 0.9})]
    ref = N.nll(4, cols, S.category_theta(th, 0), w, {"c_sp": 0.9})
    assert S.nll(cats, th) == ref
    assert S.category_theta(th, 0) == [th[0], th[1], th[10], th[2], th[3], th[11]] + list(th[4:10])


def test_sim_gradient_matches_central_differences():
    nb = 2
    cats = []
    for b in range(nb):
        for q, seed in ((1.0, 20 + 2 * b), (-1.0, 21 + 2 * b)):
            cols, w = _category(4, 300, seed, q)
            cats.append((4, cols, w, b, {"c_sp": 0.8 - 0.2 * b}))
    th = _sim_theta(nb, seed=3)
    f, g = S.nll_grad(cats, th)
    assert math.isclose(f, S.nll(cats, th), rel_tol=1e-14)
    for i in range(th.size):
        h = 1e-5 * max(1.0, abs(th[i]))
        vals = []
        for k in (-2, -1, 1, 2):
            tt = th.copy()
            tt[i] += k * h
            vals.append(S.nll(cats, tt))
        fd = (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h)
        assert abs(g[i] - fd) <= 1e-6 * max(1.0, abs(fd)), (i, g[i], fd)


def test_sim_bin_parameters_touch_only_their_bin():
    cols, w = _category(4, 200, 9, 1.0)
    th = _sim_theta(3, seed=1)
    _, g = S.nll_grad([(4, cols, w, 1, None)], th)
    s = len(S.SIM_SHARED)
    assert np.all(g[[s, s + 1, s + 4, s + 5]] == 0.0)
    assert np.all(g[[s + 2, s + 3]] != 0.0)
