"""The lockstep BFGS minimiser on problems with known minima (CPU)."""
import numpy as np

from paper_1706_01420_amd import fit


def quad_problem(nb, npar, seed):
    rng = np.random.default_rng(seed)
    A = []
    for _ in range(nb):
        Q = rng.standard_normal((npar, npar))
        A.append(Q @ Q.T + npar * np.eye(npar))
    A = np.array(A)
    xstar = rng.standard_normal((nb, npar))

    def evaluate(theta, active):
        d = theta - xstar
        f = 0.5 * np.einsum("ni,nij,nj->n", d, A, d)
        g = np.einsum("nij,nj->ni", A, d)
        return f, g
    return evaluate, A, xstar


def test_bfgs_finds_quadratic_minima_and_hessian_errors():
    ev, A, xstar = quad_problem(5, 6, 0)
    r = fit.bfgs(ev, np.zeros((5, 6)), 0.1)
    assert r["converged"].all()
    assert np.allclose(r["theta"], xstar, atol=1e-6)
    err = fit.errors(ev, r["theta"], 1e-3)
    ref = np.sqrt(np.array([np.diag(np.linalg.inv(a)) for a in A]))
    assert np.allclose(err, ref, rtol=1e-8)


def test_lockstep_equals_one_at_a_time():
    ev, A, xstar = quad_problem(4, 3, 1)
    x0 = np.ones((4, 3))
    rb = fit.bfgs(ev, x0, 0.2, init_hessian=False)
    for j in range(4):
        def ev1(theta, active, j=j):
            full = np.tile(theta, (4, 1))
            f, g = ev(full, np.ones(4, bool))
            return f[j:j + 1], g[j:j + 1]
        r1 = fit.bfgs(ev1, x0[j:j + 1], 0.2, init_hessian=False)
        assert np.array_equal(r1["theta"][0], rb["theta"][j])
        assert r1["evals"][0] == rb["evals"][j]


def test_rosenbrock_with_infinite_region():
    # NLL-like: +inf outside x0 > -1.5 (domain errors) must be backtracked over
    def ev(theta, active):
        x, y = theta[:, 0], theta[:, 1]
        f = (1 - x) ** 2 + 100 * (y - x * x) ** 2
        g = np.stack([-2 * (1 - x) - 400 * x * (y - x * x), 200 * (y - x * x)], axis=1)
        f = np.where(x > -1.5, f, np.inf)
        return f, g
    r = fit.bfgs(ev, np.array([[-1.2, 1.0]]), 0.1, edm_tol=1e-14, max_rounds=2000)
    assert r["converged"][0]
    assert np.allclose(r["theta"][0], [1.0, 1.0], atol=1e-5)


def test_restrict_holds_fixed_parameters():
    # conditional minimum of a quadratic with parameter 1 held at c:
    # x_free = x*_free - A_ff^{-1} A_f1 (c - x*_1)
    ev, A, xstar = quad_problem(3, 4, 2)
    c = 0.7
    free = np.array([True, False, True, True])
    fixed = np.zeros((3, 4))
    fixed[:, 1] = c
    r = fit.bfgs(fit.restrict(ev, fixed, free), np.zeros((3, 3)), 0.1)
    assert r["converged"].all()
    for j in range(3):
        Aff = A[j][np.ix_(free, free)]
        Af1 = A[j][free, 1]
        ref = xstar[j, free] - np.linalg.solve(Aff, Af1 * (c - xstar[j, 1]))
        assert np.allclose(r["theta"][j], ref, atol=1e-6)


def test_inverse_or_diag_same_for_stack_and_single():
    # half positive definite, half indefinite, one with a NaN: the stacked call
    # decides every problem as a call on that problem alone would
    rng = np.random.default_rng(3)
    nb, npar = 64, 6
    H = rng.standard_normal((nb, npar, npar))
    H = 0.5 * (H + np.transpose(H, (0, 2, 1)))
    H[:32] += 8 * np.eye(npar)
    H[5, 0, 0] = np.nan
    fb = np.full((nb, npar), 0.1)
    a = fit._inverse_or_diag(H, fb)
    b = np.array([fit._inverse_or_diag(H[j:j + 1], fb[j:j + 1])[0] for j in range(nb)])
    assert np.array_equal(a, b)
    for j in range(nb):
        if j < 32 and j != 5:
            assert np.allclose(a[j] @ H[j], np.eye(npar), atol=1e-10)
        else:
            assert np.array_equal(a[j], np.diag(fb[j] ** 2))
