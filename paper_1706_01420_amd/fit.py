"""Gradient-based minimisation of many likelihoods in lockstep.

The paper fits with Minuit (MIGRAD, then HESSE for errors).  Here a BFGS
quasi-Newton minimiser with an Armijo backtracking line search plays MIGRAD's
role (stopping on the estimated distance to minimum, EDM = g^T H g / 2, as
MIGRAD does), and errors come from the inverse of the Hessian built by central
differences of the analytic gradient (HESSE's role).

`bfgs` drives nb independent problems together: every round asks the
evaluator for one (NLL, gradient) per still-running problem, at that problem's
own trial point.  The per-problem arithmetic does not depend on nb, so fitting
toys one at a time (nb = 1 per call, the plain loop) or all together through
one batched evaluation per round gives the same points, hence (with bitwise
reproducible evaluations) the same minima.
"""
import numpy as np


def fd_hessian(evaluate, theta, steps, active=None):
    """Central-difference Hessian of the gradient at theta (nb, np):
    2 np batched evaluations.  Returns (nb, np, np), symmetrised."""
    nb, npar = theta.shape
    act = np.ones(nb, bool) if active is None else np.asarray(active, bool)
    H = np.full((nb, npar, npar), np.nan)
    for i in range(npar):
        tp, tm = theta.copy(), theta.copy()
        tp[:, i] += steps[:, i]
        tm[:, i] -= steps[:, i]
        _, gp = evaluate(tp, act)
        _, gm = evaluate(tm, act)
        H[:, i, :] = (gp - gm) / (2.0 * steps[:, i:i + 1])
    return 0.5 * (H + np.transpose(H, (0, 2, 1)))


def _positive_definite(H):
    """Cholesky succeeds: H (symmetric, finite) is positive definite."""
    try:
        np.linalg.cholesky(H)
        return True
    except np.linalg.LinAlgError:
        return False


def _inverse_or_diag(H, fallback):
    """Inverses of the stacked (nb, np, np) H where positive definite, else
    diag(fallback^2) per problem.  The stacked LAPACK calls work matrix by
    matrix, and a stack that fails the test as a whole is decided matrix by
    matrix, so each problem's result does not depend on nb."""
    nb, npar, _ = H.shape
    out = np.empty_like(H)
    good = np.zeros(nb, bool)
    cand = np.nonzero(np.all(np.isfinite(H), axis=(1, 2)))[0]
    if cand.size and not _positive_definite(H[cand]):
        cand = np.array([j for j in cand if _positive_definite(H[j])], dtype=np.int64)
    if cand.size:
        out[cand] = np.linalg.inv(H[cand])
        good[cand] = True
    for j in np.nonzero(~good)[0]:
        out[j] = np.diag(fallback[j] ** 2)
    return out


def bfgs(evaluate, theta0, steps, edm_tol=1e-6, max_rounds=400, c1=1e-4, init_hessian=True):
    """Minimise nb problems.

    evaluate(theta (nb, np), active (nb,) bool) -> (f (nb,), g (nb, np)); rows
    of inactive problems are ignored.  steps: (nb, np) or (np,) typical
    parameter scales (finite-difference steps and the fallback initial
    inverse Hessian diag(steps^2)).

    Returns dict: theta, f, grad, edm, converged (nb,), rounds, evals (nb,).
    """
    x = np.array(theta0, dtype=np.float64, copy=True)
    nb, npar = x.shape
    steps = np.broadcast_to(np.asarray(steps, np.float64), (nb, npar)).copy()
    evals = np.zeros(nb, np.int64)
    everyone = np.ones(nb, bool)
    f, g = evaluate(x, everyone)
    evals += 1
    if init_hessian:
        H = fd_hessian(evaluate, x, steps, everyone)
        evals += 2 * npar
        Hinv = _inverse_or_diag(H, steps)
    else:
        Hinv = steps[:, :, None] ** 2 * np.eye(npar)
    converged = np.zeros(nb, bool)
    failed = ~np.isfinite(f)
    edm = 0.5 * np.einsum("ni,nij,nj->n", g, Hinv, g)
    converged |= edm < edm_tol
    p = -np.einsum("nij,nj->ni", Hinv, g)
    alpha = np.ones(nb)
    rounds = 0
    while rounds < max_rounds:
        run = ~converged & ~failed
        if not run.any():
            break
        rounds += 1
        trial = x + alpha[:, None] * p
        ft, gt = evaluate(np.where(run[:, None], trial, x), run)
        evals += run
        slope = np.einsum("ni,ni->n", g, p)
        ok = run & np.isfinite(ft) & (ft <= f + c1 * alpha * slope)
        bad = run & ~ok
        # rejected: halve the step; give up after many halvings
        alpha[bad] *= 0.5
        failed |= bad & (alpha < 1e-12)
        # accepted: BFGS update of the inverse Hessian, all such problems at
        # once (row-wise arithmetic, independent of how many there are)
        acc = np.nonzero(ok)[0]
        if acc.size:
            s = trial[acc] - x[acc]
            y = gt[acc] - g[acc]
            sy = np.einsum("ni,ni->n", s, y)
            upd = sy > 1e-300
            if upd.any():
                u = acc[upd]
                su, yu = s[upd], y[upd]
                rho = (1.0 / sy[upd])[:, None, None]
                V = np.eye(npar) - rho * (su[:, :, None] * yu[:, None, :])
                Hinv[u] = V @ Hinv[u] @ np.transpose(V, (0, 2, 1)) + rho * (su[:, :, None] * su[:, None, :])
            x[acc], f[acc], g[acc] = trial[acc], ft[acc], gt[acc]
            edm[acc] = 0.5 * np.einsum("ni,nij,nj->n", g[acc], Hinv[acc], g[acc])
            done = edm[acc] < edm_tol
            converged[acc[done]] = True
            go = acc[~done]
            p[go] = -np.einsum("nij,nj->ni", Hinv[go], g[go])
            alpha[go] = 1.0
    return {"theta": x, "f": f, "grad": g, "edm": edm, "converged": converged, "failed": failed,
            "rounds": rounds, "evals": evals}


def restrict(evaluate, theta_fixed, free):
    """Evaluator over the free parameters only: the others stay at
    theta_fixed (nb, np); free is a boolean mask over the np parameters."""
    theta_fixed = np.asarray(theta_fixed, np.float64)
    free = np.asarray(free, bool)

    def sub(theta, active):
        full = theta_fixed.copy()
        full[:, free] = theta
        f, g = evaluate(full, active)
        return f, g[:, free]
    return sub


def errors(evaluate, theta, steps):
    """Parabolic errors: sqrt of the diagonal of the inverse FD Hessian."""
    nb, npar = theta.shape
    steps = np.broadcast_to(np.asarray(steps, np.float64), (nb, npar))
    H = fd_hessian(evaluate, theta, steps)
    err = np.full((nb, npar), np.nan)
    for j in range(nb):
        try:
            cov = np.linalg.inv(H[j])
            d = np.diag(cov)
            if np.all(d > 0):
                err[j] = np.sqrt(d)
        except np.linalg.LinAlgError:
            pass
    return err
