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


def _inverse_or_diag(H, fallback):
    try:
        w = np.linalg.eigvalsh(H)
        if np.all(np.isfinite(w)) and w.min() > 0:
            return np.linalg.inv(H)
    except np.linalg.LinAlgError:
        pass
    return np.diag(fallback ** 2)


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
    Hinv = np.empty((nb, npar, npar))
    if init_hessian:
        H = fd_hessian(evaluate, x, steps, everyone)
        evals += 2 * npar
        for j in range(nb):
            Hinv[j] = _inverse_or_diag(H[j], steps[j])
    else:
        for j in range(nb):
            Hinv[j] = np.diag(steps[j] ** 2)
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
        for j in np.nonzero(ok)[0]:
            s = trial[j] - x[j]
            y = gt[j] - g[j]
            sy = s @ y
            if sy > 1e-300:
                rho = 1.0 / sy
                I = np.eye(npar)
                V = I - rho * np.outer(s, y)
                Hinv[j] = V @ Hinv[j] @ V.T + rho * np.outer(s, s)
            x[j], f[j], g[j] = trial[j], ft[j], gt[j]
            edm[j] = 0.5 * g[j] @ Hinv[j] @ g[j]
            if edm[j] < edm_tol:
                converged[j] = True
            else:
                p[j] = -Hinv[j] @ g[j]
                alpha[j] = 1.0
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
