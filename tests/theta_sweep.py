"""Parameter points of the parity sweep: 20 random points inside each model's
limits plus fixed edge points that reach the special branches (lambda = 0
exactly, the small-|lambda| series of the exponential normalisation,
DeltaGamma < 0 and = 0, Fs at and next to 0, fL + fperp next to 1, Delta m far
from its generated value, fractions at their limits).

Parameter draws only: nothing here evaluates the likelihood.
"""
import numpy as np

N_RANDOM = 20
SEED = 1706_01420

THETA_GEN = {
    1: (0.3, 5367.0, 15.0, 0.002),
    2: (0.3, 5367.0, 15.0, 0.002, 1.5, 0.7, 1.0),
    3: (0.52, 0.25, 0.05, 3.26, 3.08, 0.35, 0.66, 0.08, 17.8, -0.03, 5367.0, 15.0),
}


def _random(model, rng):
    u = rng.uniform
    if model == 1:
        return [u(0.05, 0.95), u(5250.0, 5450.0), u(8.0, 40.0), u(-0.01, 0.01)]
    if model == 2:
        return [u(0.05, 0.95), u(5250.0, 5450.0), u(8.0, 40.0), u(-0.01, 0.01),
                u(0.4, 3.0), u(0.2, 2.0), u(0.6, 1.8)]
    while True:
        fL, fpe = u(0.25, 0.7), u(0.1, 0.35)
        if fL + fpe <= 0.95:
            break
    g = u(0.45, 0.9)
    return [fL, fpe, u(0.01, 0.5), u(-np.pi, np.pi), u(-np.pi, np.pi), u(-np.pi, np.pi),
            g, u(-0.25, 0.25), u(1.0, 25.0), u(-np.pi, np.pi), u(5330.0, 5400.0), u(8.0, 25.0)]


def _with(model, **kw):
    names = {1: ("f", "mu", "sigma", "lam"),
             2: ("f", "mu", "sigma", "lam", "tau_s", "tau_b", "s"),
             3: ("fL", "fpe", "Fs", "dpa", "dpe", "dS", "G", "DG", "DM", "phis", "mu", "sigma")}[model]
    th = list(THETA_GEN[model])
    for k, v in kw.items():
        th[names.index(k)] = v
    return th


# (label, theta, gradient defined there)
EDGES = {
    1: [("lambda=0", _with(1, lam=0.0), True),
        ("lambda=3e-6 (series)", _with(1, lam=3e-6), True),
        ("lambda=-3e-6 (series)", _with(1, lam=-3e-6), True),
        ("lambda<0", _with(1, lam=-0.01), True),
        ("f=0", _with(1, f=0.0), True),
        ("f=1", _with(1, f=1.0), True)],
    2: [("lambda=0", _with(2, lam=0.0), True),
        ("lambda=3e-6 (series)", _with(2, lam=3e-6), True),
        ("f=0", _with(2, f=0.0), True),
        ("f=1", _with(2, f=1.0), True),
        ("s=0.5", _with(2, s=0.5), True),
        ("tau_s=tau_b", _with(2, tau_s=0.9, tau_b=0.9), True)],
    3: [("Fs=0", _with(3, Fs=0.0), False),
        ("Fs=1e-10", _with(3, Fs=1e-10), True),
        ("fL+fperp=0.999", _with(3, fL=0.6, fpe=0.399), True),
        ("fL+fperp=1-1e-10", _with(3, fL=0.6, fpe=0.4 - 1e-10), True),
        ("DeltaGamma<0", _with(3, DG=-0.1), True),
        ("DeltaGamma=0", _with(3, DG=0.0), True),
        ("Delta m=0.5", _with(3, DM=0.5), True),
        ("Delta m=30", _with(3, DM=30.0), True),
        ("phis=0", _with(3, phis=0.0), True)],
}


def points(model):
    """[(label, theta, grad_defined)]: the random points then the edges."""
    rng = np.random.default_rng(SEED + model)
    out = [("random %d" % i, _random(model, rng), True) for i in range(N_RANDOM)]
    return out + EDGES[model]
