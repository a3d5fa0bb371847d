"""Seeded synthetic event samples with the shapes of the three workloads.

Input generation only: draws from numpy distributions with the ranges, widths
and mixtures of the fits (no likelihood arithmetic).  Both the GPU path and the
CPU reference are fed from these arrays in tests and benchmarks.

    mass      m: 30 % Gaussian (5367, 15) + 70 % exponential (slope 0.002/MeV),
              both truncated to [5200, 5500] MeV
    masstime  the same m; per-event sigma_t ~ U(0.03, 0.06) ps; true decay time
              exponential with tau = 1.5 ps (Gaussian part) or 0.7 ps
              (exponential part), plus Gaussian noise of width sigma_t, kept in
              [0.3, 15] ps
    angtime   cos(theta_K), cos(theta_l) ~ U(-1, 1), phi ~ U(-pi, pi); t as
              above with tau = 1/0.66 ps; m Gaussian (5367, 15) truncated;
              weights ~ U(0.8, 1.0)
    ipatia    the mass sample (a peaked signal on the exponential background)
    tagged    the angtime columns plus qd = q (1 - 2 omega): tag decision
              q = +1 / -1 with equal probability (or fixed), mistag
              probability omega ~ U(0.05, 0.45) (or fixed)
"""
import numpy as np

M_LO, M_HI = 5200.0, 5500.0
T_LO, T_HI = 0.3, 15.0

BENCH_SEED = 170601420
WORKLOAD_SIZES = {1: 100_000, 2: 2_000_000, 3: 4_000_000}


def _truncated_normal(rng, mu, sig, n, lo=M_LO, hi=M_HI):
    out = np.empty(0)
    while out.size < n:
        x = rng.normal(mu, sig, 2 * (n - out.size) + 16)
        out = np.concatenate([out, x[(x >= lo) & (x <= hi)]])
    return out[:n]


def _truncated_exponential(rng, slope, n, lo=M_LO, hi=M_HI):
    u = rng.random(n)
    L = hi - lo
    return lo - np.log1p(-u * (-np.expm1(-slope * L))) / slope


def _smeared_times(rng, tau, sigma_t):
    n = sigma_t.size
    out = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        t = rng.exponential(tau[todo]) + sigma_t[todo] * rng.standard_normal(todo.size)
        ok = (t >= T_LO) & (t <= T_HI)
        out[todo[ok]] = t[ok]
        todo = todo[~ok]
    return out


def mass_events(n, seed=BENCH_SEED + 1):
    rng = np.random.default_rng(seed)
    sig = rng.random(n) < 0.3
    m = np.empty(n)
    m[sig] = _truncated_normal(rng, 5367.0, 15.0, int(sig.sum()))
    m[~sig] = _truncated_exponential(rng, 0.002, int((~sig).sum()))
    return [m], None


def masstime_events(n, seed=BENCH_SEED + 2):
    rng = np.random.default_rng(seed)
    sig = rng.random(n) < 0.3
    m = np.empty(n)
    m[sig] = _truncated_normal(rng, 5367.0, 15.0, int(sig.sum()))
    m[~sig] = _truncated_exponential(rng, 0.002, int((~sig).sum()))
    st = rng.uniform(0.03, 0.06, n)
    t = _smeared_times(rng, np.where(sig, 1.5, 0.7), st)
    return [m, t, st], None


def angtime_events(n, seed=BENCH_SEED + 3, weights=True):
    rng = np.random.default_rng(seed)
    ck = rng.uniform(-1.0, 1.0, n)
    cl = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(-np.pi, np.pi, n)
    st = rng.uniform(0.03, 0.06, n)
    t = _smeared_times(rng, np.full(n, 1.0 / 0.66), st)
    m = _truncated_normal(rng, 5367.0, 15.0, n)
    w = rng.uniform(0.8, 1.0, n) if weights else None
    return [ck, cl, ph, t, st, m], w


def tagged_events(n, seed=BENCH_SEED + 4, weights=True, q=None, omega=None):
    cols, w = angtime_events(n, seed=seed, weights=weights)
    rng = np.random.default_rng(seed + 1000003)
    qq = np.where(rng.random(n) < 0.5, 1.0, -1.0) if q is None else np.full(n, float(q))
    om = rng.uniform(0.05, 0.45, n) if omega is None else np.full(n, float(omega))
    return cols + [qq * (1.0 - 2.0 * om)], w


def events(model, n, seed=None, **kw):
    fn = {1: mass_events, 2: masstime_events, 3: angtime_events, 4: tagged_events, 5: mass_events}[model]
    return fn(n, **kw) if seed is None else fn(n, seed=seed, **kw)


# Generation points of the three workloads (parameter order of include/ipx.h).
THETA_GEN = {
    1: (0.3, 5367.0, 15.0, 0.002),
    2: (0.3, 5367.0, 15.0, 0.002, 1.5, 0.7, 1.0),
    3: (0.52, 0.25, 0.05, 3.26, 3.08, 0.35, 0.66, 0.08, 17.8, -0.03, 5367.0, 15.0),
}
THETA_GEN[4] = THETA_GEN[3]
# the Ipatia model: f, mu, sigma, lambda, zeta, beta, a, n, a2, n2, k
THETA_GEN[5] = (0.3, 5367.0, 15.0, -2.5, 0.01, 0.0, 2.0, 2.5, 2.5, 3.0, 0.002)
