"""Pseudo-experiment (toy) studies on top of libipx.

Sizes: as the paper suggests for Example 5, the number of events of each toy
is Poisson-fluctuated on the host: mean mu_j log-uniform in [1e4, 2e5], drawn
with numpy's Philox generator keyed by the study seed, then N_j ~ Poisson(mu_j).
Events: toy_generate_batch with key (seed, toy_id = j) for toy j.
Fits: fit.bfgs either through one nll_eval_batch per round (batched, graph
replay, launch schedule from the autotuner) or through nll_grad per toy (plain
loop); the per-toy arithmetic is the same, so both give the same minima.
"""
import numpy as np

from . import fit

# Typical parameter scales per model (finite-difference steps, fallback
# inverse-Hessian diagonal); roughly the statistical errors at 1e5 events.
STEPS = {
    1: np.array([3e-3, 0.2, 0.2, 1e-4]),
    2: np.array([3e-3, 0.2, 0.2, 1e-4, 5e-3, 2e-3, 5e-3]),
    3: np.array([3e-3, 3e-3, 3e-3, 3e-2, 3e-2, 3e-2, 2e-3, 5e-3, 3e-2, 3e-2, 0.1, 0.1]),
}


def toy_sizes(seed, ntoys, lo=1e4, hi=2e5):
    rng = np.random.Generator(np.random.Philox(key=seed))
    u = rng.random(ntoys)
    mu = 10.0 ** (np.log10(lo) + u * np.log10(hi / lo))
    return mu, rng.poisson(mu)


def generate(ipx, ctx, model, theta_gen, seed, sizes, flags=0):
    """One dataset per toy (toy_id = index), all toys through one batched
    generation."""
    ds, stats = ipx.toy_generate_batch(ctx, model, theta_gen, seed, np.arange(len(sizes)), np.asarray(sizes), flags)
    for j, st in enumerate(stats):
        if st["n_violations"]:
            for d in ds:
                ipx.ipx_dataset_destroy(ctx, d)
            raise RuntimeError("acceptance bound violated in toy %d" % j)
    return ds


def batched_evaluator(ipx, ctx, plan):
    def evaluate(theta, active):
        f, g = ipx.nll_eval_batch(ctx, plan, theta, active=active.astype(np.uint8), grad=True)
        return f, g
    return evaluate


def single_evaluator(ipx, ctx, ds):
    def evaluate(theta, active):
        f = np.full(1, np.inf)
        g = np.full(theta.shape, np.nan)
        if active[0]:
            f[0], g[0] = ipx.nll_grad(ctx, ds, theta[0])
        return f, g
    return evaluate


def steps_for(model, sizes, scale=1.0):
    """Parameter steps scaled as 1/sqrt(N) from the 1e5-event reference."""
    s = np.sqrt(1e5 / np.maximum(np.asarray(sizes, np.float64), 1.0))
    return scale * STEPS[model][None, :] * s[:, None]


def fit_batched(ipx, ctx, model, datasets, theta0, steps, plan=None, tune=False, **kw):
    """Lockstep BFGS over all datasets through one batched evaluation per
    round.  plan: an existing plan over `datasets` (kept), else one is made
    for the fit; tune: give a new plan its launch schedule from the autotune
    cache, timing the candidates at theta0 when the cache has none."""
    own = plan is None
    if own:
        plan = ipx.ipx_plan_create(ctx, datasets)
    try:
        if tune:
            from . import autotune
            sizes = [ipx.ipx_dataset_size(d) for d in datasets]
            autotune.tune_plan(ipx, ctx, plan, model, theta0, sizes, grad=True)
        return fit.bfgs(batched_evaluator(ipx, ctx, plan), theta0, steps, **kw)
    finally:
        if own:
            ipx.ipx_plan_destroy(plan)


def fit_plain(ipx, ctx, model, datasets, theta0, steps, **kw):
    res = [fit.bfgs(single_evaluator(ipx, ctx, d), theta0[j:j + 1], steps[j:j + 1], **kw)
           for j, d in enumerate(datasets)]
    out = {k: np.concatenate([r[k] for r in res]) for k in ("theta", "f", "grad", "edm", "converged", "failed",
                                                           "evals")}
    out["rounds"] = max(r["rounds"] for r in res)
    return out
