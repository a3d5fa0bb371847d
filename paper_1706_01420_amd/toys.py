"""Pseudo-experiment (toy) studies on top of libipx.

Sizes: as the paper suggests for Example 5, the number of events of each toy
is Poisson-fluctuated on the host: mean mu_j log-uniform in [1e4, 2e5], drawn
with numpy's Philox generator keyed by the study seed, then N_j ~ Poisson(mu_j).
Events: toy_generate_batch with key (seed, toy_id = j) for toy j.
Fits: fit.bfgs either through one nll_eval_batch per round (batched, graph
replay, launch schedule from the autotuner) or through nll_grad per toy (plain
loop); the per-toy arithmetic is the same, so both give the same minima.
Studies: `study` fits toys in batches and appends one JSON record per toy to
a file; a study started again on the same file skips the toys it already
holds (checkpoint and resume).
"""
import json
import os

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


def completed_ids(path, seed):
    """Toy ids with a record for `seed` in the JSONL file (none if absent); a
    torn last line (an interrupted write) is ignored."""
    done = set()
    if not os.path.exists(path):
        return done
    with open(path) as fh:
        for line in fh:
            try:
                rec = json.loads(line)
            except ValueError:
                continue
            if rec.get("seed") == seed:
                done.add(int(rec["toy_id"]))
    return done


def study(ipx, ctx, model, theta_gen, seed, ntoys, path, batch=64, start_offset=0.5, errors=True, flags=0,
          limit=None, **fit_kw):
    """Toy study with checkpoints: toys 0 .. ntoys - 1 of (seed, model) are
    generated, fitted from theta_gen + start_offset x steps and written to
    `path` (JSONL, one record per toy: seed, toy_id, n, theta, errors, nll,
    edm, converged, evals), `batch` toys at a time, each batch appended and
    flushed before the next.  Toys already recorded for this seed are
    skipped, so a study interrupted at any point resumes where it stopped:
    the counter-based stream regenerates a toy exactly from (seed, toy_id),
    and a toy's fit does not depend on which toys share its batch, so the
    records are those of an uninterrupted run.  limit: fit at most this
    many toys in this call.  Returns the number of toys fitted by this
    call."""
    from . import fit
    theta_gen = np.asarray(theta_gen, np.float64)
    _, sizes = toy_sizes(seed, ntoys)
    todo = [j for j in range(ntoys) if j not in completed_ids(path, seed)]
    if limit is not None:
        todo = todo[:max(int(limit), 0)]
    fitted = 0
    for b0 in range(0, len(todo), batch):
        ids = np.array(todo[b0:b0 + batch])
        n = sizes[ids]
        ds, stats = ipx.toy_generate_batch(ctx, model, theta_gen, seed, ids, n, flags)
        try:
            for j, st in zip(ids, stats):
                if st["n_violations"]:
                    raise RuntimeError("acceptance bound violated in toy %d" % j)
            steps = steps_for(model, n)
            theta0 = theta_gen[None, :] + start_offset * steps
            plan = ipx.ipx_plan_create(ctx, ds)
            try:
                ev = batched_evaluator(ipx, ctx, plan)
                res = fit.bfgs(ev, theta0, steps, **fit_kw)
                err = fit.errors(ev, res["theta"], steps) if errors else np.full_like(res["theta"], np.nan)
            finally:
                ipx.ipx_plan_destroy(plan)
        finally:
            for d in ds:
                ipx.ipx_dataset_destroy(ctx, d)
        with open(path, "a+") as fh:
            # a torn last line (an interrupted write) is closed off first
            if fh.tell() > 0:
                fh.seek(fh.tell() - 1)
                if fh.read(1) != "\n":
                    fh.write("\n")
            for k, j in enumerate(ids):
                rec = {"seed": int(seed), "model": int(model), "toy_id": int(j), "n": int(n[k]),
                       "theta": res["theta"][k].tolist(), "errors": err[k].tolist(), "nll": float(res["f"][k]),
                       "edm": float(res["edm"][k]), "converged": bool(res["converged"][k]),
                       "evals": int(res["evals"][k])}
                fh.write(json.dumps(rec) + "\n")
            fh.flush()
            os.fsync(fh.fileno())
        fitted += len(ids)
    return fitted
