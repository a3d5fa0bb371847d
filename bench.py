"""Benchmark: NLL + gradient evaluations per second on one MI355X.

One step = one nll_grad call over the angular x decay-time workload
(N = 4,000,000 events, 6 FP64 columns + weights, 12 free parameters): parameter
hoisting, the per-event PDF / normalisation / weighted log / adjoint kernel, the
two-level tile reduction, the 53-double readback and the host Jacobian.
The event sample is resident in HBM before the timed region starts.

Prints one JSON line.  Usage:
    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "NLL+grad evaluations/sec and events/sec (FP64); fits/sec batched vs plain; p99"
PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 vector: 256 CU x 2.4 GHz x 128 FLOP/clk
PEAK_HBM_GBS = 8000.0

# Algorithmic FP64 operations, counted on the formulas (not on the generated
# code): +, -, x, / and sqrt 1; a*b+c 2; exp and log 20; a sin/cos pair 40.
# Per event outside the resolution corrections:
FLOP_BASE = {
    (1, False): 73, (1, True): 93,
    (2, False): 193, (2, True): 348,
    (3, False): 467, (3, True): 672,      # angular (gradient: with the 40 coefficient adjoints, 40 a*b+c)
}
# A resolution correction needed at one time point costs a + b K with K the
# continued-fraction depth that event needs (a real erfcx is 6 + 7K, the
# complex w 25 + 21K): at the range ends (with the Phi term of the
# normalisation) and at the event time t.
CORR_FLOP = {2: {"range": (56, 21), "t": (46, 14)}, 3: {"range": (88, 42), "t": (78, 35)}}
# Continued-fraction depth table (paper_1706_01420_amd/csrc/cf_depth.h).
CF_DEPTH_E = [24.625, 20.875, 17.875, 15.625, 13.750, 12.375, 10.625, 8.375, 6.375]
CORR_SKIP = 36.5          # cf_depth.h: kCfSkipE
T_LO, T_HI = 0.3, 15.0


def _lane_depths(x, re2, e_shift):
    """Per-event need flag and depth at one time point: the correction is
    counted where its size relative to the main term reaches 2^-57, at the
    smallest continued-fraction depth whose error bound meets the same
    target for that event (its own accuracy requirement, whatever events
    share its wave or however they are stored)."""
    import numpy as np
    with np.errstate(invalid="ignore"):
        E = np.where(x > 0.0, x * x - re2, -1.0) - e_shift
    need = ~(E >= CORR_SKIP)
    eff = np.where(need, E, CORR_SKIP)
    depth = 1 + sum((eff < th).astype(np.int64) for th in CF_DEPTH_E)
    return need, depth


def algorithmic_flops(model, t, sig_t, theta, grad):
    """FP64 operations of one evaluation over the events (t, sigma_t in any
    order): the formulas' base count per event plus, for every event, each
    resolution correction its accuracy needs at the depth it needs.  The
    count follows the method, not the kernel: a wave that evaluates a
    correction or a deeper fraction for some of its lanes earns nothing for
    the others, and the count does not change with the storage order."""
    import numpy as np
    n = t.size
    total = float(FLOP_BASE[(model, grad)]) * n
    if model == 1:
        return total
    if model == 2:
        gmax = max(1.0 / theta[4], 1.0 / theta[5])
        sig = theta[6] * sig_t
        re2 = np.zeros(n)
    else:
        g, dg, dm = theta[6], theta[7], theta[8]
        gmax = g + abs(dg) / 2.0
        sig = sig_t
        re2 = (dm * sig / np.sqrt(2.0)) ** 2
    inv_r2s = 1.0 / (np.sqrt(2.0) * sig)
    s2 = sig * sig
    for tau, kind, shift in ((t, "t", 0.0), (T_LO, "range", gmax * T_LO), (T_HI, "range", gmax * T_HI)):
        x = (tau - gmax * s2) * inv_r2s
        need, depth = _lane_depths(x, re2, shift)
        a, b = CORR_FLOP[model][kind]
        total += float(np.sum(np.where(need, a + b * depth, 0)))
    return total


BYTES_PER_EVENT = {1: 8, 2: 24, 3: 56}


def progress(msg):
    """One line per finished leg on stderr (the JSON line stays alone on stdout)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=200)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-extra", action="store_true", help="skip the secondary per-model rates")
    p.add_argument("--no-batched", action="store_true", help="skip the batched toy-fit leg")
    p.add_argument("--no-served", action="store_true", help="skip the served-likelihood leg")
    p.add_argument("--profile", action="store_true",
                   help="profiling run: the timed steps, then a plain 512 MiB device copy (counter calibration)")
    return p.parse_args()


# HBM traffic of the dominant kernel from the rocprofv3 FETCH_SIZE / WRITE_SIZE
# runs (scaled by the calibration copy), valid for the kernel sources whose
# hash is recorded with it; reported as null once those sources change.
TRAFFIC = {"sources_sha256": "78ae25fba20e74df60c97f24c12e7a03afa430f3aa03f5192e8e1772ef7658b5", "bytes_per_launch": 231475645}
KERNEL_SOURCES = ["ipx_kernels.h", "ipx_batch.h", "ipx_math.h", "ipx_models.h", "weideman_coeffs.h", "cf_depth.h",
                  "minimax_coeffs.h"]


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1706_01420_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def calibration_copy(nbytes=512 << 20, reps=3):
    """A plain device-to-device copy kernel of known size (torch's copy),
    used to scale the HBM byte counters of a profiled run."""
    import torch
    x = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    return {"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}


# Secondary legs warm the GPU up for this long before their timed calls: after
# the host prepares a leg's data the GPU has idled and needs ~50 ms of work to
# reach its steady clock again (the main leg reports its own cold start).
SECONDARY_WARM_S = 0.06


def _warm(call, warmup, warm_s):
    """warmup calls, then more until warm_s seconds of calls have run."""
    import torch
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < warm_s:
        call()
        torch.cuda.synchronize()


def timed_rate(ipx, ctx, ds, theta, steps, warmup, grad, warm_s=0.0):
    """(seconds per call, seconds per launch of the per-event kernel).  The
    call rate is timed with the library's kernel timing off; the kernel time
    comes from a second pass of the same calls with HIP events around the
    per-event kernel on its stream."""
    import torch
    call = (lambda: ipx.nll_grad(ctx, ds, theta)) if grad else (lambda: ipx.nll_eval(ctx, ds, theta))
    _warm(call, warmup, warm_s)
    t0 = time.perf_counter()
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ipx.ipx_timing_read(ctx, reset=True)
    ipx.ipx_timing_enable(ctx, True)
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    ipx.ipx_timing_enable(ctx, False)
    kms, launches = ipx.ipx_timing_read(ctx, reset=True)
    return (t1 - t0) / steps, kms / max(launches, 1) / 1e3


# ---------------------------------------------------------------------------
# CPU baseline: the oracle as it stands, on this host's cores
# ---------------------------------------------------------------------------
_CPU = {}   # inputs shared with the forked worker processes


def _cpu_workers():
    """One worker process per core this process may run on, at most 16 (the
    CPU share of one GPU on the benchmark hosts)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_eval_chunk(i):
    from oracle import nll as N
    cols, w, theta, chunks = _CPU["eval"]
    lo, hi = chunks[i]
    return N.nll_grad(3, [c[lo:hi] for c in cols], theta, None if w is None else w[lo:hi])


def _cpu_gen_toy(j):
    from oracle import generate as OG
    theta, seed, sizes = _CPU["gen"]
    r = OG.generate(3, theta, seed, j, int(sizes[j]))
    return r["cols"], r["w"]


def _cpu_fit_toy(j):
    import numpy as np
    from oracle import nll as N
    from paper_1706_01420_amd import fit
    cols, w = _CPU["toys"][j]
    start, steps = _CPU["fit"]

    def evaluate(th, active):
        f, g = N.nll_grad(3, cols, th[0], w)
        return np.array([f]), g[None, :]

    r = fit.bfgs(evaluate, start[j:j + 1], steps[j:j + 1])
    return bool(r["converged"][0]), int(r["evals"][0])


def _cpu_request(i):
    from oracle import nll as N
    j, th, grad = _CPU["mix"][i]
    model, cols, w = _CPU["mix_data"][j]
    return N.nll_grad(model, cols, th, w) if grad else N.nll(model, cols, th, w)


def _noop(_):
    return None


def cpu_baseline(cols, w, theta, reps=5, ntoys=16, nreq=16):
    """The oracle (numpy/scipy FP64, exactly rounded sums, dual-number
    gradient) timed on the host's cores: worker processes forked before this
    process touches the GPU, each running the oracle single-threaded on its
    share of the work.
      value       NLL+grad evaluations/s of the full angular sample (events
                  split into chunks over the workers; median of `reps`);
      toy_fits    fits/s of the first `ntoys` toys of the batched-fit study
                  (generated by the oracle's generator, one BFGS fit per
                  worker with the oracle's gradient, same start and steps);
      served_mix  evaluations/s over the first `nreq` requests of the served
                  mix (datasets of the mix's models and sizes)."""
    import multiprocessing as mp
    import numpy as np
    import oracle  # noqa: F401  (imported once, before the workers fork)
    from oracle import generate, nll  # noqa: F401
    from paper_1706_01420_amd import fit, toys, workloads  # noqa: F401
    workers = _cpu_workers()
    fork = mp.get_context("fork")
    n = cols[0].size
    edges = np.linspace(0, n, 2 * workers + 1).astype(np.int64)
    _CPU["eval"] = (cols, w, list(theta), list(zip(edges[:-1].tolist(), edges[1:].tolist())))
    times = []
    with fork.Pool(workers) as pool:
        pool.map(_noop, range(workers))
        for _ in range(reps):
            t0 = time.perf_counter()
            pool.map(_cpu_eval_chunk, range(len(edges) - 1))
            times.append(time.perf_counter() - t0)
    med = float(np.median(times))
    progress("cpu baseline: full-sample evaluations %s s" % ", ".join("%.2f" % t for t in times))
    # one thread: two of the chunks in this process, scaled to the full sample
    t0 = time.perf_counter()
    for c in (0, 1):
        _cpu_eval_chunk(c)
    t_one = (time.perf_counter() - t0) / 2 * (len(edges) - 1)
    out = {"value": 1.0 / med, "unit": "NLL+grad evals/s", "cores": workers, "kind": "oracle",
           "sample": "oracle nll_grad over all %d events of the angular workload, split into %d chunks over %d "
                     "single-threaded worker processes; median of %d repetitions (%s s)"
                     % (n, len(edges) - 1, workers, reps, ", ".join("%.2f" % t for t in times)),
           "host": {"cpu_model": _cpu_model(), "nproc": os.cpu_count(), "workers": workers},
           "single_thread": {"evals_per_s": 1.0 / t_one,
                             "sample": "chunks 0 and 1 of the %d on one thread, scaled to the full sample"
                                       % (len(edges) - 1)}}

    # batched-toy fits: the same toys (seed, ids, sizes) and start points
    seed = 170601424
    _, sizes = toys.toy_sizes(seed, 512)
    steps = toys.steps_for(3, sizes)
    start = fit_start(np.array(theta), steps, seed)[:ntoys]   # the GPU study's first toys
    sizes, steps = sizes[:ntoys], steps[:ntoys]
    _CPU["gen"] = (list(theta), seed, sizes)
    with fork.Pool(workers) as pool:
        _CPU["toys"] = pool.map(_cpu_gen_toy, range(ntoys))
    _CPU["fit"] = (start, steps)
    with fork.Pool(workers) as pool:
        pool.map(_noop, range(workers))
        t0 = time.perf_counter()
        fits = pool.map(_cpu_fit_toy, range(ntoys))
        t_fit = time.perf_counter() - t0
    progress("cpu baseline: %d toy fits in %.2f s" % (ntoys, t_fit))
    out["toy_fits"] = {"fits_per_s": ntoys / t_fit, "wall_s": t_fit, "toys": ntoys,
                       "events": int(sizes.sum()), "converged": float(np.mean([c for c, _ in fits])),
                       "evals_per_fit_mean": float(np.mean([e for _, e in fits])),
                       "sample": "first %d toys of the 512-toy study, generated by the oracle, one fit per worker "
                                 "(%d workers)" % (ntoys, workers)}

    # served mix: the first requests of the served benchmark's stream
    sizes_s, models_s, reqs = served_mix(nreq=nreq)
    used = sorted({j for j, _, _ in reqs})
    _CPU["mix"] = reqs
    _CPU["mix_data"] = {j: (models_s[j],) + tuple(workloads.events(models_s[j], int(sizes_s[j]), seed=170601425 + j))
                        for j in used}
    with fork.Pool(workers) as pool:
        pool.map(_noop, range(workers))
        t0 = time.perf_counter()
        pool.map(_cpu_request, range(len(reqs)))
        t_mix = time.perf_counter() - t0
    out["served_mix"] = {"evals_per_s": len(reqs) / t_mix, "wall_s": t_mix, "requests": len(reqs),
                         "events": int(sum(int(sizes_s[j]) for j, _, _ in reqs)),
                         "sample": "first %d requests of the served stream (half with gradient), datasets of the "
                                   "mix's models and sizes drawn by the workload generator, one request per worker "
                                   "at a time" % len(reqs)}
    _CPU.clear()
    return out


def served_mix(ndatasets=64, nclients=256, nreq=600, seed=170601425):
    """The served benchmark's datasets (models cycled 1, 2, 3; sizes
    log-uniform in [1e3, 5e6]) and request stream: 256 clients, each bound to
    one dataset, half asking NLL only (random-walk chains), half NLL +
    gradient (minimisers), parameters jittered around the generation point."""
    import numpy as np
    from paper_1706_01420_amd import workloads
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(np.log(1e3), np.log(5e6), ndatasets)).astype(np.int64)
    models = [1 + (j % 3) for j in range(ndatasets)]
    client_ds = rng.integers(ndatasets, size=nclients)
    client_grad = np.arange(nclients) >= nclients // 2
    reqs = []
    for _ in range(nreq):
        c = rng.integers(nclients)
        j = int(client_ds[c])
        th = np.array(workloads.THETA_GEN[models[j]])
        th = th * (1.0 + 0.002 * rng.standard_normal(th.size))
        reqs.append((j, th, bool(client_grad[c])))
    return sizes, models, reqs


def fit_start(theta, steps, seed):
    """Start points of the study's fits: theta + 2 steps with seeded signs."""
    import numpy as np
    signs = np.random.default_rng(seed).choice(np.array([-1.0, 1.0]), size=steps.shape)
    return np.asarray(theta, np.float64)[None, :] + 2.0 * signs * steps


def bench_batched_fits(ipx, ctx, ntoys=512, plain_subset=64, seed=170601424):
    """512 pseudo-experiments of the angular model, sizes Poisson(mu), mu
    log-uniform in [1e4, 2e5]; generated on the device, each fitted by the
    lockstep BFGS with the analytic gradient: all toys through one batched
    evaluation per round (graph replay) versus the plain per-toy loop (one
    nll_grad call per evaluation), same algorithm and stopping rule.  Each
    fit starts two parameter steps (about two statistical errors) from the
    generation point in every parameter, with seeded random signs."""
    import numpy as np
    import torch
    from paper_1706_01420_amd import fit, toys, workloads
    theta = np.array(workloads.THETA_GEN[3])
    _, sizes = toys.toy_sizes(seed, ntoys)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ds = toys.generate(ipx, ctx, 3, theta, seed, sizes)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    steps = toys.steps_for(3, sizes)
    start = fit_start(theta, steps, seed)
    plan = None
    try:
        # launch schedule: the autotuner times its candidates on this plan
        # (the cache is per run, so the timing is always done and reported)
        plan = ipx.ipx_plan_create(ctx, ds)
        t0 = time.perf_counter()
        best, us, rows = ipx.ipx_plan_autotune(ctx, plan, start, grad=True, reps=5)
        t_tune = time.perf_counter() - t0
        t0 = time.perf_counter()
        rb = toys.fit_batched(ipx, ctx, 3, ds, start, steps, plan=plan)
        t_b = time.perf_counter() - t0
        k = plain_subset
        t0 = time.perf_counter()
        rp = toys.fit_plain(ipx, ctx, 3, ds[:k], start[:k], steps[:k])
        t_p = time.perf_counter() - t0
    finally:
        if plan is not None:
            ipx.ipx_plan_destroy(plan)
        for d in ds:
            ipx.ipx_dataset_destroy(ctx, d)
    same = bool(np.array_equal(rb["theta"][:k], rp["theta"]))
    return {"workload": "512 angular toys, N ~ Poisson(mu), mu log-uniform [1e4, 2e5], total %d events" % int(sizes.sum()),
            "generate_s": t_gen, "generated_events_per_s": float(sizes.sum()) / t_gen,
            "fits_per_s_batched": ntoys / t_b, "fits_per_s_plain": k / t_p,
            "plain_sample": "first %d toys" % k, "speedup": (ntoys / t_b) / (k / t_p),
            "rounds_batched": int(rb["rounds"]), "evals_per_fit_mean": float(rb["evals"].mean()),
            "converged_batched": float(rb["converged"].mean()), "converged_plain": float(rp["converged"].mean()),
            "same_minima_bitwise": same,
            "autotune": {"schedule": best, "us_per_eval": us, "tune_s": t_tune,
                         "candidates": [[r[0]["workgroups"], r[0]["order"], r[0]["graph"], round(r[1], 1)] for r in rows]}}


SERVE_POLICY_NAMES = {0: "spread", 1: "oldest_first", 2: "fewest_first"}


def bench_served(ipx, ctx, ndatasets=64, nclients=256, nreq=600, seed=170601425,
                 policies=((0, (0.5, 0.8, None)),)):
    """Served likelihood: 64 resident datasets (models cycled 1, 2, 3; sizes
    log-uniform in [1e3, 5e6]; generated on the device), 256 clients (half
    random-walk chains asking NLL only, half minimisers asking NLL +
    gradient), Poisson arrivals at 0.5x and 0.8x the plain one-call-per-request
    throughput.  Latency = submission to completion.  The first claim policy
    listed gives the main figures; the others, run on the same datasets and
    the same arrival times, are reported beside them."""
    import numpy as np
    from paper_1706_01420_amd import workloads
    sizes, models, reqs = served_mix(ndatasets, nclients, nreq, seed)
    ds = []
    try:
        for j in range(ndatasets):
            d, _ = ipx.toy_generate(ctx, models[j], workloads.THETA_GEN[models[j]], seed, j, int(sizes[j]))
            ds.append(d)
        # plain: one call per request, back to back
        lat_plain = []
        t0 = time.perf_counter()
        for j, th, g in reqs:
            a = time.perf_counter()
            if g:
                ipx.nll_grad(ctx, ds[j], th)
            else:
                ipx.nll_eval(ctx, ds[j], th)
            lat_plain.append((time.perf_counter() - a) * 1e6)
        plain_rate = nreq / (time.perf_counter() - t0)
        out = {"workload": "64 datasets (models 1/2/3, %d events in total), 256 clients, %d requests per rate, "
                           "half with gradient" % (int(sizes.sum()), nreq),
               "plain_evals_per_s": plain_rate,
               "plain_latency_us_p50": float(np.percentile(lat_plain, 50)),
               "plain_latency_us_p99": float(np.percentile(lat_plain, 99))}
        for i, (policy, rates) in enumerate(policies):
            res = _served_rates(ipx, ctx, ds, models, reqs, plain_rate, policy, rates, seed)
            if i == 0:
                out["policy"] = SERVE_POLICY_NAMES[policy]
                out.update(res)
            else:
                out.setdefault("other_policies", {})[SERVE_POLICY_NAMES[policy]] = res
        return out
    finally:
        for d in ds:
            ipx.ipx_dataset_destroy(ctx, d)


def _served_rates(ipx, ctx, ds, models, reqs, plain_rate, policy, rates, seed):
    import numpy as np
    from paper_1706_01420_amd import workloads
    nreq = len(reqs)
    # arrival times from their own stream, the same for every policy
    rng = np.random.default_rng(seed + 1)
    out = {}
    srv = ipx.ipx_server_start(ctx, slots=64, policy=policy)
    try:
        # warm-up (untimed): the first launch of the device loop and every
        # dataset's first request
        warm = [ipx.ipx_submit(srv, ds[j], np.array(workloads.THETA_GEN[models[j]]), g)
                for j in range(len(ds)) for g in (False, True)]
        for t in warm:
            ipx.ipx_wait(srv, t, 60.0)
        for frac in rates:
            key = "served_at_%.1fx" % frac if frac is not None else "served_saturated"
            # one thread submits at the paced times, then collects: latencies
            # are stamped inside the library (submission to completion), so no
            # Python thread sits between a request and its result
            tickets = []
            results = []
            errors = []
            t_end = time.perf_counter() + 60.0   # the whole rate step is bounded
            # the arrival process is paced by this Python loop: a collection of
            # the interpreter's garbage (tens of ms with the objects of the
            # earlier legs) would stall it and release a burst
            gc.collect()
            gc.disable()
            t0 = time.perf_counter()
            nxt = t0
            t_sub = []
            for j, th, g in reqs:
                if frac is not None:
                    nxt += rng.exponential(1.0 / (frac * plain_rate))
                    while time.perf_counter() < nxt:
                        pass
                t_sub.append(time.perf_counter())
                tickets.append(ipx.ipx_submit(srv, ds[j], th, g))
            try:
                for t in tickets:
                    results.append(ipx.ipx_wait(srv, t, max(t_end - time.perf_counter(), 0.0)))
            except ipx.IpxError as e:
                errors.append(str(e))
            finally:
                gc.enable()
            # from the first submission to the last completion (submission
            # time + the library's latency stamp), not to the end of the
            # collection loop
            elapsed = (max(ts + r["latency_us"] * 1e-6 for ts, r in zip(t_sub, results)) - t0
                       if len(results) == nreq else time.perf_counter() - t0)
            if errors or len(results) < nreq:
                out[key] = {"error": errors[0] if errors else "incomplete", "completed": len(results),
                            "server": ipx.ipx_server_stats_read(srv)}
                break
            lat = np.array([r["latency_us"] for r in results])
            out[key] = {"offered_per_s": None if frac is None else frac * plain_rate,
                        "evals_per_s": nreq / elapsed,
                        "latency_us_p50": float(np.percentile(lat, 50)),
                        "latency_us_p99": float(np.percentile(lat, 99)),
                        "all_ok": bool(all(r["status"] == 0 for r in results)),
                        "server": ipx.ipx_server_stats_read(srv)}
    finally:
        ipx.ipx_server_stop(srv)
    return out


def _timed_calls(call, steps, warmup, ipx=None, ctx=None, warm_s=SECONDARY_WARM_S):
    """(seconds per call, seconds per timed kernel launch or None)."""
    import torch
    _warm(call, warmup, warm_s)
    t0 = time.perf_counter()
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    if ipx is None:
        return dt, None
    ipx.ipx_timing_read(ctx, reset=True)
    ipx.ipx_timing_enable(ctx, True)
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    ipx.ipx_timing_enable(ctx, False)
    kms, launches = ipx.ipx_timing_read(ctx, reset=True)
    return dt, (kms / launches / 1e3 if launches else None)


def bench_next(ipx, ctx, steps, warmup):
    """The extensions of the angular and mass paths: the tagged angular
    model, the simultaneous fit over 6 KK-mass bins x 2 flavours, the Ipatia
    model with its grid normalisation, and the binned path (smearing, binned
    NLL, CL_s toys)."""
    import numpy as np
    import torch
    from paper_1706_01420_amd import workloads
    out = {}
    n = workloads.WORKLOAD_SIZES[3]
    # tagged angular model at the angular workload's size
    c4, w4 = workloads.events(4, n)
    d4 = ipx.ipx_dataset_create(ctx, 4, c4, w4)
    th = np.array(workloads.THETA_GEN[4])
    s, k = _timed_calls(lambda: ipx.nll_grad(ctx, d4, th), steps, warmup, ipx, ctx)
    out["tagged_nll_grad"] = {"n_events": n, "evals_per_s": 1 / s, "kernel_us": k * 1e6,
                              "events_per_s": n / s}
    ipx.ipx_dataset_destroy(ctx, d4)
    del c4, w4
    # simultaneous fit: 12 categories sharing the 4e6 events
    nbins, per = 6, n // 12
    dss, bins = [], []
    csp = [0.95, 0.81, 0.64, 0.52, 0.46, 0.39]
    for b in range(nbins):
        for q in (1.0, -1.0):
            c, w = workloads.events(4, per, seed=workloads.BENCH_SEED + 40 + 2 * b + (q > 0), q=q)
            d = ipx.ipx_dataset_create(ctx, 4, c, w)
            ipx.ipx_dataset_set_angular(ctx, d, None, csp[b])
            dss.append(d)
            bins.append(b)
    sim = ipx.ipx_sim_create(ctx, dss, bins, nbins)
    g = workloads.THETA_GEN[3]
    ths = np.array([g[0], g[1], g[3], g[4], g[6], g[7], g[8], g[9], g[10], g[11]] + [0.05, 0.35] * nbins)
    s, k = _timed_calls(lambda: ipx.nll_sim(ctx, sim, ths, grad=True), steps, warmup)
    out["sim_12cat_nll_grad"] = {"categories": 12, "n_events": per * 12, "nparams": int(ths.size),
                                 "evals_per_s": 1 / s, "events_per_s": per * 12 / s}
    ipx.ipx_sim_destroy(sim)
    for d in dss:
        ipx.ipx_dataset_destroy(ctx, d)
    # Ipatia model at the mass workload's size
    nm = workloads.WORKLOAD_SIZES[1]
    c5, _ = workloads.events(5, nm)
    d5 = ipx.ipx_dataset_create(ctx, 5, c5, None)
    th5 = np.array(workloads.THETA_GEN[5])
    s, k = _timed_calls(lambda: ipx.nll_eval(ctx, d5, th5), steps, warmup, ipx, ctx)
    out["ipatia_nll_eval"] = {"n_events": nm, "grid_points": 16384, "evals_per_s": 1 / s,
                              "us_per_eval": s * 1e6, "event_kernel_us": k * 1e6}
    ipx.ipx_dataset_destroy(ctx, d5)
    # and at the large sample size of the paper's Example 1 table (10^7 events)
    nl = 10_000_000
    c5, _ = workloads.events(5, nl)
    d5 = ipx.ipx_dataset_create(ctx, 5, c5, None)
    s, k = _timed_calls(lambda: ipx.nll_eval(ctx, d5, th5), steps, warmup, ipx, ctx)
    out["ipatia_nll_eval_1e7"] = {"n_events": nl, "grid_points": 16384, "evals_per_s": 1 / s,
                                  "us_per_eval": s * 1e6, "event_kernel_us": k * 1e6,
                                  "events_per_s": nl / s}
    ipx.ipx_dataset_destroy(ctx, d5)
    # binned path: 10^4 bins (CL_s workload)
    nb_bins, lo, hi = 10_000, 5179.0, 5379.0
    h = torch.rand(nb_bins, dtype=torch.float64, device="cuda")
    s, _ = _timed_calls(lambda: ipx.ipx_smear(ctx, h, (hi - lo) / nb_bins, 2.0), steps, warmup)
    out["smear_10k_bins"] = {"us_per_call": s * 1e6, "fma": nb_bins * nb_bins,
                             "tflops": 2.0 * nb_bins * nb_bins / s / 1e12}
    H = ipx.ipx_hist_create(ctx, nb_bins, lo, hi, 5279.0, 3.0, 2.0)
    thb = (70.0, 50_000.0, 0.004)
    ipx.ipx_hist_set_counts(ctx, H, ipx.ipx_binned_toy(ctx, H, thb, 7, 0, 0))
    s, _ = _timed_calls(lambda: ipx.nll_binned(ctx, H, thb, grad=True), steps, warmup)
    out["binned_nll_grad_10k_bins"] = {"evals_per_s": 1 / s, "us_per_eval": s * 1e6}
    ntoys = 10_000
    s, k = _timed_calls(lambda: ipx.cls_toys(ctx, H, thb, 2024, ntoys), max(steps // 10, 3),
                        max(warmup // 10, 1), ipx, ctx)
    r = ipx.cls_toys(ctx, H, thb, 2024, ntoys)
    out["cls_10k_toys"] = {"bins": nb_bins, "toys_per_hypothesis": ntoys, "seconds_per_cls": s,
                           "toy_kernel_ms": k * 1e3, "poisson_draws_per_s": 2 * ntoys * nb_bins / k,
                           "cl_b": r["cl_b"], "cl_sb": r["cl_sb"], "cl_s": r["cl_s"]}
    ipx.ipx_hist_destroy(ctx, H)
    return out


def bench_mass_batch(ipx, ctx, steps, warmup, nb=64):
    """The mass model's HBM roofline on a batch: one 10^5-event call moves
    0.8 MB and is launch-latency bound, so 64 datasets of that size are
    evaluated per call (one plan, graph replay); 51 MB per call, which the
    256 MB last-level cache (MALL) can hold."""
    import numpy as np
    import torch
    from paper_1706_01420_amd import workloads
    nm = workloads.WORKLOAD_SIZES[1]
    dsl = []
    plan = None
    try:
        for j in range(nb):
            c, _ = workloads.events(1, nm, seed=workloads.BENCH_SEED + 100 + j)
            dsl.append(ipx.ipx_dataset_create(ctx, 1, c, None))
        plan = ipx.ipx_plan_create(ctx, dsl)
        th = np.tile(np.array(workloads.THETA_GEN[1]), (nb, 1))
        _warm(lambda: ipx.nll_eval_batch(ctx, plan, th), warmup, SECONDARY_WARM_S)
        t0 = time.perf_counter()
        for _ in range(steps):
            ipx.nll_eval_batch(ctx, plan, th)
        dt = (time.perf_counter() - t0) / steps
    finally:
        if plan is not None:
            ipx.ipx_plan_destroy(plan)
        for d in dsl:
            ipx.ipx_dataset_destroy(ctx, d)
    nbytes = BYTES_PER_EVENT[1] * nm * nb
    return {"datasets": nb, "events": nm * nb, "us_per_call": dt * 1e6, "evals_per_s": nb / dt,
            "bytes_per_call": nbytes, "gbs": nbytes / dt / 1e9, "frac_hbm": nbytes / dt / 1e9 / PEAK_HBM_GBS,
            "note": "wall time per batched call (graph replay, reduction and readback included); the 51 MB "
                    "of columns fit in the 256 MB MALL"}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the likelihood path is measured on a single MI355X "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    from paper_1706_01420_amd import workloads

    model = 3
    n = workloads.WORKLOAD_SIZES[model]
    cols, w = workloads.events(model, n)
    theta = np.array(workloads.THETA_GEN[model])
    cpu = None
    if not args.no_cpu_baseline and not args.profile:
        # first, while this process has not touched the GPU: the oracle's
        # worker processes are forked from it
        cpu = cpu_baseline(cols, w, theta)
        progress("cpu baseline done: %.4g evals/s on %d workers" % (cpu["value"], cpu["cores"]))

    import torch
    from paper_1706_01420_amd import ipx
    ctx = ipx.ipx_create(0)
    ds = ipx.ipx_dataset_create(ctx, model, cols, w)
    torch.cuda.synchronize()

    # the GPU's clock rises over the first ~50 ms of work after it idled
    # (the CPU baseline above, or a fresh process): the first calls, timed
    # as they come, are reported as the cold start, and the timed steps then
    # measure the steady state; the FP64 ceiling probe (75 ms of FMA loop,
    # reported below) runs after them, since the GPU runs slower for a while
    # after it
    cold = None
    if not args.profile:
        ipx.nll_grad(ctx, ds, theta)
        cold = []
        for _ in range(10):
            cold.append(_timed_calls(lambda: ipx.nll_grad(ctx, ds, theta), 25, 0, warm_s=0.0)[0])
    step_s, kernel_s = timed_rate(ipx, ctx, ds, theta, args.steps, args.warmup, grad=True)
    value = 1.0 / step_s
    progress("angular nll_grad: %.4f ms per call, kernel %.1f us" % (step_s * 1e3, kernel_s * 1e6))
    flops = algorithmic_flops(model, cols[3], cols[4], theta, True)
    achieved = flops / kernel_s / 1e12
    # what this GPU sustains on a pure FP64 FMA loop (clock under load)
    fma_tflops, clock_ghz = ipx.ipx_fp64_peak_probe(ctx)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "NLL+grad evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded numpy draws with the workload's ranges and distributions)",
        "config": {"workload": "angular x decay-time unbinned NLL+gradient, N=4,000,000 events, "
                               "12 free parameters, per-event weights U(0.8,1)",
                   "n_events": n, "parallelism": "single GPU"},
        "events_per_s": value * n,
        "cold_start": None if cold is None else {
            "ms_per_step_by_25": [round(c * 1e3, 4) for c in cold],
            "note": "the first 250 steps after the process started (one untimed call first), in groups of 25, "
                    "before the warm-up and timed steps: the GPU still reaching its steady clock"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": TRAFFIC["bytes_per_launch"] if TRAFFIC["sources_sha256"] == kernel_sources_hash() else None,
                     "traffic_unit": "bytes",
                     "kernel": "k_angtime_batch<true>", "kernel_us": kernel_s * 1e6,
                     "flop_per_event": flops / n,
                     "fp64_fma_loop": {"tflops": fma_tflops, "clock_ghz": clock_ghz,
                                       "frac": achieved / fma_tflops if fma_tflops > 0 else None}},
    }
    extra = {}
    if not args.no_extra:
        e_step, e_kern = timed_rate(ipx, ctx, ds, theta, max(args.steps // 2, 5), max(args.warmup // 2, 2), grad=False,
                                    warm_s=SECONDARY_WARM_S)
        fe = algorithmic_flops(model, cols[3], cols[4], theta, False)
        extra["angtime_nll_eval"] = {"evals_per_s": 1 / e_step, "kernel_us": e_kern * 1e6,
                                     "flop_per_event": fe / n, "tflops": fe / e_kern / 1e12}
    ipx.ipx_dataset_destroy(ctx, ds)
    if not args.no_extra:
        for m in (1, 2):
            nm = workloads.WORKLOAD_SIZES[m]
            c, wm = workloads.events(m, nm)
            d = ipx.ipx_dataset_create(ctx, m, c, wm)
            th = np.array(workloads.THETA_GEN[m])
            for grad in (False, True):
                s, k = timed_rate(ipx, ctx, d, th, max(args.steps // 2, 5), max(args.warmup // 2, 2), grad,
                                  warm_s=SECONDARY_WARM_S)
                key = ("mass" if m == 1 else "masstime") + ("_nll_grad" if grad else "_nll_eval")
                fm = algorithmic_flops(m, c[1], c[2], th, grad) if m == 2 else FLOP_BASE[(m, grad)] * nm
                extra[key] = {"n_events": nm, "evals_per_s": 1 / s, "us_per_eval": s * 1e6,
                              "kernel_us": k * 1e6, "flop_per_event": fm / nm,
                              "tflops": fm / k / 1e12,
                              "hbm_gbs": BYTES_PER_EVENT[m] * nm / k / 1e9}
            ipx.ipx_dataset_destroy(ctx, d)
        extra["mass_nll_eval_batch64"] = bench_mass_batch(ipx, ctx, max(args.steps // 2, 5),
                                                          max(args.warmup // 2, 2))
        extra.update(bench_next(ipx, ctx, max(args.steps // 2, 5), max(args.warmup // 2, 2)))
        extra["warm_up"] = ("each secondary leg runs W/2 warm-up calls and then %.0f ms of further calls before "
                            "its timed calls (the GPU idles while the host prepares a leg's data)"
                            % (SECONDARY_WARM_S * 1e3))
        out["extra"] = extra
        progress("secondary rates done")
    if not args.no_batched and not args.profile:
        out["batched"] = bench_batched_fits(ipx, ctx)
        progress("batched fits done")
    if not args.no_served and not args.profile:
        # the library's default claim policy first, the other two beside it
        out["served"] = bench_served(ipx, ctx, policies=((0, (0.5, 0.8, None)), (1, (0.5, 0.8)), (2, (0.5, 0.8))))
        progress("served leg done")
    ipx.ipx_destroy(ctx)
    if args.profile:
        out["calibration"] = calibration_copy()
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
