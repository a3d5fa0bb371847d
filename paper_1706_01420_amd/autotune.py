"""Launch-schedule cache for batched plans.

ipx_plan_autotune (in libipx) times the candidate schedules of a plan's
per-event kernel and keeps the fastest; this module remembers the choice in a
JSON file keyed by (kernel, model, gradient or not, number of segments and
total events, both rounded to powers of two, GPU architecture), so a plan of
the same shape on the same GPU gets its schedule without timing again.  The
schedule never changes results (every tile writes its own partials, summed in
tile order), only the time.

The cache file is IPX_AUTOTUNE_CACHE if set, else
~/.cache/paper_1706_01420_amd/autotune.json.
"""
import json
import math
import os
import tempfile

KERNELS = {1: "k_nll_batch<1>", 2: "k_nll_batch<2>", 3: "k_angtime_batch"}


def cache_path():
    return os.environ.get("IPX_AUTOTUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_1706_01420_amd", "autotune.json")


def bucket(x):
    """x rounded to the nearest power of two (in log2), at least 1."""
    return 1 << max(0, int(round(math.log2(max(1, int(x))))))


def key(model, grad, n_segments, n_events, arch):
    return "%s|model=%d|grad=%d|segments=%d|events=%d|%s" % (
        KERNELS[model], model, 1 if grad else 0, bucket(n_segments), bucket(n_events), arch)


def load(path=None):
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save(cache, path=None):
    path = path or cache_path()
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d or ".", prefix=".autotune.")
    with os.fdopen(fd, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def device_arch(device=0):
    import torch
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def tune_plan(ipx, ctx, plan, model, theta, sizes, grad=True, reps=5, path=None, arch=None):
    """Apply the cached schedule for this plan's shape, or time the candidates
    (ipx_plan_autotune at theta, shape (nb, np)) and cache the fastest.
    Returns (schedule, source) with source "cache" or "tuned"."""
    k = key(model, grad, len(sizes), int(sum(int(n) for n in sizes)), arch or device_arch())
    cache = load(path)
    entry = cache.get(k)
    if entry is not None:
        sched = {"workgroups": entry["workgroups"], "order": entry["order"], "graph": entry.get("graph", 1),
                 "variant": entry.get("variant", 0)}
        ipx.ipx_plan_set_schedule(plan, **sched)
        return sched, "cache"
    best, us, rows = ipx.ipx_plan_autotune(ctx, plan, theta, grad=grad, reps=reps)
    cache = load(path)  # another process may have written meanwhile
    cache[k] = {"workgroups": best["workgroups"], "order": best["order"], "graph": best["graph"],
                "variant": best["variant"], "us": us,
                "candidates": [[r[0]["workgroups"], r[0]["order"], r[0]["graph"], r[0]["variant"], r[1]] for r in rows]}
    save(cache, path)
    return best, "tuned"
