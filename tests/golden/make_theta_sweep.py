"""Writes tests/golden/theta_sweep.json: the oracle's NLL, gradient and
gradient scale (sum_i |w_i d ln P_i / d theta_j|) for every point of the
parity sweep (tests/theta_sweep.py), on the full workload samples
(10^5 / 2x10^6 / 4x10^6 events, seeded draws of paper_1706_01420_amd.workloads).

Calls only oracle/ (and the seeded input generators); nothing here comes from
the HIP path.  The oracle at these sizes takes minutes, too long to recompute
inside the GPU test; the stored values carry the SHA-256 of the input columns
they were computed on, which the tests check before using them.

    python tests/golden/make_theta_sweep.py [--jobs 8]
"""
import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import numpy as np  # noqa: E402

import theta_sweep  # noqa: E402
from oracle import nll as N  # noqa: E402
from paper_1706_01420_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "theta_sweep.json")
_DATA = {}


def data_hash(cols, w):
    h = hashlib.sha256()
    for c in cols:
        h.update(np.ascontiguousarray(c, np.float64).tobytes())
    if w is not None:
        h.update(np.ascontiguousarray(w, np.float64).tobytes())
    return h.hexdigest()


def _task(arg):
    model, i = arg
    label, theta, grad_ok = theta_sweep.points(model)[i]
    cols, w = _DATA[model]
    if grad_ok:
        f, g, sc = N.nll_grad_scale(model, cols, theta, w)
        return model, i, f, [float(x) for x in g], [float(x) for x in sc]
    return model, i, N.nll(model, cols, theta, w), None, None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    args = ap.parse_args()
    out = {}
    for model in (1, 2, 3):
        n = W.WORKLOAD_SIZES[model]
        _DATA[model] = W.events(model, n)
        pts = theta_sweep.points(model)
        out[str(model)] = {"n": n, "data_sha256": data_hash(*_DATA[model]),
                           "points": [{"label": lab, "theta": [float(x) for x in th], "grad_defined": ok}
                                      for lab, th, ok in pts]}
    tasks = [(m, i) for m in (3, 2, 1) for i in range(len(theta_sweep.points(m)))]
    with mp.get_context("fork").Pool(args.jobs) as pool:
        for model, i, f, g, sc in pool.imap_unordered(_task, tasks):
            p = out[str(model)]["points"][i]
            p["nll"] = f
            p["grad"] = g
            p["grad_scale"] = sc
            print("model %d point %d: nll %.17g" % (model, i, f), flush=True)
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
