"""The stored oracle values of the parity sweep (tests/golden/theta_sweep.json,
written by tests/golden/make_theta_sweep.py) belong to the current input
draws and to the oracle as it stands: the input hashes are recomputed, and
the cheapest model's points are re-evaluated with the oracle."""
import hashlib
import json
import os

import numpy as np

import theta_sweep
from oracle import nll as N
from paper_1706_01420_amd import workloads as W

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "theta_sweep.json")


def _hash(cols, w):
    h = hashlib.sha256()
    for c in cols:
        h.update(np.ascontiguousarray(c, np.float64).tobytes())
    if w is not None:
        h.update(np.ascontiguousarray(w, np.float64).tobytes())
    return h.hexdigest()


def test_sweep_file_matches_inputs_and_points():
    with open(GOLD) as fh:
        gold = json.load(fh)
    for model in (1, 2, 3):
        g = gold[str(model)]
        assert g["n"] == W.WORKLOAD_SIZES[model]
        assert g["data_sha256"] == _hash(*W.events(model, g["n"]))
        pts = theta_sweep.points(model)
        assert [p["label"] for p in g["points"]] == [lab for lab, _, _ in pts]
        for p, (_, th, ok) in zip(g["points"], pts):
            assert p["theta"] == [float(x) for x in th] and p["grad_defined"] == ok
            assert np.isfinite(p["nll"])
            assert (p["grad"] is not None) == ok


def test_sweep_values_are_the_oracles():
    with open(GOLD) as fh:
        g = json.load(fh)["1"]
    cols, w = W.events(1, g["n"])
    for p in g["points"]:
        f, gr, sc = N.nll_grad_scale(1, cols, p["theta"], w)
        assert abs(f - p["nll"]) <= 1e-13 * abs(f)
        assert np.allclose(gr, p["grad"], rtol=1e-10, atol=1e-12 * np.max(sc))
        assert np.allclose(sc, p["grad_scale"], rtol=1e-12)
