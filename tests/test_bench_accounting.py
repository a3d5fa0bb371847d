"""The measurement code's own arithmetic (CPU): the algorithmic FLOP count
follows the method, not the storage order; its depth table is the device's;
the per-event figures stay where the design puts them; and the bench refuses
more than one GPU."""
import os
import re
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1706_01420_amd import workloads as W  # noqa: E402


def _header_table():
    txt = open(os.path.join(ROOT, "paper_1706_01420_amd", "csrc", "cf_depth.h")).read()
    skip = float(re.search(r"kCfSkipE\s*=\s*([0-9.]+)", txt).group(1))
    body = re.search(r"kCfDepthE\[\d+\]\s*=\s*\{([^}]*)\}", txt).group(1)
    vals = [float(v) for v in body.replace("\n", " ").split(",") if v.strip()]
    return skip, vals


def test_depth_table_is_the_devices():
    skip, vals = _header_table()
    assert bench.CORR_SKIP == skip
    assert bench.CF_DEPTH_E == vals[:-1]          # the last entry is the always-accepted full depth
    assert all(a > b for a, b in zip(bench.CF_DEPTH_E, bench.CF_DEPTH_E[1:]))


def test_lane_depths_follow_the_exponent():
    x = np.array([-1.0, 0.0, 1.0, 2.5, 3.0, 4.0, 4.5, 5.0, 6.0, 7.0, 50.0])
    need, depth = bench._lane_depths(x, 0.0, 0.0)
    E = np.where(x > 0.0, x * x, -1.0)
    assert np.array_equal(need, E < bench.CORR_SKIP)
    # depth is one plus the number of thresholds above E: monotone, 1 .. 10
    assert np.all(np.diff(depth[x > 0.0]) <= 0)
    assert depth.min() >= 1 and depth.max() <= 10
    assert depth[0] == 10 and depth[1] == 10          # no positive Im u: the full depth
    for e, d in zip(E, depth):
        assert d == 1 + sum(e < th for th in bench.CF_DEPTH_E)


def test_flop_count_ignores_the_storage_order():
    n = 200_000
    cols, _ = W.events(3, n)
    th = np.array(W.THETA_GEN[3])
    f0 = bench.algorithmic_flops(3, cols[3], cols[4], th, True)
    perm = np.random.default_rng(5).permutation(n)
    f1 = bench.algorithmic_flops(3, cols[3][perm], cols[4][perm], th, True)
    assert f0 == f1
    cols2, _ = W.events(2, n)
    th2 = np.array(W.THETA_GEN[2])
    g0 = bench.algorithmic_flops(2, cols2[1], cols2[2], th2, False)
    perm2 = np.random.default_rng(6).permutation(n)
    assert bench.algorithmic_flops(2, cols2[1][perm2], cols2[2][perm2], th2, False) == g0


def test_per_event_counts_of_the_workloads():
    # the figures the design quotes for the workloads' sigma_t ~ U(0.03, 0.06) ps
    n = 400_000
    cols, _ = W.events(3, n)
    th = np.array(W.THETA_GEN[3])
    grad = bench.algorithmic_flops(3, cols[3], cols[4], th, True) / n
    nll = bench.algorithmic_flops(3, cols[3], cols[4], th, False) / n
    assert abs(grad - 870.0) < 3.0, grad
    assert abs(nll - 665.0) < 3.0, nll
    assert abs((grad - nll) - (bench.FLOP_BASE[(3, True)] - bench.FLOP_BASE[(3, False)])) < 1e-9
    cols2, _ = W.events(2, n)
    th2 = np.array(W.THETA_GEN[2])
    assert abs(bench.algorithmic_flops(2, cols2[1], cols2[2], th2, True) / n - 460.0) < 3.0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
