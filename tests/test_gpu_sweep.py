"""GPU parity over a wide parameter sweep and per event, at the full workload
sizes (10^5 / 2x10^6 / 4x10^6 events, resolution-band storage order, the
launch configuration the benchmark times).

  * Sweep: 20 random points inside each model's limits plus the edge points
    of tests/theta_sweep.py; NLL (relative 1e-10) and gradient (the bound of
    test_gpu_parity.check_grad) against the oracle's values stored by
    tests/golden/make_theta_sweep.py for the same seeded samples (their
    SHA-256 is checked first).
  * Per event: ipx_event_logp against the oracle's w_i ln P_i on the events
    as stored (the band permutation read back from the dataset), element by
    element: |got - ref| <= 1e-12 max(1, |ref|).  Every factor of P is
    evaluated with a relative error of a few units in the last place (the
    elementary functions <= 3 ulp, the Faddeeva corrections ~1e-13 of a
    term that is itself <= 6e-7 of the main term), so ln P carries an
    absolute error of ~1e-15 and the bound leaves a factor of ~100.
  * Gradient domain: on the boundary where an amplitude modulus vanishes the
    gradient forms return IPX_EDOMAIN (+inf, NaN), the NLL does not.
"""
import hashlib
import json
import math
import os
import sys

import numpy as np
import pytest

import theta_sweep
from storage_order import band_order

from oracle import models as M
from oracle import nll as N
from paper_1706_01420_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD_PATH = os.path.join(HERE, "golden", "theta_sweep.json")
EVENT_TOL = 1e-12


def say(*a):
    print("[gpu]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def lib():
    from paper_1706_01420_amd import ipx
    return ipx


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.ipx_create(0)
    yield c
    lib.ipx_destroy(c)


@pytest.fixture(scope="module")
def gold():
    with open(GOLD_PATH) as fh:
        return json.load(fh)


def data_hash(cols, w):
    h = hashlib.sha256()
    for c in cols:
        h.update(np.ascontiguousarray(c, np.float64).tobytes())
    if w is not None:
        h.update(np.ascontiguousarray(w, np.float64).tobytes())
    return h.hexdigest()


@pytest.mark.parametrize("model", [1, 2, 3])
def test_sweep_nll_and_gradient_at_full_size(lib, ctx, gold, model):
    g = gold[str(model)]
    cols, w = W.events(model, g["n"])
    assert data_hash(cols, w) == g["data_sha256"], "the stored oracle values belong to other input draws"
    ds = lib.ipx_dataset_create(ctx, model, cols, w)
    n = g["n"]
    try:
        for p in g["points"]:
            th = np.array(p["theta"])
            say("sweep model", model, p["label"])
            f = lib.nll_eval(ctx, ds, th)
            assert math.isfinite(f)
            assert abs(f - p["nll"]) <= 1e-10 * abs(p["nll"]), (p["label"], f, p["nll"])
            fg, gg = lib.nll_grad(ctx, ds, th)
            if p["grad_defined"]:
                assert fg == f
                gref, scale = np.array(p["grad"]), np.array(p["grad_scale"])
                bound = 1e-6 * np.abs(gref) + 1e-9 * scale + 1e-13 * n
                assert np.all(np.abs(gg - gref) <= bound), (p["label"], gg, gref,
                                                            np.abs(gg - gref) / bound)
            else:
                assert fg == math.inf and np.all(np.isnan(gg)), p["label"]
    finally:
        lib.ipx_dataset_destroy(ctx, ds)


def _stored(lib, ctx, ds, model, weighted):
    cols = [lib.ipx_dataset_read(ctx, ds, c) for c in range(M.NCOLS[model])]
    w = lib.ipx_dataset_read(ctx, ds, M.NCOLS[model]) if weighted else None
    return cols, w


def _check_events(got, ref, label):
    err = np.abs(got - ref)
    bound = EVENT_TOL * np.maximum(1.0, np.abs(ref))
    worst = int(np.argmax(err / bound))
    say("  max |got - ref| %.3g, worst ratio to the bound %.3g at event %d" % (err.max(), err[worst] / bound[worst],
                                                                             worst))
    assert np.all(err <= bound), (label, worst, got[worst], ref[worst])


@pytest.mark.parametrize("model", [1, 2, 3])
def test_per_event_terms_match_oracle_at_full_size(lib, ctx, model):
    n = W.WORKLOAD_SIZES[model]
    cols, w = W.events(model, n)
    ds = lib.ipx_dataset_create(ctx, model, cols, w)
    try:
        sc, sw = _stored(lib, ctx, ds, model, w is not None)
        if model >= 2:
            tcol, scol = (1, 2) if model == 2 else (3, 4)
            order = band_order(cols[tcol], cols[scol])
            for c in range(len(cols)):
                assert np.array_equal(sc[c], cols[c][order])
        edge = {1: "lambda=0", 2: "s=0.5", 3: "Delta m=30"}[model]
        th_edge = [t for lab, t, _ in theta_sweep.points(model) if lab == edge][0]
        for label, th in (("gen", M.THETA_GEN[model]), (edge, th_edge)):
            say("per-event terms model", model, label, "n", n)
            got = lib.ipx_event_logp(ctx, ds, th).cpu().numpy()
            ref = N.log_pdf(model, sc, th) * (1.0 if sw is None else sw)
            _check_events(got, ref, label)
            # the hook's terms are the ones the evaluation sums
            f = lib.nll_eval(ctx, ds, th)
            assert abs(-math.fsum(got.tolist()) - f) <= 1e-12 * abs(f)
    finally:
        lib.ipx_dataset_destroy(ctx, ds)


@pytest.mark.parametrize("model", [2, 3])
def test_per_event_terms_at_resolution_extremes(lib, ctx, model):
    """sigma_t log-uniform over [0.002, 0.5] ps, in input order: every event's
    term against the oracle where the corrections are skipped, at every
    continued-fraction depth, on the rational-series branch (Im u < 3.4) and,
    for the complex rate, at |u| >= 6 with E < 0."""
    n = 20000
    cols, w = W.events(model, n, seed=131)
    scol = 2 if model == 2 else 4
    cols = [c.copy() for c in cols]
    cols[scol] = np.exp(np.random.default_rng(132).uniform(np.log(0.002), np.log(0.5), n))
    ds = lib.ipx_dataset_create(ctx, model, cols, w, flags=lib.IPX_COPY_HOST | lib.IPX_KEEP_ORDER)
    try:
        for label, th in (("gen", M.THETA_GEN[model]), theta_sweep.points(model)[3][:2]):
            say("per-event terms at resolution extremes, model", model, label)
            got = lib.ipx_event_logp(ctx, ds, th).cpu().numpy()
            _check_events(got, N.log_pdf(model, cols, th) * (1.0 if w is None else w), label)
    finally:
        lib.ipx_dataset_destroy(ctx, ds)


@pytest.mark.parametrize("model", [1, 2, 3])
@pytest.mark.parametrize("n", [0, 1, 63, 65, 1025])
def test_per_event_terms_small_and_ragged(lib, ctx, model, n):
    cols, w = W.events(model, max(n, 1), seed=100 + n)
    cols = [c[:n] for c in cols]
    w = None if w is None else w[:n]
    ds = lib.ipx_dataset_create(ctx, model, cols, w, flags=lib.IPX_COPY_HOST | lib.IPX_KEEP_ORDER)
    try:
        th = theta_sweep.points(model)[3][1]
        say("per-event terms model", model, "n", n)
        got = lib.ipx_event_logp(ctx, ds, th).cpu().numpy()
        assert got.shape == (n,)
        if n:
            _check_events(got, N.log_pdf(model, cols, th) * (1.0 if w is None else w), "n=%d" % n)
        bad = list(M.THETA_GEN[model])
        bad[0] = 1.5 if model < 3 else 0.9   # f > 1, or fL + fperp > 1
        with pytest.raises(lib.IpxError) as e:
            lib.ipx_event_logp(ctx, ds, bad)
        assert e.value.status == lib.IPX_EDOMAIN
    finally:
        lib.ipx_dataset_destroy(ctx, ds)


def test_gradient_domain_boundary_in_every_form(lib, ctx):
    cols, w = W.events(3, 5000, seed=41)
    ds = lib.ipx_dataset_create(ctx, 3, cols, w)
    ds2 = lib.ipx_dataset_create(ctx, 3, [c[:3000] for c in cols], w[:3000])
    edge = list(M.THETA_GEN[3])
    edge[2] = 0.0                                   # Fs = 0
    try:
        say("gradient domain: plain, batched, served")
        f = lib.nll_eval(ctx, ds, edge)
        assert abs(f - N.nll(3, cols, edge, w)) <= 1e-10 * abs(f)
        fg, gg = lib.nll_grad(ctx, ds, edge)
        assert fg == math.inf and np.all(np.isnan(gg))
        plan = lib.ipx_plan_create(ctx, [ds, ds2])
        try:
            th = np.array([edge, M.THETA_GEN[3]])
            nll, g = lib.nll_eval_batch(ctx, plan, th, grad=True)
            assert nll[0] == math.inf and np.all(np.isnan(g[0]))
            f2, g2 = lib.nll_grad(ctx, ds2, M.THETA_GEN[3])
            assert nll[1] == f2 and np.array_equal(g[1], g2)
            assert np.array_equal(lib.nll_eval_batch(ctx, plan, th), [f, lib.nll_eval(ctx, ds2, M.THETA_GEN[3])])
        finally:
            lib.ipx_plan_destroy(plan)
        srv = lib.ipx_server_start(ctx, slots=4)
        try:
            r_grad = lib.ipx_wait(srv, lib.ipx_submit(srv, ds, edge, True), 30.0)
            r_nll = lib.ipx_wait(srv, lib.ipx_submit(srv, ds, edge, False), 30.0)
        finally:
            lib.ipx_server_stop(srv)
        assert r_grad["status"] == lib.IPX_EDOMAIN and r_grad["nll"] == math.inf
        assert r_nll["status"] == lib.IPX_OK and r_nll["nll"] == f
    finally:
        lib.ipx_dataset_destroy(ctx, ds)
        lib.ipx_dataset_destroy(ctx, ds2)
