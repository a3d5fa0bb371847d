"""Served likelihood (persistent device loop): every result equals the plain
nll_eval / nll_grad on the same dataset bitwise, alone and in mixed traffic;
admission waits for scratch memory; errors stay with their request."""
import sys
import threading
import time

import numpy as np
import pytest

from oracle import models as M
from oracle import nll as N
from paper_1706_01420_amd import workloads as W

pytestmark = pytest.mark.gpu


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


DATASET_SIZES = ((1, [1000, 50000]), (2, [777, 40000]), (3, [1, 5000, 100000]))


@pytest.fixture(scope="module")
def datasets(lib, ctx):
    out = []
    for model, sizes in DATASET_SIZES:
        for j, n in enumerate(sizes):
            cols, w = W.events(model, n, seed=300 + 10 * model + j)
            out.append((model, lib.ipx_dataset_create(ctx, model, cols, w)))
    yield out
    for _, d in out:
        lib.ipx_dataset_destroy(ctx, d)


def _theta(model, rng):
    base = np.array(M.THETA_GEN[model])
    while True:
        th = base * (1.0 + 0.02 * rng.standard_normal(base.size))
        if M.theta_valid(model, th):
            return th


def _plain(lib, ctx, d, th, grad):
    if grad:
        return lib.nll_grad(ctx, d, th)
    return lib.nll_eval(ctx, d, th), None


def test_single_requests_equal_plain_calls(lib, ctx, datasets):
    srv = lib.ipx_server_start(ctx, slots=8)
    try:
        rng = np.random.default_rng(1)
        for model, d in datasets:
            for grad in (False, True):
                th = _theta(model, rng)
                say("serve single model", model, "grad", grad)
                t = lib.ipx_submit(srv, d, th, grad)
                r = lib.ipx_wait(srv, t, 60.0)
                f, g = _plain(lib, ctx, d, th, grad)
                assert r["status"] == 0 and r["nll"] == f
                if grad:
                    assert np.array_equal(r["grad"], g)
                assert r["latency_us"] > 0
        # two served requests directly against the oracle
        for model, j in ((2, 0), (3, 1)):
            n = DATASET_SIZES[model - 1][1][j]
            cols, w = W.events(model, n, seed=300 + 10 * model + j)
            d = [dd for mm, dd in datasets if mm == model][j]
            th = _theta(model, rng)
            r = lib.ipx_wait(srv, lib.ipx_submit(srv, d, th, True), 60.0)
            fref, gref = N.nll_grad(model, cols, th, w)
            assert abs(r["nll"] - fref) <= 1e-10 * abs(fref), (model, r["nll"], fref)
            scale = np.abs(N.event_grad(model, cols, th) * (1.0 if w is None else w)).sum(axis=1)
            bound = 1e-6 * np.abs(gref) + 1e-9 * scale + 1e-13 * n
            assert np.all(np.abs(r["grad"] - gref) <= bound), (model, r["grad"], gref)
    finally:
        lib.ipx_server_stop(srv)


@pytest.mark.parametrize("policy", [0, 1, 2])
def test_mixed_concurrent_traffic_is_bitwise_equal_to_alone(lib, ctx, datasets, policy):
    srv = lib.ipx_server_start(ctx, slots=16, policy=policy)
    rng = np.random.default_rng(2)
    jobs = []
    for i in range(160):
        model, d = datasets[rng.integers(len(datasets))]
        jobs.append((d, _theta(model, rng), bool(rng.integers(2))))
    results = [None] * len(jobs)

    def client(k):
        for i in range(k, len(jobs), 8):
            d, th, grad = jobs[i]
            t = lib.ipx_submit(srv, d, th, grad)
            if i % 3 == 0:                      # some clients poll
                deadline = time.time() + 60
                r = None
                while r is None and time.time() < deadline:
                    r = lib.ipx_poll(srv, t)
                results[i] = r
            else:
                results[i] = lib.ipx_wait(srv, t, 60.0)
    try:
        say("serve mixed traffic 160 requests, 8 client threads, policy", policy)
        threads = [threading.Thread(target=client, args=(k,)) for k in range(8)]
        for th in threads:
            th.start()
        for th in threads:
            th.join(120)
        assert all(r is not None for r in results)
    finally:
        lib.ipx_server_stop(srv)
    for (d, th, grad), r in zip(jobs, results):
        f, g = _plain(lib, ctx, d, th, grad)
        assert r["status"] == 0 and r["nll"] == f
        if grad:
            assert np.array_equal(r["grad"], g)


def test_admission_by_scratch_budget(lib, ctx, datasets):
    model, d = datasets[-1]          # angular, 100000 events
    need = (52 * 98 * 8 + 255) // 256 * 256   # the tile partials of 98 tiles, 256-byte aligned
    srv = lib.ipx_server_start(ctx, slots=8, scratch_bytes=need + 1024)
    try:
        rng = np.random.default_rng(3)
        ths = [_theta(3, rng) for _ in range(6)]
        say("serve admission, budget for one angular gradient request")
        tickets = [lib.ipx_submit(srv, d, th, True) for th in ths]
        for th, t in zip(ths, tickets):
            r = lib.ipx_wait(srv, t, 60.0)
            f, g = lib.nll_grad(ctx, d, th)
            assert r["nll"] == f and np.array_equal(r["grad"], g)
        big = lib.ipx_dataset_create(ctx, 3, *W.events(3, 400000, seed=5))
        try:
            with pytest.raises(lib.IpxError) as e:
                lib.ipx_submit(srv, big, ths[0], True)
            assert e.value.status == lib.IPX_ENOMEM
        finally:
            lib.ipx_dataset_destroy(ctx, big)
    finally:
        lib.ipx_server_stop(srv)


def test_errors_stay_with_their_request_and_idle_relaunch(lib, ctx, datasets):
    model, d = datasets[0]
    srv = lib.ipx_server_start(ctx, slots=4, idle_iterations=50)
    try:
        say("serve domain error + idle relaunch")
        good = np.array(M.THETA_GEN[1])
        bad = good.copy()
        bad[0] = 2.0
        t1 = lib.ipx_submit(srv, d, bad, True)
        t2 = lib.ipx_submit(srv, d, good, True)
        r1 = lib.ipx_wait(srv, t1, 60.0)
        r2 = lib.ipx_wait(srv, t2, 60.0)
        assert r1["status"] == lib.IPX_EDOMAIN and r1["nll"] == np.inf
        f, g = lib.nll_grad(ctx, d, good)
        assert r2["nll"] == f and np.array_equal(r2["grad"], g)
        time.sleep(0.5)                   # the device loop has exited by now
        t3 = lib.ipx_submit(srv, d, good, False)
        assert lib.ipx_wait(srv, t3, 60.0)["nll"] == lib.nll_eval(ctx, d, good)
        with pytest.raises(lib.IpxError):
            lib.ipx_poll(srv, 987654321)
    finally:
        lib.ipx_server_stop(srv)


def test_cancel_withdraws_waiting_requests(lib, ctx, datasets):
    """One slot and a queue of large gradient requests: the late ones are
    still waiting when cancelled (IPX_OK, result status IPX_ECANCELED); a
    request on the device or finished is not (IPX_EBUSY) and completes with
    the plain call's result; a taken ticket is unknown (IPX_ENOTFOUND)."""
    model, d = max(datasets, key=lambda md: (md[0] == 3, lib.ipx_dataset_size(md[1])))
    th = np.array(M.THETA_GEN[model])
    f, g = lib.nll_grad(ctx, d, th)
    srv = lib.ipx_server_start(ctx, slots=1)
    try:
        say("serve cancel")
        tickets = [lib.ipx_submit(srv, d, th, True) for _ in range(12)]
        cancelled = []
        for t in tickets[::-1][:6]:
            try:
                lib.ipx_cancel(srv, t)
                cancelled.append(t)
            except lib.IpxError as err:
                assert err.status == lib.IPX_EBUSY
        assert cancelled, "every request had reached the device"
        with pytest.raises(lib.IpxError) as e:
            lib.ipx_cancel(srv, tickets[0])          # on the device or finished
        assert e.value.status == lib.IPX_EBUSY
        for t in tickets:
            r = lib.ipx_wait(srv, t, 60.0)
            if t in cancelled:
                assert r["status"] == lib.IPX_ECANCELED and r["nll"] == np.inf
            else:
                assert r["status"] == 0 and r["nll"] == f and np.array_equal(r["grad"], g)
        with pytest.raises(lib.IpxError) as e:
            lib.ipx_cancel(srv, tickets[-1])         # taken
        assert e.value.status == lib.IPX_ENOTFOUND
        assert lib.ipx_server_stats_read(srv)["cancelled"] == len(cancelled)
    finally:
        lib.ipx_server_stop(srv)


def test_drain_then_stop_with_blocked_waiters(lib, ctx, datasets):
    """ipx_server_drain finishes every request submitted before it (with two
    slots, most of the six wait for a slot when it is called): afterwards
    every ticket polls done, with the plain call's bits.  Clients waiting in ipx_wait on other threads get
    their results; the server stops cleanly after them."""
    import threading
    model, d = datasets[-1]
    srv = lib.ipx_server_start(ctx, slots=2)
    th = np.array(M.THETA_GEN[3])
    say("serve drain")
    stopped = False
    try:
        tickets = [lib.ipx_submit(srv, d, th, True) for _ in range(6)]
        lib.ipx_server_drain(srv)
        st = lib.ipx_server_stats_read(srv)
        assert st["published"] == 6 and st["completed"] == 6
        assert st["pending"] == 0 and st["in_flight"] == 0
        f, g = lib.nll_grad(ctx, d, th)
        for t in tickets:
            r = lib.ipx_poll(srv, t)          # done: never IPX_EBUSY after the drain
            assert r["status"] == 0 and r["nll"] == f and np.array_equal(r["grad"], g)
        # waiters blocked on their own tickets while the server drains and stops
        tickets = [lib.ipx_submit(srv, d, th, bool(i % 2)) for i in range(8)]
        got = {}

        def waiter(t):
            got[t] = lib.ipx_wait(srv, t, 60.0)

        threads = [threading.Thread(target=waiter, args=(t,)) for t in tickets]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        say("serve stop")
        lib.ipx_server_stop(srv)
        stopped = True
        assert sorted(got) == sorted(tickets)
        f0 = lib.nll_eval(ctx, d, th)
        for i, t in enumerate(tickets):
            assert got[t]["status"] == 0
            assert got[t]["nll"] == (f if i % 2 else f0)
    finally:
        if not stopped:
            lib.ipx_server_stop(srv)


def test_two_workgroups_and_counters(lib, ctx, datasets):
    # one poller and one worker: the worker takes every per-event tile before
    # the coefficient-adjoint tiles, so the angular gradient needs no second
    # workgroup; the host counters account for every request
    with pytest.raises(lib.IpxError):
        lib.ipx_server_start(ctx, workgroups=1)
    srv = lib.ipx_server_start(ctx, slots=4, workgroups=2)
    try:
        rng = np.random.default_rng(7)
        n = 0
        for model, d in datasets:
            th = _theta(model, rng)
            say("serve two workgroups model", model)
            r = lib.ipx_wait(srv, lib.ipx_submit(srv, d, th, True), 60.0)
            f, g = _plain(lib, ctx, d, th, True)
            assert r["status"] == 0 and r["nll"] == f and np.array_equal(r["grad"], g)
            n += 1
        st = lib.ipx_server_stats_read(srv)
        assert st["published"] == n and st["completed"] == n
        assert st["pending"] == 0 and st["in_flight"] == 0 and st["launches"] >= 1
    finally:
        lib.ipx_server_stop(srv)
