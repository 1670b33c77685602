"""Serving with continuous batching: requests submitted while others run
join the in-flight launches; every transcript equals the oracle's; the HBM
budget bounds admission; an impossible budget fails cleanly."""
import random
import time

import numpy as np
import pytest

from gpu_util import say, oracle_threads
from oracle import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def G():
    import paper_1202_1350_amd as mod
    return mod


def wait_all(srv, ids, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(ids):
        for rid in ids:
            if rid in out:
                continue
            done, m, lat = srv.poll(rid)
            if done:
                out[rid] = (m, lat)
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.001)
    return out


def test_served_results_equal_oracle_in_a_mix():
    O.set_threads(oracle_threads())
    shapes = [("F2", W.f2_circuit(1 << k)) for k in (6, 10, 12, 14)] + \
             [("PM", W.pm_circuit(1 << 10)), ("MM", W.matmult_circuit(8)), ("MM", W.matmult_circuit(16))]
    circs = [(name, c, G().Circuit.from_workload(c)) for name, c in shapes]
    rng = random.Random(5)
    reqs = []
    for k in range(40):
        name, c, gc = circs[rng.randrange(len(circs))]
        if name == "F2":
            x = W.f2_inputs(c.sizes[-1], 1000 + k)
        elif name == "PM":
            x = W.pm_inputs(1 << 10, 1000 + k)[0]
        else:
            N = int(round((c.sizes[-1] // 2) ** 0.5))
            x = W.matmult_inputs(N, 1000 + k)
        reqs.append((c, gc, x, 77 + k))
    srv = G().Server(8 << 30, 12)
    try:
        ids = []
        say("serve: first wave")
        for c, gc, x, sd in reqs[:20]:
            ids.append(srv.submit(gc, x, sd))
        time.sleep(0.002)  # the second wave arrives while the first runs
        say("serve: second wave")
        for c, gc, x, sd in reqs[20:]:
            ids.append(srv.submit(gc, x, sd))
        res = wait_all(srv, ids)
    finally:
        srv.close()
    for (c, gc, x, sd), rid in zip(reqs, ids):
        want, _ = O.prove(c, x, sd)
        m, lat = res[rid]
        assert np.array_equal(m, want)
        assert lat > 0


def test_tiny_budget_fails_cleanly():
    c = W.f2_circuit(1 << 10)
    gc = G().Circuit.from_workload(c)
    srv = G().Server(1 << 10, 4)  # 1 KiB: no proof fits
    try:
        rid = srv.submit(gc, W.f2_inputs(1 << 10, 1), 1)
        t0 = time.time()
        while True:
            try:
                done, _, _ = srv.poll(rid)
            except G().GkrError as e:
                assert e.code == G().GKR_ERR_NOMEM
                break
            assert not done, "a proof ran beyond the budget"
            assert time.time() - t0 < 30
            time.sleep(0.001)
    finally:
        srv.close()


def test_budget_limits_scratch_in_use():
    c = W.f2_circuit(1 << 12)
    gc = G().Circuit.from_workload(c)
    probe = G().Server(1 << 34, 1)
    try:
        wait_all(probe, [probe.submit(gc, W.f2_inputs(1 << 12, 0), 0)])
        one = probe.stats()[2]  # scratch of one proof, now pooled
    finally:
        probe.close()
    assert one > 0
    budget = int(2.5 * one)  # room for two proofs at a time
    srv = G().Server(budget, 16)
    try:
        say("serve: budget for two proofs, 10 requests")
        ids = [srv.submit(gc, W.f2_inputs(1 << 12, k), k) for k in range(10)]
        peak_used, peak_running = 0, 0
        t0 = time.time()
        while True:
            assert time.time() - t0 < 60, "server stalled"
            running, queued, used = srv.stats()
            peak_used = max(peak_used, used)
            peak_running = max(peak_running, running)
            if running == 0 and queued == 0:
                break
            time.sleep(0.0002)
        res = wait_all(srv, ids)
        assert peak_used <= budget and peak_running <= 2
        for k in (0, 3, 9):
            want, _ = O.prove(c, W.f2_inputs(1 << 12, k), k)
            assert np.array_equal(res[ids[k]][0], want)
    finally:
        srv.close()


def test_destroyed_circuit_releases_pooled_scratch():
    """Idle pooled scratch refers to its circuit's device arrays: destroying
    the circuit frees it, and a circuit created afterwards (possibly at the
    same address) gets scratch of its own shape."""
    import gc
    O.set_threads(oracle_threads())
    srv = G().Server(8 << 30, 4)
    try:
        ca = W.f2_circuit(1 << 12)
        ga = G().Circuit.from_workload(ca)
        say("serve: circuit A then destroy it")
        wait_all(srv, [srv.submit(ga, W.f2_inputs(1 << 12, 1), 1)])
        assert srv.stats()[2] > 0
        del ga
        gc.collect()
        assert srv.stats()[2] == 0, "pooled scratch of a destroyed circuit kept"
        cb = W.pm_circuit(1 << 10)
        xb = W.pm_inputs(1 << 10, 3)[0]
        for k in range(3):
            gb = G().Circuit.from_workload(cb)
            say("serve: circuit B after A was destroyed, round", k)
            m = wait_all(srv, [rid := srv.submit(gb, xb, 9 + k)])[rid][0]
            assert np.array_equal(m, O.prove(cb, xb, 9 + k)[0])
            del gb
            gc.collect()
    finally:
        srv.close()


def test_algorithm_change_discards_pooled_scratch():
    O.set_threads(oracle_threads())
    c = W.matmult_circuit(8)
    x = W.matmult_inputs(8, 4)
    gc_ = G().Circuit.from_workload(c)
    srv = G().Server(8 << 30, 4)
    try:
        for algo in (G().GKR_OMEGA_TABLES, G().GKR_OMEGA_GATES, G().GKR_OMEGA_TABLES):
            gc_.set_algorithm(algo)
            say("serve: omega algorithm", algo)
            m = wait_all(srv, [rid := srv.submit(gc_, x, 5)])[rid][0]
            assert np.array_equal(m, O.prove(c, x, 5)[0])
    finally:
        srv.close()
