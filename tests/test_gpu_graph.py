"""gkr_prove replays a captured graph of the proof's launches (one per
workspace and plan).  Every replay is checked against the launch-by-launch
path (taken while per-launch profiling is on) and the oracle, with other
proofs and host synchronisation between the replays, and after a re-plan."""
import numpy as np
import pytest

from gpu_util import say, device_tensor, oracle_threads
from oracle import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def G():
    import paper_1202_1350_amd as mod
    return mod


def eager(gc, x, seed):
    g = G()
    g.gkr_profile_read()
    g.gkr_profile_enable(True)
    try:
        return g.gkr_prove(gc, x, seed)
    finally:
        g.gkr_profile_enable(False)
        g.gkr_profile_read()


def test_graph_replays_match_eager_and_oracle():
    import torch
    g = G()
    circ, x, seed = W.c2_f2(10)
    other, y, oseed = W.c3_matmult(8)
    gc = g.Circuit.from_workload(circ)
    go = g.Circuit.from_workload(other)
    O.set_threads(oracle_threads())
    want_m, want_c = O.prove(circ, x, seed)
    em, ec = eager(gc, x, seed)
    assert np.array_equal(em, want_m) and np.array_equal(ec, want_c)
    xt = device_tensor(x)
    for rep in range(4):
        say("graph replay", rep)
        m, c = g.gkr_prove(gc, xt if rep % 2 else x, seed)
        assert np.array_equal(m, em), f"replay {rep}: transcript differs from the eager path"
        assert np.array_equal(c, ec), f"replay {rep}: challenges differ"
        g.gkr_prove(go, y, oseed + rep)  # another circuit's proof in between
        torch.cuda.synchronize()
    # another seed and other inputs through the same graph
    x2 = (x.astype(np.uint64) * 3 + 1) % ((1 << 61) - 1)
    m2, c2 = g.gkr_prove(gc, x2, seed + 7)
    w2m, w2c = O.prove(circ, x2, seed + 7)
    assert np.array_equal(m2, w2m) and np.array_equal(c2, w2c)


def test_graph_recaptured_after_replan():
    g = G()
    circ, x, seed = W.c2_f2(11)
    gc = g.Circuit.from_workload(circ)
    m0, c0 = g.gkr_prove(gc, x, seed)
    saved = g.gkr_tune_get()
    try:
        g.gkr_autotune([gc], [x], reps=1)  # new launch shapes: the plan and its graph are rebuilt
        m1, c1 = g.gkr_prove(gc, x, seed)
        assert np.array_equal(m1, m0) and np.array_equal(c1, c0)
    finally:
        g.gkr_tune_set(saved)
    m2, c2 = g.gkr_prove(gc, x, seed)
    assert np.array_equal(m2, m0) and np.array_equal(c2, c0)
