"""The first layers of a circuit in one launch (ST_TOP, GKR_OMEGA_TABLES)
against the oracle and against the same tables layer by layer
(GKR_OMEGA_TABLES_STEPWISE): where the fused region ends (a wire with more
than one chunk of gates, a one-gate layer, a layer wider than 1024 values),
a whole circuit fused, mixed gate types, repeated proofs on one workspace,
and the host-memory placement and batches that run it too."""
import random

import numpy as np
import pytest

from gpu_util import say, device_tensor, oracle_threads
from oracle import oracle as O
import workloads as W
from workloads.circuits import Circuit

P = (1 << 61) - 1
pytestmark = pytest.mark.gpu


def G():
    import paper_1202_1350_amd as mod
    return mod


def layered(rng, sizes, fanout_at=None, fan=40, kinds=None):
    """Random wiring; at layer fanout_at one wire of the next layer feeds fan
    gates (more than one chunk of 32)."""
    d = len(sizes) - 1
    types, in1, in2 = [], [], []
    for i in range(d):
        lim = 1 << (sizes[i + 1] - 1).bit_length() if sizes[i + 1] > 1 else 1
        a = [rng.randrange(min(lim, sizes[i + 1])) for _ in range(sizes[i])]
        b = [rng.randrange(lim) for _ in range(sizes[i])]
        if i == fanout_at:
            assert sizes[i] >= fan
            for g in range(fan):
                a[g] = 0
        t = [rng.randrange(2) for _ in range(sizes[i])] if kinds is None else [kinds[i]] * sizes[i]
        types.append(np.array(t, np.uint8))
        in1.append(np.array(a, np.uint32))
        in2.append(np.array(b, np.uint32))
    return Circuit(list(sizes), types, in1, in2, name=f"layered {sizes} fan-out at {fanout_at}")


def prove_all(circ, x, seeds, device=False):
    O.set_threads(oracle_threads())
    want = {sd: O.prove(circ, x, sd) for sd in seeds}
    inp = device_tensor(x) if device else x
    for algo in (G().GKR_OMEGA_TABLES, G().GKR_OMEGA_TABLES_STEPWISE):
        gc = G().Circuit.from_workload(circ, omega_algo=algo)
        for sd in seeds:  # consecutive proofs on one workspace and graph
            say(circ.name, "algo", algo, "seed", sd)
            m, c = G().gkr_prove(gc, inp, sd)
            bad = np.nonzero(m != want[sd][0])[0]
            assert len(bad) == 0, (circ.name, algo, sd, bad[:5])
            assert np.array_equal(c, want[sd][1])
            assert G().gkr_verify(gc, inp, sd, m)[0]


@pytest.mark.parametrize("case", [
    ([1, 2, 4, 8, 64, 200, 700], None),        # fused throughout
    ([1, 3, 6, 50, 100, 30, 9], 3),            # a wire with 40 gates in layer 3 ends the region
    ([3, 60, 7, 1000, 1000, 5], 1),            # ... in layer 1
    ([4, 2, 1, 5, 9], None),                   # a one-gate layer ends it
    ([2, 1000, 1024, 1025, 700, 3], None),     # layer 2 reads 1025 values
    ([1, 1024, 1024, 1024], None),             # full 1024-value layers
])
def test_fused_region_boundaries(case):
    sizes, fan_at = case
    rng = random.Random(sum(sizes))
    circ = layered(rng, sizes, fan_at)
    x = np.array([rng.randrange(P) for _ in range(sizes[-1])], np.uint64)
    prove_all(circ, x, (3, 4))


@pytest.mark.parametrize("kinds", [[0] * 6, [1] * 6, [0, 1, 0, 1, 1, 0]])
def test_fused_gate_kinds(kinds):
    rng = random.Random(len(kinds) + sum(kinds))
    circ = layered(rng, [2, 9, 33, 130, 513, 1000, 77], None, kinds=kinds)
    x = np.array([rng.randrange(P) for _ in range(77)], np.uint64)
    prove_all(circ, x, (5,), device=True)


def test_fused_f2_circuits():
    for n in (1 << 10, 1 << 11, 5000):
        prove_all(W.f2_circuit(n), W.f2_inputs(n, 12), (12, 13), device=True)


def test_fused_in_host_memory_and_batches():
    O.set_threads(oracle_threads())
    items = [(W.f2_circuit(1 << 10), W.f2_inputs(1 << 10, 1), 7),
             (W.pm_f0_circuit(1 << 6, 4), W.pm_inputs(1 << 6, 2, 4)[0], 8),
             (W.f0_circuit(1 << 8), W.f0_inputs(1 << 8, 3), 9)]
    want = [O.prove(c, x, sd)[0] for c, x, sd in items]
    circs = [G().Circuit.from_workload(c) for c, _, _ in items]
    say("batch with fused top layers")
    got = G().gkr_batch_prove(circs, [device_tensor(x) for _, x, _ in items], [sd for _, _, sd in items])
    for g, w in zip(got, want):
        assert np.array_equal(g, w)
    for gc, (c, x, sd), w in zip(circs, items, want):
        say("copy every message, fused top layers", c.name)
        gc.set_memory(G().GKR_MEM_MESSAGE)
        assert np.array_equal(G().gkr_prove(gc, x, sd)[0], w)
