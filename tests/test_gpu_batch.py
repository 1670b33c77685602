"""Batched proving (many proofs per launch, optionally replayed from a HIP
graph): every transcript equals the oracle's for the same circuit, inputs
and seed, whatever else is in the batch."""
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


def mixed_batch():
    rng = random.Random(8)
    items = []
    for n in (1, 7, 1 << 10, 3000, 1 << 14):
        items.append((W.f2_circuit(n), W.f2_inputs(n, 100 + n)))
    for n in (9, 300, 1 << 12):
        c = W.pm_circuit(n)
        items.append((c, W.pm_inputs(n, 200 + n)[0]))
    for N in (2, 16):
        items.append((W.matmult_circuit(N), W.matmult_inputs(N, 300 + N)))
    # a random mixed-gate circuit with padding wires
    sizes = [5, 77, 300, 1000]
    types, in1, in2 = [], [], []
    for i in range(3):
        lim = 1 << (sizes[i + 1] - 1).bit_length()
        types.append(np.array([rng.randrange(2) for _ in range(sizes[i])], np.uint8))
        in1.append(np.array([rng.randrange(lim) for _ in range(sizes[i])], np.uint32))
        in2.append(np.array([rng.randrange(lim) for _ in range(sizes[i])], np.uint32))
    items.append((Circuit(sizes, types, in1, in2), np.array([rng.randrange(P) for _ in range(1000)], np.uint64)))
    return items


@pytest.mark.parametrize("graph", [False, True])
def test_batch_equals_oracle(graph):
    items = mixed_batch()
    O.set_threads(oracle_threads())
    circs = [G().Circuit.from_workload(c) for c, _ in items]
    xs = [device_tensor(x) for _, x in items]
    for call, base in enumerate((11, 5000)):
        seeds = [base + k for k in range(len(items))]
        say("batch", len(items), "graph", graph, "call", call)
        got = G().gkr_batch_prove(circs, xs, seeds, graph=graph)
        for k, ((c, x), m) in enumerate(zip(items, got)):
            want, _ = O.prove(c, x, seeds[k])
            assert np.array_equal(m, want), (k, c.name, call)


def test_batch_same_circuit_twice_and_plain_agree():
    c = W.f2_circuit(1 << 12)
    x1, x2 = W.f2_inputs(1 << 12, 1), W.f2_inputs(1 << 12, 2)
    gc = G().Circuit.from_workload(c)
    say("batch with a repeated circuit")
    got = G().gkr_batch_prove([gc, gc], [device_tensor(x1), device_tensor(x2)], [3, 4])
    assert np.array_equal(got[0], G().gkr_prove(gc, x1, 3)[0])
    assert np.array_equal(got[1], G().gkr_prove(gc, x2, 4)[0])


def test_batch_range_error():
    c = W.f2_circuit(64)
    x = W.f2_inputs(64, 1)
    x[5] = np.uint64(P)
    gc = G().Circuit.from_workload(c)
    with pytest.raises(G().GkrError) as e:
        G().gkr_batch_prove([gc], [device_tensor(x)], [1])
    assert e.value.code == G().GKR_ERR_RANGE
