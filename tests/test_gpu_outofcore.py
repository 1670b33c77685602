"""Out-of-core proofs (copy once per layer, copy every message; Sec. 5.1.2,
5.1.3): the transcript of every memory placement equals the oracle's and the
resident path's, on circuits of every depth (the three value-table slots
wrap from depth 3 on), ragged and multi-workgroup layers, mixed gates, both
omega algorithms, batched and served proofs, and device budgets that force
each placement."""
import random
import time

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


def random_circuit(rng, sizes):
    d = len(sizes) - 1
    types, in1, in2 = [], [], []
    for i in range(d):
        lim = 1 << (sizes[i + 1] - 1).bit_length() if sizes[i + 1] > 1 else 1
        types.append(np.array([rng.randrange(2) for _ in range(sizes[i])], np.uint8))
        in1.append(np.array([rng.randrange(lim) for _ in range(sizes[i])], np.uint32))
        in2.append(np.array([rng.randrange(lim) for _ in range(sizes[i])], np.uint32))
    return Circuit(list(sizes), types, in1, in2, name=f"rand {sizes}")


def cases():
    rng = random.Random(41)
    out = []
    for sizes in ([1, 2], [3, 5], [2, 3, 5], [1, 2, 3, 4], [4, 3, 2, 7, 9], [5, 1, 1, 7, 2, 3],
                  [3001, 70001, 140001], [9, 70000, 300, 5000, 2, 64, 1000]):
        c = random_circuit(rng, sizes)
        out.append((c, np.array([rng.randrange(P) for _ in range(sizes[-1])], np.uint64), 7))
    out.append((W.f2_circuit(3000), W.f2_inputs(3000, 3), 3))
    out.append((W.f2_circuit(1 << 16), W.f2_inputs(1 << 16, 4), 4))
    out.append((W.matmult_circuit(16), W.matmult_inputs(16, 5), 5))
    out.append((W.pm_circuit(300), W.pm_inputs(300, 6)[0], 6))
    out.append((W.f0_circuit(64), W.f0_inputs(64, 8), 8))
    return out


@pytest.mark.parametrize("algo", [1, 0])
def test_every_placement_equals_oracle(algo):
    O.set_threads(oracle_threads())
    for circ, x, seed in cases():
        want_m, want_c = O.prove(circ, x, seed)
        gc = G().Circuit.from_workload(circ, omega_algo=algo)
        for mode in (G().GKR_MEM_LAYER, G().GKR_MEM_MESSAGE, G().GKR_MEM_RESIDENT):
            say("placement", mode, "algo", algo, circ.name)
            assert gc.set_memory(mode) == mode
            for inp in (x, device_tensor(x)):
                m, c = G().gkr_prove(gc, inp, seed)
                bad = np.nonzero(m != want_m)[0]
                assert len(bad) == 0, (circ.name, mode, bad[:5])
                assert np.array_equal(c, want_c)
        say("verify out of core", circ.name)
        gc.set_memory(G().GKR_MEM_MESSAGE)
        assert G().gkr_verify(gc, x, seed, want_m)[0]
        bad = want_m.copy()
        bad[-1] = np.uint64((int(bad[-1]) + 1) % P)
        assert not G().gkr_verify(gc, x, seed, bad)[0]


def test_repeated_proofs_reuse_slots():
    """Consecutive per-layer proofs on one workspace: the copies of one proof
    never race the steps of the next."""
    O.set_threads(oracle_threads())
    circ = W.f2_circuit(1 << 14)
    gc = G().Circuit.from_workload(circ)
    gc.set_memory(G().GKR_MEM_LAYER)
    for k in range(6):
        x = W.f2_inputs(1 << 14, 20 + k)
        say("per-layer proof", k)
        m, _ = G().gkr_prove(gc, device_tensor(x), 30 + k)
        assert np.array_equal(m, O.prove(circ, x, 30 + k)[0])


def test_auto_placement_within_budget():
    O.set_threads(oracle_threads())
    circ, x = W.f0_circuit(1 << 12), W.f0_inputs(1 << 12, 6)
    want, _ = O.prove(circ, x, 6)
    gc = G().Circuit.from_workload(circ)
    need = {m: gc.memory_need(m) for m in (0, 1, 2)}
    assert need[0][0] > need[1][0] > need[2][0] > 0, need
    for budget, expect in ((0, 0), (need[0][0], 0), (need[0][0] - 1, 1), (need[1][0] - 1, 2)):
        say("auto placement, budget", budget)
        assert gc.set_memory(G().GKR_MEM_AUTO, budget) == expect
        assert np.array_equal(G().gkr_prove(gc, x, 6)[0], want)
    with pytest.raises(G().GkrError) as e:
        gc.set_memory(G().GKR_MEM_AUTO, need[2][0] - 1)
    assert e.value.code == G().GKR_ERR_NOMEM
    with pytest.raises(G().GkrError):
        gc.set_memory(G().GKR_MEM_RESIDENT, need[0][0] - 1)


def test_batches_with_out_of_core_circuits():
    O.set_threads(oracle_threads())
    items = [(W.f2_circuit(1 << 10), W.f2_inputs(1 << 10, 1)), (W.pm_circuit(200), W.pm_inputs(200, 2)[0])]
    circs = [G().Circuit.from_workload(c) for c, _ in items]
    circs[1].set_memory(G().GKR_MEM_MESSAGE)
    xs = [device_tensor(x) for _, x in items]
    say("batch with a per-message circuit")
    got = G().gkr_batch_prove(circs, xs, [5, 6])
    for (c, x), m, sd in zip(items, got, (5, 6)):
        assert np.array_equal(m, O.prove(c, x, sd)[0])
    circs[1].set_memory(G().GKR_MEM_LAYER)
    with pytest.raises(G().GkrError) as e:
        G().gkr_batch_prove(circs, xs, [5, 6])
    assert e.value.code == G().GKR_ERR_INVALID


def test_server_admits_over_budget_proofs_out_of_core():
    """A request whose resident scratch exceeds the server's budget runs with
    its tables in host memory instead of failing."""
    O.set_threads(oracle_threads())
    circ = W.f2_circuit(1 << 16)
    gc = G().Circuit.from_workload(circ)
    res_need = gc.memory_need(G().GKR_MEM_RESIDENT)[0]
    msg_need = gc.memory_need(G().GKR_MEM_MESSAGE)[0]
    budget = (res_need + msg_need) // 2
    assert msg_need < budget < res_need
    srv = G().Server(budget, 4)
    try:
        ids = [srv.submit(gc, W.f2_inputs(1 << 16, k), 40 + k) for k in range(3)]
        say("serve over-budget requests")
        t0 = time.time()
        out = {}
        while len(out) < len(ids):
            for rid in ids:
                if rid not in out:
                    done, m, _ = srv.poll(rid)
                    if done:
                        out[rid] = m
            assert time.time() - t0 < 120
            time.sleep(0.001)
        assert srv.stats()[2] <= budget
        for k, rid in enumerate(ids):
            assert np.array_equal(out[rid], O.prove(circ, W.f2_inputs(1 << 16, k), 40 + k)[0])
    finally:
        srv.close()
