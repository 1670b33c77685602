"""Pins of the oracle's GKR prover and verifier.

- tiny circuits: every transcript element equals its definition (brute
  force over the hypercube, tests/brute.py);
- any size: the sum-check invariants hold in every round, the honest
  transcript is accepted, single-element changes are rejected;
- circuit outputs equal the directly computed F2, C = AB and pattern-match
  distances (the unverifiable algorithms of Sec. 6.2.4);
- gate counts match Table 2."""
import os
import random

import numpy as np
import pytest

from oracle import oracle as O
import brute
import workloads as W
from workloads.circuits import Circuit

P = O.P


def random_circuit(rng, sizes):
    d = len(sizes) - 1
    types, in1, in2 = [], [], []
    for i in range(d):
        lim = 1 << brute.log2ceil(sizes[i + 1])
        types.append(np.array([rng.randrange(2) for _ in range(sizes[i])], np.uint8))
        in1.append(np.array([rng.randrange(lim) for _ in range(sizes[i])], np.uint32))
        in2.append(np.array([rng.randrange(lim) for _ in range(sizes[i])], np.uint32))
    return Circuit(list(sizes), types, in1, in2, name=f"rand {sizes}")


TINY = [[1, 1], [1, 2], [2, 1], [3, 5], [1, 2, 3], [3, 4, 4], [2, 3, 5], [1, 2, 2, 4],
        [4, 3, 2], [1, 1, 2], [2, 2, 1, 3], [4, 4, 4], [1, 3, 8]]


@pytest.mark.parametrize("sizes", TINY)
def test_transcript_equals_definition(sizes):
    rng = random.Random(hash(tuple(sizes)) & 0xFFFF)
    circ = random_circuit(rng, sizes)
    x = np.array([rng.randrange(P) for _ in range(sizes[-1])], np.uint64)
    seed = rng.randrange(1 << 20)
    msgs, chals = O.prove(circ, x, seed)
    assert np.array_equal(chals, O.splitmix_field(seed, 2, len(chals)))
    want = brute.transcript_by_definition(circ, x, chals)
    assert [int(v) for v in msgs] == want


def test_layer_sum_identity():
    """sum over the hypercube of f_i equals ~V_i(z): the claim the layer's
    sum-check starts from."""
    rng = random.Random(11)
    for sizes in ([2, 3, 5], [4, 3, 2], [3, 4, 4]):
        circ = random_circuit(rng, sizes)
        x = [rng.randrange(P) for _ in range(sizes[-1])]
        V = brute.evaluate(circ, x)
        z = [rng.randrange(P) for _ in range(brute.log2ceil(sizes[0]))]
        assert brute.layer_sum(circ, V, 0, z) == brute.mle(V[0], z)


def replay_invariants(circ, x, seed, msgs, chals):
    """Walk the transcript: G(0)+G(1) equals the running claim in every
    round; at the end of a layer the claim equals the wiring identity; the
    last claim is the input's extension at z_d."""
    V = O.evaluate(circ, x)
    d = len(circ.sizes) - 1
    mi, ci = 0, 0
    s0 = O.log2ceil(circ.sizes[0])
    outs = msgs[:circ.sizes[0]]
    assert np.array_equal(outs, V[0][:circ.sizes[0]])
    mi = circ.sizes[0]
    z = [int(c) for c in chals[:s0]]
    ci = s0
    claim = O.mle(V[0], z)
    for i in range(d):
        s, sp = O.log2ceil(circ.sizes[i]), O.log2ceil(circ.sizes[i + 1])
        r = []
        for j in range(s + 2 * sp):
            g0, g1, g2 = (int(v) for v in msgs[mi:mi + 3])
            mi += 3
            assert (g0 + g1) % P == claim, (i, j)
            rj = int(chals[ci]); ci += 1
            r.append(rj)
            claim = O.lagrange([g0, g1, g2], rj)
        v1, v2 = int(msgs[mi]), int(msgs[mi + 1]); mi += 2
        a, b, c = r[:s], r[s:s + sp], r[s + sp:]
        assert v1 == O.mle(V[i + 1], b) and v2 == O.mle(V[i + 1], c)
        Ea, Eb, Ec = O.eq_table(a), O.eq_table(b), O.eq_table(c)
        add = mul = 0
        for g in range(circ.sizes[i]):
            w = int(Ea[g]) * int(Eb[int(circ.in1[i][g])]) % P * int(Ec[int(circ.in2[i][g])]) % P
            if circ.types[i][g] == 0:
                add = (add + w) % P
            else:
                mul = (mul + w) % P
        beta = 1
        for zk, ak in zip(z, a):
            beta = beta * ((zk * ak + (1 - zk) * (1 - ak)) % P) % P
        assert claim == beta * ((add * (v1 + v2) + mul * v1 % P * v2) % P) % P
        ys = [v1, v2] + [int(v) for v in msgs[mi:mi + max(sp - 1, 0)]]
        mi += max(sp - 1, 0)
        tau = int(chals[ci]); ci += 1
        claim = O.lagrange(ys, tau)
        z = [(bk + tau * (ck - bk)) % P for bk, ck in zip(b, c)]
        assert claim == O.mle(V[i + 1], z)
    assert mi == len(msgs) and ci == len(chals)
    assert claim == O.mle(V[d], z)


def test_invariants_random_circuits():
    rng = random.Random(12)
    for _ in range(25):
        d = rng.randrange(1, 5)
        sizes = [rng.randrange(1, 40) for _ in range(d + 1)]
        circ = random_circuit(rng, sizes)
        x = np.array([rng.randrange(P) for _ in range(sizes[-1])], np.uint64)
        seed = rng.randrange(1 << 30)
        msgs, chals = O.prove(circ, x, seed)
        replay_invariants(circ, x, seed, msgs, chals)
        assert O.verify(circ, x, seed, msgs)[0]


def test_invariants_benchmark_circuits():
    for circ, x, seed in (W.c1_f2(), (W.matmult_circuit(8), W.matmult_inputs(8, 3), 3),
                          (W.pm_circuit(64), W.pm_inputs(64, 6)[0], 6)):
        msgs, chals = O.prove(circ, x, seed)
        replay_invariants(circ, x, seed, msgs, chals)


@pytest.mark.parametrize("sizes", [[2, 3, 5], [4, 3, 2], [1, 2, 2, 4], [1, 1, 2], [3, 1, 2]])
def test_every_single_change_is_rejected(sizes):
    rng = random.Random(13 + len(sizes))
    circ = random_circuit(rng, sizes)
    x = np.array([rng.randrange(P) for _ in range(sizes[-1])], np.uint64)
    msgs, _ = O.prove(circ, x, 99)
    assert O.verify(circ, x, 99, msgs) == (True, -1, -1, 0)
    for k in range(len(msgs)):
        for delta in (1, P - 1, 1 << 40):
            bad = msgs.copy()
            bad[k] = np.uint64((int(bad[k]) + delta) % P)
            ok, layer, rnd, check = O.verify(circ, x, 99, bad)
            assert not ok, (k, delta)
            assert check in (2, 3, 4, 5)


def test_malformed_transcripts_rejected():
    circ, x, seed = W.c1_f2()
    msgs, _ = O.prove(circ, x, seed)
    assert O.verify(circ, x, seed, msgs[:-1])[3] == 1
    bad = msgs.copy()
    bad[5] = np.uint64(P)  # not canonical
    assert O.verify(circ, x, seed, bad)[3] == 1


def test_wrong_input_or_seed_rejected():
    circ, x, seed = W.c1_f2()
    msgs, _ = O.prove(circ, x, seed)
    y = x.copy()
    y[17] += np.uint64(1)
    assert O.verify(circ, y, seed, msgs)[:1] == (False,)
    assert not O.verify(circ, x, seed + 1, msgs)[0]


def test_outputs_equal_direct_computations():
    # F2 = sum a_i^2 (Sec. 6.2.4: the unverifiable algorithm sums squares)
    circ, x, seed = W.c1_f2()
    V = O.evaluate(circ, x)
    assert int(V[0][0]) == sum(int(v) ** 2 for v in x) % P
    # C = AB (naive matrix multiplication)
    N = 16
    circ = W.matmult_circuit(N)
    inp = W.matmult_inputs(N, 3)
    A = inp[:N * N].reshape(N, N).astype(np.int64)
    B = inp[N * N:].reshape(N, N).astype(np.int64)
    V = O.evaluate(circ, inp)
    assert np.array_equal(V[0][:N * N].astype(np.int64), (A @ B).reshape(-1))
    # pattern matching: D_i = sum_j (t_{i+j} - p_j)^2, zero exactly at matches
    n, q = 300, 8
    circ = W.pm_circuit(n, q)
    inp, text, pat = W.pm_inputs(n, 21, q)
    V = O.evaluate(circ, inp)
    t = text.astype(np.int64)
    pp = pat.astype(np.int64)
    D = np.array([int(((t[i:i + q] - pp) ** 2).sum()) for i in range(n - q + 1)])
    assert np.array_equal(V[0][:n - q + 1].astype(np.int64), D)
    naive = sum(1 for i in range(n - q + 1) if all(t[i + j] == pp[j] for j in range(q)))
    assert naive >= 1 and int((V[0][:n - q + 1] == 0).sum()) == naive


def test_f0_circuits_equal_direct_computations():
    # F0 (Sec. 6.2.1): the output is 2 |{i : a_i != 0}| by Fermat's little theorem
    for n, seed in ((1, 1), (7, 2), (200, 3)):
        x = W.f0_inputs(n, seed)
        x[::5] = 0
        V = O.evaluate(W.f0_circuit(n), x)
        assert int(V[0][0]) == 2 * int(np.count_nonzero(x)), n
        top = len(V) - 1 - 61  # the Fermat stage's last layer: 2 x^(p-1) per value
        assert [int(v) for v in V[top][:n]] == [2 if v else 0 for v in x.tolist()]
    # PM with the F0 count: twice the shifts where the pattern does not occur
    n, q = 120, 8
    inp, text, pat = W.pm_inputs(n, 22, q)
    V = O.evaluate(W.pm_f0_circuit(n, q), inp)
    t, pp = text.astype(np.int64), pat.astype(np.int64)
    miss = sum(1 for i in range(n - q + 1) if any(t[i + j] != pp[j] for j in range(q)))
    assert miss < n - q + 1 and int(V[0][0]) == 2 * miss
    # MatMult check: zero iff C = AB, else twice the wrong entries
    for N, bad in ((2, 0), (4, 0), (4, 3), (8, 5)):
        inp, wrong = W.matmult_check_inputs(N, 9, bad)
        V = O.evaluate(W.matmult_check_circuit(N), inp)
        assert wrong == bad and int(V[0][0]) == 2 * wrong, (N, bad)


def test_gate_counts_and_transcript_sizes():
    path = os.path.join(os.path.dirname(__file__), "golden", "table2_circuit_sizes.txt")
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        prob, logn, millions = line.split()
        if prob == "F2":
            c = W.f2_circuit(1 << int(logn))
            assert c.gates == 3 * (1 << int(logn)) - 1
            assert round(c.gates / 1e6, 1) == float(millions)
            continue
        n = 1 << int(logn)
        gates = {"F0": lambda: 122 * n - 1,  # the builder's count, checked below at small n
                 "PM": lambda: W.pm_f0_circuit(n, 8).gates,
                 "MM": lambda: W.matmult_check_circuit(n).gates}[prob]()
        assert abs(gates / 1e6 - float(millions)) < 0.06, (prob, gates)
    for n in (1, 2, 64, 1024):  # powers of two: a complete sum tree of n - 1 gates
        assert W.f0_circuit(n).gates == 122 * n - 1
    assert W.matmult_circuit(256).gates == 2 * 256 ** 3 + 256 ** 2
    assert O.transcript_size(W.f2_circuit(1 << 10)) == (632, 196)
    assert O.transcript_size(W.f2_circuit(1 << 22)) == (2708, 826)
    assert O.transcript_size(W.matmult_circuit(256)) == (67352, 567)


def test_thread_count_does_not_change_results():
    circ, x, seed = W.f2_circuit(1 << 14), W.f2_inputs(1 << 14, 5), 5
    O.set_threads(1)
    a = O.prove(circ, x, seed)
    O.set_threads(7)
    b = O.prove(circ, x, seed)
    O.set_threads(1)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
