"""GPU GKR prover and verifier through the C ABI, bit-exact against the CPU
oracle on the same seeds (transcripts and challenges), from tiny random
circuits with padding and shared wires to the full benchmark sizes."""
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


def random_circuit(rng, sizes, kinds=None, live_wires=False):
    """Random gates; wires read any slot of the next layer's padded table,
    or (live_wires) only its gates."""
    d = len(sizes) - 1
    types, in1, in2 = [], [], []
    for i in range(d):
        lim = 1 << (sizes[i + 1] - 1).bit_length() if sizes[i + 1] > 1 else 1
        if live_wires:
            lim = sizes[i + 1]
        if kinds is None:
            t = [rng.randrange(2) for _ in range(sizes[i])]
        else:
            t = [kinds[i]] * sizes[i]
        types.append(np.array(t, np.uint8))
        in1.append(np.array([rng.randrange(lim) for _ in range(sizes[i])], np.uint32))
        in2.append(np.array([rng.randrange(lim) for _ in range(sizes[i])], np.uint32))
    return Circuit(list(sizes), types, in1, in2, name=f"rand {sizes}")


def check_same(circ, x, seed, name, device_inputs=False, algos=(1, 2, 0)):
    """The omega-phase algorithms (tables with the first small layers in one
    launch, tables layer by layer, per-gate rounds) against the oracle;
    returns the circuit handle (first algorithm) and its transcript."""
    say(name, "gates", circ.gates, "seed", seed)
    O.set_threads(oracle_threads())
    want_m, want_c = O.prove(circ, x, seed)
    inp = device_tensor(x) if device_inputs else x
    first = None
    for algo in algos:
        say(name, "omega algorithm", algo)
        gc = G().Circuit.from_workload(circ, omega_algo=algo)
        got_m, got_c = G().gkr_prove(gc, inp, seed)
        assert len(got_m) == len(want_m) and len(got_c) == len(want_c)
        bad = np.nonzero(got_m != want_m)[0]
        assert len(bad) == 0, f"{name} algo {algo}: first differing msg {bad[:5]} of {len(want_m)}"
        assert np.array_equal(got_c, want_c), name
        if first is None:
            first = (gc, got_m)
    return first


TINY = [[1, 1], [1, 2], [2, 1], [3, 5], [1, 2, 3], [3, 4, 4], [2, 3, 5], [1, 2, 2, 4],
        [4, 3, 2], [1, 1, 2], [2, 2, 1, 3], [4, 4, 4], [1, 3, 8], [5, 1, 1, 7]]


@pytest.mark.parametrize("sizes", TINY)
def test_tiny_random_circuits(sizes):
    rng = random.Random(hash(tuple(sizes)) & 0xFFFF)
    circ = random_circuit(rng, sizes)
    x = np.array([rng.randrange(P) for _ in range(sizes[-1])], np.uint64)
    check_same(circ, x, rng.randrange(1 << 20), f"tiny {sizes}")


def test_random_circuits_all_kinds():
    rng = random.Random(77)
    for trial in range(40):
        d = rng.randrange(1, 6)
        sizes = [rng.choice([1, 2, 3, 5, 8, 13, 64, 100, 257, 1000, 4096, 5000])
                 for _ in range(d + 1)]
        kinds = None if trial % 3 == 0 else [rng.randrange(2) for _ in range(d)]
        circ = random_circuit(rng, sizes, kinds)
        x = np.array([rng.randrange(P) for _ in range(sizes[-1])], np.uint64)
        check_same(circ, x, rng.randrange(1 << 30), f"random {sizes} kinds {kinds}")


def test_many_blocks_and_ragged_tail():
    """Layers spanning many workgroups (grid-stride loops) with non-power-of-two
    sizes and wires into padding."""
    rng = random.Random(5)
    for sizes in ([3001, 70001, 140001], [1, 300000, 2], [70000, 70000, 9]):
        circ = random_circuit(rng, sizes)
        x = np.array([rng.randrange(P) for _ in range(sizes[-1])], np.uint64)
        check_same(circ, x, 11, f"ragged {sizes}")


def test_wire_fanout_around_chunk_size():
    """Wires read by 0, 1, 31, 32, 33, 64 and 100 gates: layers whose wires
    all fit one chunk of gates take the fused pass, the others the per-chunk
    pass; both phases and both gate kinds."""
    rng = random.Random(21)
    fan = [0, 1, 31, 32, 33, 64, 100, 2, 0, 5, 17, 40, 0, 3, 1, 9]
    for kinds in (None, [0, 1], [1, 0]):
        reads = [x for x, f in enumerate(fan) for _ in range(f)]
        rng.shuffle(reads)
        S0 = len(reads)
        other = [rng.randrange(16) for _ in range(S0)]
        small = [rng.randrange(16) for _ in range(16)]
        t0 = [rng.randrange(2) if kinds is None else kinds[0] for _ in range(S0)]
        t1 = [rng.randrange(2) if kinds is None else kinds[1] for _ in range(16)]
        for swap in (False, True):
            a, b = (other, reads) if swap else (reads, other)
            circ = Circuit([S0, 16, 16], [np.array(t0, np.uint8), np.array(t1, np.uint8)],
                           [np.array(a, np.uint32), np.array(small, np.uint32)],
                           [np.array(b, np.uint32), np.array(small[::-1], np.uint32)],
                           name="fan-out")
            x = np.array([rng.randrange(P) for _ in range(16)], np.uint64)
            check_same(circ, x, 31, f"fan-out kinds {kinds} swap {swap}")


def test_heavy_wires_in_big_chunks():
    """Wires read by 2047 .. 5000 gates: above 2048 gates a wire's gates are
    cut into chunks of 512 summed by a whole wave; both phases, both kinds,
    light wires beside them."""
    rng = random.Random(23)
    fan = [2047, 2048, 2049, 2560, 2561, 5000, 3, 0, 1, 700, 31, 33, 0, 2, 9, 64]
    for kinds in (None, [1, 0], [0, 1]):
        reads = [x for x, f in enumerate(fan) for _ in range(f)]
        rng.shuffle(reads)
        S0 = len(reads)
        other = [rng.randrange(16) for _ in range(S0)]
        small = [rng.randrange(16) for _ in range(16)]
        t0 = [rng.randrange(2) if kinds is None else kinds[0] for _ in range(S0)]
        t1 = [rng.randrange(2) if kinds is None else kinds[1] for _ in range(16)]
        for swap in (False, True):
            a, b = (other, reads) if swap else (reads, other)
            circ = Circuit([S0, 16, 16], [np.array(t0, np.uint8), np.array(t1, np.uint8)],
                           [np.array(a, np.uint32), np.array(small, np.uint32)],
                           [np.array(b, np.uint32), np.array(small[::-1], np.uint32)],
                           name="heavy wires")
            x = np.array([rng.randrange(P) for _ in range(16)], np.uint64)
            check_same(circ, x, 37, f"heavy wires kinds {kinds} swap {swap}")


def test_line_by_folding_on_wide_layers():
    """Layers reading 2^11 .. 2^22 values take the line as a fold of V along
    it (ST_LFOLD, its rows added up by ST_FINISH): ragged sizes at both ends
    of that range, mixed gates, every omega algorithm (the per-gate one
    finishes its last round in the fold's launch)."""
    rng = random.Random(29)
    for sizes in ([5, 70001, 131072 + 7], [3, (1 << 21) + 5], [1000, (1 << 22)], [7, 1025, 2048 + 3, 40000]):
        circ = random_circuit(rng, sizes)
        x = np.array([rng.randrange(P) for _ in range(sizes[-1])], np.uint64)
        check_same(circ, x, 41, f"line fold {sizes}", device_inputs=True)
    n = (1 << 17) + 3
    check_same(W.f2_circuit(n), W.f2_inputs(n, 43), 43, f"line fold F2 n={n}")


def test_line_by_folding_above_2p22_entries():
    """Input layers of 2^22 + 5 and 2^23 + 3 values (s' = 23, 24: 257 and
    513 folding workgroups, one per 2^14 entries up to the layer's size,
    whose rows ST_FINISH adds) read by a few gates, so the oracle stays
    quick."""
    rng = random.Random(31)
    for sizes in ([3, 5, (1 << 22) + 5], [2, (1 << 23) + 3]):
        circ = random_circuit(rng, sizes)
        x = np.random.default_rng(sizes[-1]).integers(0, P, sizes[-1], dtype=np.uint64)
        check_same(circ, x, 47, f"line fold {sizes}", device_inputs=True)


def test_wires_below_the_padding():
    """Layers whose gates read only the next layer's gates (not its zero
    padding): the omega phases' grid steps take the tables' first entries
    only, rounded up to 2^k0, and the tail zeroes the rest of its level.
    Next-layer sizes just above a power of two, at a multiple of it plus one,
    and tiny, for every omega algorithm."""
    rng = random.Random(37)
    for sizes in ([5, 70001, 131072 + 7], [3, 300, 1500, (1 << 20) + (1 << 16) + 5],
                  [7, 1025, 2048 + 3, 40000], [2, 9, 17, 33, 300, 4097, 3 * 8192 + 1]):
        circ = random_circuit(rng, sizes, live_wires=True)
        x = np.random.default_rng(sizes[-1]).integers(0, P, sizes[-1], dtype=np.uint64)
        check_same(circ, x, 53, f"live wires {sizes}", device_inputs=True)


def test_extreme_values_through_every_kernel():
    """Inputs at the ends of the field (all p - 1, all zero, p - 1 and 0 in
    turn) through layers wide enough for the grid steps, the line fold and
    the tails, on every omega algorithm: differences, line values and
    running sums are kept unreduced below fixed multiples of p inside the
    kernels, and these inputs put the first layers' values at those ends."""
    n = (1 << 14) + 5
    for name, x in (("p-1", np.full(n, P - 1, np.uint64)), ("zero", np.zeros(n, np.uint64)),
                    ("alternating", np.array([P - 1 if i % 2 else 0 for i in range(n)], np.uint64))):
        check_same(W.f2_circuit(n), x, 3, f"F2 n={n} inputs {name}")
    rng = random.Random(61)
    sizes = [3, 300, 5000, 20000]
    circ = random_circuit(rng, sizes)
    check_same(circ, np.full(sizes[-1], P - 1, np.uint64), 5, f"mixed {sizes} inputs p-1")


def test_c1_f2_1024():
    circ, x, seed = W.c1_f2()
    gc, m = check_same(circ, x, seed, "C1 F2 n=2^10")
    assert int(m[0]) == sum(int(v) ** 2 for v in x) % P


def test_device_inputs_equal_host_inputs():
    circ, x, seed = W.c1_f2()
    check_same(circ, x, seed, "C1 device inputs", device_inputs=True)


def test_matmult_and_pm_small():
    for N in (2, 4, 16, 32):
        circ = W.matmult_circuit(N)
        x = W.matmult_inputs(N, 3)
        gc, m = check_same(circ, x, 3, f"MatMult N={N}")
        A = x[:N * N].reshape(N, N).astype(np.int64)
        B = x[N * N:].reshape(N, N).astype(np.int64)
        assert np.array_equal(m[:N * N].astype(np.int64), (A @ B).reshape(-1))
    for n in (8, 9, 100, 4096):
        circ = W.pm_circuit(n)
        x, _, _ = W.pm_inputs(n, 6)
        check_same(circ, x, 6, f"PM n={n}")


def test_f2_odd_sizes():
    for n in (1, 2, 3, 7, 1000, 3 * 4096 + 1):
        check_same(W.f2_circuit(n), W.f2_inputs(n, 9), 9, f"F2 n={n}")


def test_input_range_error():
    circ, x, seed = W.c1_f2()
    gc = G().Circuit.from_workload(circ)
    y = x.copy()
    y[3] = np.uint64(P)
    for dev in (False, True):
        say("range error, device inputs", dev)
        with pytest.raises(G().GkrError) as e:
            G().gkr_prove(gc, device_tensor(y) if dev else y, seed)
        assert e.value.code == G().GKR_ERR_RANGE


def test_invalid_circuits_rejected_on_create():
    g = G()
    with pytest.raises(g.GkrError):
        g.Circuit([1], [], [], [])
    with pytest.raises(g.GkrError):  # wire beyond the padded next layer
        g.Circuit([1, 2], [np.zeros(1, np.uint8)], [np.array([2], np.uint32)],
                  [np.array([0], np.uint32)])
    with pytest.raises(g.GkrError):  # unknown gate type
        g.Circuit([1, 2], [np.array([2], np.uint8)], [np.array([0], np.uint32)],
                  [np.array([1], np.uint32)])


# ------------------------------------------------------------------ verifier

def test_verifier_accepts_and_agrees_with_oracle_on_rejections():
    rng = random.Random(21)
    for sizes in ([2, 3, 5], [4, 3, 2], [1, 2, 2, 4], [3, 1, 2], [1, 1]):
        circ = random_circuit(rng, sizes)
        x = np.array([rng.randrange(P) for _ in range(sizes[-1])], np.uint64)
        gc, m = check_same(circ, x, 5, f"verify {sizes}")
        say("verify honest", sizes)
        assert G().gkr_verify(gc, x, 5, m) == (True, -1, -1, 0)
        assert G().gkr_verify(gc, device_tensor(x), 5, m)[0]
        for k in range(len(m)):
            bad = m.copy()
            bad[k] = np.uint64((int(bad[k]) + 1) % P)
            got = G().gkr_verify(gc, x, 5, bad)
            want = O.verify(circ, x, 5, bad)
            assert got == want, (sizes, k, got, want)
        assert G().gkr_verify(gc, x, 5, m[:-1])[3] == 1
        if gc.rounds > 0:  # with no round, no challenge affects the transcript
            assert not G().gkr_verify(gc, x, 6, m)[0]


def test_verifier_c1_and_input_change():
    circ, x, seed = W.c1_f2()
    gc = G().Circuit.from_workload(circ)
    m, _ = G().gkr_prove(gc, x, seed)
    assert G().gkr_verify(gc, x, seed, m)[0]
    y = x.copy()
    y[100] ^= np.uint64(1)
    ok, layer, rnd, check = G().gkr_verify(gc, y, seed, m)
    assert not ok and check == 5


# ------------------------------------------------------------ full sizes

def test_c2_f2_4m_full_bit_exact():
    circ, x, seed = W.c2_f2()
    gc, m = check_same(circ, x, seed, "C2 F2 n=2^22", device_inputs=True)
    assert int(m[0]) == int((x.astype(object) ** 2).sum()) % P
    say("C2 verify")
    assert G().gkr_verify(gc, device_tensor(x), seed, m) == (True, -1, -1, 0)
    # again in the launch shapes bench.py times: its committed table when it
    # matches the kernel sources, else tuned on this proof as bench.py does
    import bench
    say("C2 in the launch shapes of bench.py")
    xt = device_tensor(x)
    try:
        if not bench.load_tune_table(G(), bench.TUNE_FILE):
            G().gkr_autotune([gc], [xt], reps=1)
        m2, _ = G().gkr_prove(gc, xt, seed)
        assert np.array_equal(m2, m)
    finally:
        G().gkr_tune_set(None)


def test_c3_matmult_256_full_bit_exact():
    circ, x, seed = W.c3_matmult()
    gc, m = check_same(circ, x, seed, "C3 MatMult N=256", device_inputs=True)
    N = 256
    A = x[:N * N].reshape(N, N).astype(np.int64)
    B = x[N * N:].reshape(N, N).astype(np.int64)
    assert np.array_equal(m[:N * N].astype(np.int64), (A @ B).reshape(-1))
    say("C3 verify")
    assert G().gkr_verify(gc, device_tensor(x), seed, m)[0]
