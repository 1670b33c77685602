"""GPU prover on the circuits built on the F0 (Fermat) stage: F0, pattern
matching with the F0 count and the MatMult check (Table 2's other rows).
Small and medium instances: transcripts and challenges bit-exact against
the oracle.  Table 2's sizes: the circuit outputs (the first messages)
equal the direct computations and the GPU verifier accepts."""
import numpy as np
import pytest

from gpu_util import say, device_tensor, oracle_threads
from oracle import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def G():
    import paper_1202_1350_amd as mod
    return mod


def same_as_oracle(circ, x, seed, name):
    say(name, "gates", circ.gates, "depth", circ.depth, "seed", seed)
    O.set_threads(oracle_threads())
    want_m, want_c = O.prove(circ, x, seed)
    gc = G().Circuit.from_workload(circ)
    got_m, got_c = G().gkr_prove(gc, x, seed)
    bad = np.nonzero(got_m != want_m)[0]
    assert len(bad) == 0, f"{name}: first differing msg {bad[:5]} of {len(want_m)}"
    assert np.array_equal(got_c, want_c), name
    assert G().gkr_verify(gc, x, seed, got_m)[0], name
    return got_m


@pytest.mark.parametrize("n", [1, 3, 64, 257, 4096])
def test_f0_matches_oracle(n):
    x = W.f0_inputs(n, 10 + n)
    m = same_as_oracle(W.f0_circuit(n), x, 11, f"F0 n={n}")
    assert int(m[0]) == 2 * int(np.count_nonzero(x))


@pytest.mark.parametrize("n,q", [(16, 4), (100, 8), (2048, 8)])
def test_pm_f0_matches_oracle(n, q):
    inp, text, pat = W.pm_inputs(n, 12, q)
    m = same_as_oracle(W.pm_f0_circuit(n, q), inp, 13, f"PM-F0 n={n} q={q}")
    t, pp = text.astype(np.int64), pat.astype(np.int64)
    miss = sum(1 for i in range(n - q + 1) if any(t[i + j] != pp[j] for j in range(q)))
    assert int(m[0]) == 2 * miss


@pytest.mark.parametrize("N,bad", [(2, 0), (4, 3), (16, 0), (16, 7)])
def test_matmult_check_matches_oracle(N, bad):
    inp, wrong = W.matmult_check_inputs(N, 14, bad)
    m = same_as_oracle(W.matmult_check_circuit(N), inp, 15, f"MatMult-check N={N} bad={bad}")
    assert int(m[0]) == 2 * wrong


@pytest.mark.parametrize("which", ["F0", "PM", "MM"])
def test_table2_sizes_outputs_and_verifier(which):
    """At Table 2's sizes (in the launch shapes the bench uses): the output
    is the direct computation, the verifier accepts, a changed message is
    rejected."""
    if which == "F0":
        circ, x, seed = W.f1_f0()
        want = 2 * int(np.count_nonzero(x))
    elif which == "PM":
        circ, x, seed = W.f1_pm_f0()
        n, q = 1 << 19, 8
        _, text, pat = W.pm_inputs(n, 7, q)
        win = np.lib.stride_tricks.sliding_window_view(text, q)
        want = 2 * int(np.count_nonzero((win != pat[None, :]).any(axis=1)))
    else:
        circ, x, seed = W.f1_matmult_check()
        want = 0  # C = AB
    say(which, "Table 2 size, gates", circ.gates)
    gc = G().Circuit.from_workload(circ)
    xt = device_tensor(x)
    m, _ = G().gkr_prove(gc, xt, seed)
    assert int(m[0]) == want
    assert G().gkr_verify(gc, xt, seed, m)[0]
    m2 = m.copy()
    m2[len(m2) // 2] = (int(m2[len(m2) // 2]) + 1) % W.P
    assert not G().gkr_verify(gc, xt, seed, m2)[0]
