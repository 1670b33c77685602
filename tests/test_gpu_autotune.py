"""Launch-shape autotuning: the chosen shapes change timing only; every
transcript still equals the oracle's, alone and batched."""
import numpy as np
import pytest

from gpu_util import say, device_tensor, oracle_threads
from oracle import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def test_autotune_keeps_transcripts():
    import paper_1202_1350_amd as G
    O.set_threads(oracle_threads())
    cases = [(W.f2_circuit(1 << 13), W.f2_inputs(1 << 13, 8), 8),
             (W.pm_circuit(1 << 10), W.pm_inputs(1 << 10, 9)[0], 9),
             (W.matmult_circuit(16), W.matmult_inputs(16, 10), 10)]
    circs = [G.Circuit.from_workload(c) for c, _, _ in cases]
    xs = [device_tensor(x) for _, x, _ in cases]
    want = [O.prove(c, x, sd)[0] for c, x, sd in cases]
    G.gkr_tune_set(None)
    default = G.gkr_tune_get()
    say("autotune on", len(circs), "circuits")
    G.gkr_autotune(circs, xs, reps=1)
    tuned = G.gkr_tune_get()
    assert len(tuned) == len(default) and tuned != default
    for gc, x, (_, _, sd), w in zip(circs, xs, cases, want):
        m, _ = G.gkr_prove(gc, x, sd)
        assert np.array_equal(m, w)
    got = G.gkr_batch_prove(circs, xs, [sd for _, _, sd in cases])
    assert all(np.array_equal(a, b) for a, b in zip(got, want))
    # back to the defaults and to the tuned table: same transcripts
    for table in (None, tuned):
        G.gkr_tune_set(table)
        for gc, x, (_, _, sd), w in zip(circs, xs, cases, want):
            assert np.array_equal(G.gkr_prove(gc, x, sd)[0], w)
    assert G.gkr_tune_get() == tuned
    G.gkr_tune_set(None)
