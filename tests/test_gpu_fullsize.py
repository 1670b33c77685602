"""Full-size parity: the batched, served and Table 2 workloads at their
benchmark sizes and seeds, every transcript element compared with the
oracle's (and, for served proofs, with the same proof made alone by
gkr_prove).  Each test runs the oracle on the host's threads for up to about
a minute."""
import time

import numpy as np
import pytest

from gpu_util import say, device_tensor, oracle_threads
from oracle import oracle as O
import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def G():
    import paper_1202_1350_amd as mod
    return mod


def same(got, want, what):
    assert len(got) == len(want), (what, len(got), len(want))
    bad = np.nonzero(got != want)[0]
    assert len(bad) == 0, f"{what}: first differing messages {bad[:5]} of {len(want)}"


def test_batch_of_64_uneven_proofs_equals_oracle():
    """The 64-proof batch of the benchmark (F2 n log-uniform in [2^12, 2^20],
    PM text in [2^14, 2^18], seed 4), batched with graph replay."""
    O.set_threads(oracle_threads())
    mix = W.batch_mix(4, 64)
    circs = [G().Circuit.from_workload(c) for _, c, _, _ in mix]
    xs = [device_tensor(x) for _, _, x, _ in mix]
    seeds = [sd for _, _, _, sd in mix]
    say("batch of 64, seed 4")
    got = G().gkr_batch_prove(circs, xs, seeds)
    for k, ((kind, c, x, sd), m) in enumerate(zip(mix, got)):
        say("oracle of batch entry", k, kind, c.sizes[-1])
        same(m, O.prove(c, x, sd)[0], f"batch entry {k} ({c.name})")


def test_served_shapes_under_load_equal_oracle_and_alone():
    """One request of each serving shape (F2 at powers of two and between
    them up to 2^22, MatMult 64/128/256, PM 2^16), submitted among a stream
    of other requests so that they share launches with it."""
    O.set_threads(oracle_threads())
    probes = [("F2", n) for n in (1 << 14, 3 << 15, 1 << 18, 5 << 18, 1 << 22)] + \
             [("MM", N) for N in (64, 128, 256)] + [("PM", 1 << 16)]
    cache = {}

    def make(kind, size, seed):
        if (kind, size) not in cache:
            if kind == "F2":
                c = W.f2_circuit(size)
            elif kind == "MM":
                c = W.matmult_circuit(size)
            else:
                c = W.pm_circuit(size)
            cache[(kind, size)] = (c, G().Circuit.from_workload(c))
        c, gc = cache[(kind, size)]
        if kind == "F2":
            x = W.f2_inputs(size, seed)
        elif kind == "MM":
            x = W.matmult_inputs(size, seed)
        else:
            x = W.pm_inputs(size, seed)[0]
        return c, gc, x

    load = [("F2", 1 << 12), ("F2", 3000), ("PM", 1 << 12), ("MM", 16), ("F2", 1 << 16)]
    srv = G().Server(32 << 30, 32)
    try:
        ids = []
        for k, (kind, size) in enumerate(probes):
            for j in range(4):  # background requests around every probe
                lk, ls = load[(k + j) % len(load)]
                c, gc, x = make(lk, ls, 500 + 10 * k + j)
                srv.submit(gc, x, 900 + 10 * k + j)
            c, gc, x = make(kind, size, 100 + k)
            say("serve probe", kind, size)
            ids.append((srv.submit(gc, x, 200 + k), c, gc, x, 200 + k))
        out = {}
        t0 = time.time()
        while len(out) < len(ids):
            for rid, *_ in ids:
                if rid not in out:
                    done, m, _ = srv.poll(rid)
                    if done:
                        out[rid] = m
            assert time.time() - t0 < 300, "server did not finish"
            time.sleep(0.001)
    finally:
        srv.close()
    for rid, c, gc, x, sd in ids:
        say("compare served", c.name)
        alone, _ = G().gkr_prove(gc, x, sd)
        same(out[rid], alone, f"served vs alone {c.name}")
        same(out[rid], O.prove(c, x, sd)[0], f"served vs oracle {c.name}")


@pytest.mark.parametrize("name", ["MatMult check N=256", "PM-F0 text 2^19"])
def test_table2_circuits_equal_oracle(name):
    """Table 2's MatMult (with the C = AB check, N = 256, seed 8) and pattern
    matching (with the F0 count, text 2^19, q = 8, seed 7) at their sizes."""
    O.set_threads(oracle_threads())
    circ, x, seed = W.f1_matmult_check() if name.startswith("MatMult") else W.f1_pm_f0()
    gc = G().Circuit.from_workload(circ)
    say("prove", name, "gates", circ.gates)
    m, c = G().gkr_prove(gc, device_tensor(x), seed)
    say("oracle", name)
    wm, wc = O.prove(circ, x, seed)
    same(m, wm, name)
    assert np.array_equal(c, wc)
    assert G().gkr_verify(gc, device_tensor(x), seed, m)[0]
