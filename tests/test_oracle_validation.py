"""Pins of the oracle's input validation: which circuits and inputs its
prover and verifier refuse.  A circuit is layered with fan-in 2 and gates of
two types, addition and multiplication (Sec. 3.1); a wire names a gate of
the next layer or one of its zero padding slots, so the largest admissible
wire is 2^ceil(log2 S_{i+1}) - 1; inputs are field elements, below p = 2^61
- 1 (Sec. 6.1).  The boundaries are tested on both sides, so an off-by-one
in any check fails here."""
import ctypes as C

import numpy as np
import pytest

from oracle import oracle as O
from workloads.circuits import Circuit

P = O.P


def one_layer(S0, S1, t, a, b):
    return Circuit([S0, S1], [np.array(t, np.uint8)], [np.array(a, np.uint32)],
                   [np.array(b, np.uint32)])


def rc_prove(circ, x, seed=1):
    M = O._Marshal(circ)
    nm, nc = O.transcript_size(circ) if len(circ.sizes) >= 2 and min(circ.sizes) > 0 else (1, 1)
    msgs = np.zeros(max(nm, 1) + 8, np.uint64)
    chals = np.zeros(max(nc, 1) + 8, np.uint64)
    xin = np.ascontiguousarray(x, np.uint64) if len(x) else np.zeros(1, np.uint64)
    return O.lib().or_prove(*M.args(), xin, seed, msgs, chals)


def rc_verify(circ, x, msgs, seed=1):
    M = O._Marshal(circ)
    acc, wl, wr, wc = C.c_int(), C.c_int(), C.c_int(), C.c_int()
    m = np.ascontiguousarray(msgs, np.uint64) if len(msgs) else np.zeros(1, np.uint64)
    xin = np.ascontiguousarray(x, np.uint64) if len(x) else np.zeros(1, np.uint64)
    rc = O.lib().or_verify(*M.args(), xin, seed, m, len(msgs), C.byref(acc), C.byref(wl),
                           C.byref(wr), C.byref(wc))
    return rc, bool(acc.value)


def test_fewer_than_two_layers_rejected():
    assert not O.check_circuit(Circuit([1]))
    assert rc_prove(Circuit([1]), [5]) == -1


def test_empty_layer_rejected():
    # an empty output layer, and an empty input layer
    assert not O.check_circuit(one_layer(0, 2, [], [], []))
    assert not O.check_circuit(Circuit([1, 1, 0], [np.zeros(1, np.uint8), np.zeros(1, np.uint8)],
                                       [np.zeros(1, np.uint32), np.zeros(1, np.uint32)],
                                       [np.zeros(1, np.uint32), np.zeros(1, np.uint32)]))
    assert rc_prove(one_layer(0, 2, [], [], []), [1, 2]) == -1


@pytest.mark.parametrize("t,ok", [(0, True), (1, True), (2, False), (255, False)])
def test_gate_types(t, ok):
    c = one_layer(1, 2, [t], [0], [1])
    assert O.check_circuit(c) == ok
    assert (rc_prove(c, [3, 4]) == 0) == ok


@pytest.mark.parametrize("S1", [1, 2, 3, 4, 5, 8, 9])
def test_wire_limit_is_the_padded_next_layer(S1):
    lim = 1 << (S1 - 1).bit_length()  # 2^ceil(log2 S1); 1 for S1 = 1
    x = list(range(1, S1 + 1))
    for side in (0, 1):
        good = [lim - 1, 0] if side == 0 else [0, lim - 1]
        bad = [lim, 0] if side == 0 else [0, lim]
        cg = one_layer(1, S1, [1], [good[0]], [good[1]])
        cb = one_layer(1, S1, [1], [bad[0]], [bad[1]])
        assert O.check_circuit(cg), (S1, side)
        assert not O.check_circuit(cb), (S1, side)
        assert rc_prove(cg, x) == 0
        assert rc_prove(cb, x) == -1
        # a wire into a padding slot reads zero: the product is 0
        if lim - 1 >= S1:
            m, _ = O.prove(cg, np.array(x, np.uint64), 1)
            assert int(m[0]) == 0


def test_input_range_on_both_sides():
    c = one_layer(1, 2, [0], [0], [1])
    assert rc_prove(c, [P - 1, 7]) == 0
    assert rc_prove(c, [P, 7]) == -2
    assert rc_prove(c, [7, (1 << 64) - 1]) == -2
    m, _ = O.prove(c, np.array([P - 1, 7], np.uint64), 1)
    assert int(m[0]) == (P - 1 + 7) % P
    assert rc_verify(c, [P - 1, 7], m) == (0, True)
    assert rc_verify(c, [P, 7], m)[0] == -2
    assert rc_verify(one_layer(1, 2, [2], [0], [1]), [1, 7], m)[0] == -1


def test_f2_sumcheck_length_must_be_a_power_of_two():
    for n in (1, 2, 4, 1024):
        O.f2sc_prove(np.arange(n, dtype=np.uint32), 1)
    for n in (3, 6, 1000):
        with pytest.raises(ValueError):
            O.f2sc_prove(np.arange(n, dtype=np.uint32), 1)
