"""Pins of the oracle's sum-check for F2 = sum_x ~a(x)^2 (the sum-check
primitive of Sec. 7 applied to the second frequency moment of Sec. 3.2)."""
import random

import numpy as np
import pytest

from oracle import oracle as O
import brute
import workloads as W

P = O.P


@pytest.mark.parametrize("logn", [0, 1, 2, 3, 5])
def test_transcript_equals_definition(logn):
    rng = random.Random(logn)
    a = np.array([rng.randrange(1 << 16) for _ in range(1 << logn)], np.uint32)
    msgs, chals = O.f2sc_prove(a, 31)
    assert np.array_equal(chals, O.splitmix_field(31, 4, logn))
    assert [int(v) for v in msgs] == brute.f2sc_by_definition(a, chals)


def test_invariants_and_accept():
    a = W.f2sc_vector(1 << 12, 2)
    msgs, chals = O.f2sc_prove(a, 2)
    assert int(msgs[0]) == sum(int(v) ** 2 for v in a) % P
    claim = int(msgs[0])
    for j in range(12):
        g = [int(v) for v in msgs[1 + 3 * j:4 + 3 * j]]
        assert (g[0] + g[1]) % P == claim
        claim = O.lagrange(g, int(chals[j]))
    ar = O.mle(a.astype(np.uint64), chals)
    assert claim == ar * ar % P
    assert O.f2sc_verify(a, 2, msgs) == (True, -1, 0)


def test_single_changes_rejected():
    a = W.f2sc_vector(1 << 6, 9)
    msgs, _ = O.f2sc_prove(a, 9)
    for k in range(len(msgs)):
        bad = msgs.copy()
        bad[k] = np.uint64((int(bad[k]) + 1) % P)
        ok, rnd, check = O.f2sc_verify(a, 9, bad)
        assert not ok and check in (2, 5)
    b = a.copy()
    b[3] += 1
    assert not O.f2sc_verify(b, 9, msgs)[0]
    assert O.f2sc_verify(a, 9, msgs[:-1])[2] == 1


def test_rejects_non_power_of_two():
    with pytest.raises(ValueError):
        O.f2sc_prove(np.zeros(3, np.uint32), 1)
