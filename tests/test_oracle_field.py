"""Oracle field and generator pins: F_p arithmetic against Python big
integers (p = 2^61 - 1, Sec. 6.1) and SplitMix64 against its published
known answers."""
import os
import random

import numpy as np
import pytest

from oracle import oracle as O
import brute
import workloads as W

P = O.P
EDGE = [0, 1, 2, 3, P - 1, P - 2, (1 << 60), (1 << 32) - 1, 1 << 32, (1 << 32) + 1,
        (1 << 61) - 3, 12345678901234567]


def test_add_sub_mul_edges():
    for a in EDGE:
        for b in EDGE:
            assert O.add(a, b) == (a + b) % P
            assert O.sub(a, b) == (a - b) % P
            assert O.mul(a, b) == (a * b) % P


def test_random_products():
    rng = random.Random(7)
    for _ in range(20000):
        a, b = rng.randrange(P), rng.randrange(P)
        assert O.mul(a, b) == a * b % P
        assert O.add(a, b) == (a + b) % P


def test_inverse():
    rng = random.Random(8)
    for a in [1, 2, 3, P - 1] + [rng.randrange(1, P) for _ in range(200)]:
        assert O.mul(a, O.inv(a)) == 1
    assert O.inv(2) == 1 << 60  # 2 * 2^60 = 2^61 = 1 mod p


def test_reduce_full_u128():
    rng = random.Random(9)
    for x in [0, P, P + 1, (1 << 128) - 1, (1 << 64) - 1, 1 << 122] + \
             [rng.randrange(1 << 128) for _ in range(1000)]:
        assert O.reduce128(x) == x % P


def _golden():
    path = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_known_answers.txt")
    rows = {}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, v = line.split(":")
        rows[int(k)] = [int(x) for x in v.split()]
    return rows


def test_splitmix_known_answers():
    for state, want in _golden().items():
        # a stream state (seed << 8) | purpose equal to `state`
        seed, purpose = state >> 8, state & 0xFF
        assert [int(v) for v in O.splitmix_raw(seed, purpose, 3)] == want
        assert [int(v) for v in W.splitmix64(seed, purpose, 3)] == want
        assert brute.splitmix64(seed, purpose, 3) == want


def test_splitmix_streams_agree():
    for seed in (0, 1, 2, 3, 4, 5, 123456789):
        for purpose in range(1, 7):
            a = O.splitmix_raw(seed, purpose, 257)
            b = W.splitmix64(seed, purpose, 257)
            assert np.array_equal(a, b)
            assert np.array_equal(W.splitmix64(seed, purpose, 7, start=250), b[250:])


def test_field_draws_are_low_61_bits():
    raw = O.splitmix_raw(5, 2, 400)
    f = O.splitmix_field(5, 2, 399)
    mask = np.uint64(P)
    # no output here has all 61 low bits set, so no redraw happens
    assert not np.any((raw & mask) == mask)
    assert np.array_equal(f, (raw & mask)[:399])
    assert np.all(f < np.uint64(P))
