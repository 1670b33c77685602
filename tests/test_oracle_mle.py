"""Pins of the oracle's multilinear-extension machinery against the
definition ~T(r) = sum_x chi_x(r) T[x] and its properties."""
import random

import numpy as np

from oracle import oracle as O
import brute

P = O.P


def _rand(rng, n):
    return [rng.randrange(P) for _ in range(n)]


def test_boolean_points_give_table_entries():
    rng = random.Random(1)
    for s in range(0, 6):
        T = np.array(_rand(rng, 1 << s), np.uint64)
        for x in range(1 << s):
            pt = [(x >> k) & 1 for k in range(s)]
            assert O.mle(T, pt) == int(T[x])


def test_mle_matches_definition():
    rng = random.Random(2)
    for s in range(0, 7):
        for _ in range(5):
            T = _rand(rng, 1 << s)
            r = _rand(rng, s)
            assert O.mle(np.array(T, np.uint64), r) == brute.mle(T, r)


def test_mle_is_affine_in_each_coordinate():
    rng = random.Random(3)
    T = np.array(_rand(rng, 32), np.uint64)
    r = _rand(rng, 5)
    for k in range(5):
        vals = []
        for t in (0, 1, 2):
            q = list(r)
            q[k] = t
            vals.append(O.mle(T, q))
        assert (2 * vals[1] - vals[0]) % P == vals[2]


def test_eq_table_sums_to_one_and_matches_chi():
    rng = random.Random(4)
    for s in range(0, 8):
        r = _rand(rng, s)
        E = O.eq_table(r)
        assert int(sum(int(e) for e in E) % P) == 1
        for x in rng.sample(range(1 << s), min(1 << s, 20)):
            assert int(E[x]) == brute.chi(x, r)


def test_lagrange_reproduces_polynomials():
    rng = random.Random(5)
    for D in range(1, 8):
        coef = _rand(rng, D + 1)
        poly = lambda x: sum(c * pow(x, k, P) for k, c in enumerate(coef)) % P
        y = [poly(t) for t in range(D + 1)]
        for x in [0, 1, D, D + 1, rng.randrange(P)]:
            assert O.lagrange(y, x) == poly(x)
