"""The oracle of the non-interactive F2 protocol (Sec. 3.2), pinned
to definitions computed here independently: the F2 value, the degree bound
of the proof polynomial, a brute-force interpolation of every row on tiny
grids, the subgroup orders, completeness and soundness."""
import numpy as np
import pytest

from oracle import oracle as O

P = (1 << 61) - 1
PRIMES_OF_P_MINUS_1 = [2, 3, 5, 7, 11, 13, 31, 41, 61, 151, 331, 1321]


def interp_eval(xs, ys, x):
    """The polynomial of degree < len(xs) through (xs, ys) at x (plain
    Lagrange over arbitrary distinct points, Python integers)."""
    total = 0
    for i, (xi, yi) in enumerate(zip(xs, ys)):
        num, den = 1, 1
        for j, xj in enumerate(xs):
            if j != i:
                num = num * (x - xj) % P
                den = den * (xi - xj) % P
        total = (total + yi * num * pow(den, P - 2, P)) % P
    return total


def grid(a, h):
    v = -(-len(a) // h)
    return v, [[int(a[j * v + y]) if j * v + y < len(a) else 0 for j in range(h)] for y in range(v)]


@pytest.mark.parametrize("N", [3, 5, 9, 15, 45, 90, 585, 1170, 5005, 10010])
def test_subgroup_generators_have_order_N(N):
    w = O.nif2_root(N)
    assert pow(w, N, P) == 1
    for q in PRIMES_OF_P_MINUS_1:
        if N % q == 0:
            assert pow(w, N // q, P) != 1
    assert O.nif2_root(4) == 0 and O.nif2_root(1000) == 0  # 4 does not divide p - 1


@pytest.mark.parametrize("n,h", [(1, 3), (7, 3), (20, 5), (31, 9), (45, 15)])
def test_proof_equals_brute_force_interpolation(n, h):
    rng = np.random.default_rng(n * 100 + h)
    a = rng.integers(0, 1 << 20, n).astype(np.uint64)
    msgs = O.nif2_prove(a, h)
    v, rows = grid(a, h)
    wh, xi = pow(37, (P - 1) // h, P), pow(37, (P - 1) // (2 * h), P)
    xs = [pow(wh, j, P) for j in range(h)]
    for k in range(2 * h):
        x = pow(xi, k, P)
        want = sum(interp_eval(xs, row, x) ** 2 for row in rows) % P
        assert int(msgs[k]) == want, k


@pytest.mark.parametrize("n,h", [(100, 9), (1000, 45), (4000, 585)])
def test_f2_value_and_degree_bound(n, h):
    rng = np.random.default_rng(n + h)
    a = rng.integers(0, 1 << 20, n).astype(np.uint64)
    msgs = [int(m) for m in O.nif2_prove(a, h)]
    assert sum(msgs[0::2]) % P == sum(int(x) ** 2 for x in a) % P
    # g has degree <= 2h - 2: its coefficient of X^(2h-1) over the order-2h
    # subgroup, (1/2h) sum_k g(xi^k) xi^(-k(2h-1)) = (1/2h) sum_k g(xi^k) xi^k, is 0
    xi = O.nif2_root(2 * h)
    assert sum(m * pow(xi, k, P) for k, m in enumerate(msgs)) % P == 0


def test_completeness_and_soundness():
    rng = np.random.default_rng(7)
    a = rng.integers(0, 1 << 16, 200).astype(np.uint64)
    h = 15
    msgs = O.nif2_prove(a, h)
    f2 = sum(int(x) ** 2 for x in a) % P
    for seed in range(1, 6):
        assert O.nif2_verify(a, h, seed, msgs) == (True, f2)
    for k in range(2 * h):  # every single changed value is caught
        bad = msgs.copy()
        bad[k] = (int(bad[k]) + 1 + k) % P
        assert not O.nif2_verify(a, h, 3, bad)[0], k
    b = a.copy()
    b[17] += np.uint64(1)  # a different stream
    assert not O.nif2_verify(b, h, 3, msgs)[0]
    assert not O.nif2_verify(a, h, 3, msgs[:-1])[0]  # wrong length


def test_rejects_h_without_subgroups():
    a = np.ones(10, np.uint64)
    for h in (2, 4, 10, 17):
        with pytest.raises(ValueError):
            O.nif2_prove(a, h)
