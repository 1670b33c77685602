"""GPU prover and verifier of the non-interactive F2 protocol (Sec. 3.2,
4.2): proofs bit-exact against the oracle on grids the oracle
finishes quickly (every supported factor, ragged last rows); at Table 3's
universe size (n = 25 million) the proof's F2 value, its degree bound and
the oracle's verifier pin every value; errors and the verifier's rejections."""
import numpy as np
import pytest

from gpu_util import say, device_tensor, oracle_threads
from oracle import oracle as O

pytestmark = pytest.mark.gpu
P = (1 << 61) - 1


def G():
    import paper_1202_1350_amd as mod
    return mod


def values(n, seed, bits=20):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 1 << bits, n).astype(np.uint64)


@pytest.mark.parametrize("n,h", [(1, 3), (10, 3), (100, 9), (1000, 45), (45 * 13 + 7, 45),
                                 (225 * 7 + 200, 225), (585 * 40 + 11, 585), (1287 * 9, 1287),
                                 (2475 * 6 + 3, 2475), (1001 * 5 + 1000, 1001)])
def test_proof_matches_oracle(n, h):
    a = values(n, n + h)
    say("nif2", "n", n, "h", h)
    O.set_threads(oracle_threads())
    want = O.nif2_prove(a, h)
    got = G().nif2_prove(a, h)
    bad = np.nonzero(got != want)[0]
    assert len(bad) == 0, f"first differing values {bad[:5]} of {2 * h}"
    f2 = sum(int(x) ** 2 for x in a) % P
    assert G().nif2_verify(a, h, 7, got) == (True, f2)
    assert O.nif2_verify(a, h, 7, got) == (True, f2)


def test_device_inputs_and_rejections():
    n, h = 585 * 11 + 5, 585
    a = values(n, 3)
    at = device_tensor(a)
    m = G().nif2_prove(at, h)
    assert np.array_equal(m, G().nif2_prove(a, h))
    f2 = sum(int(x) ** 2 for x in a) % P
    assert G().nif2_verify(at, h, 11, m) == (True, f2)
    for k in (0, 1, 2 * h - 1, h):
        bad = m.copy()
        bad[k] = (int(bad[k]) + 5) % P
        assert not G().nif2_verify(a, h, 11, bad)[0], k
    assert not G().nif2_verify(a, h, 11, m[:-1])[0]
    b = a.copy()
    b[100] += np.uint64(1)
    assert not G().nif2_verify(b, h, 11, m)[0]


def test_errors():
    import paper_1202_1350_amd as mod
    a = values(100, 1)
    for h in (2, 31, 41, 61, 4):  # even, or factors without a supported DFT length
        with pytest.raises(mod.GkrError):
            mod.nif2_prove(a, h)
    big = a.copy()
    big[3] = np.uint64(P)
    with pytest.raises(mod.GkrError):
        mod.nif2_prove(big, 45)
    with pytest.raises(mod.GkrError):
        mod.nif2_prove(device_tensor(big), 45)


@pytest.mark.parametrize("h", [5005, 2475, 1287, 585, 45])
def test_table3_size_properties(h):
    """n = 25 million (Table 3): F2 equals the sum of squares, the 2h values
    lie on a polynomial of degree <= 2h - 2, and the oracle's verifier (and
    the GPU's) accepts for two secrets."""
    n = 25_000_000
    a = values(n, 25, bits=16)
    say("nif2 Table 3 size", "h", h)
    at = device_tensor(a)
    m = G().nif2_prove(at, h)
    counts = np.bincount(a.astype(np.int64), minlength=1 << 16)
    f2 = sum(int(c) * x * x for x, c in enumerate(counts.tolist())) % P
    assert sum(int(x) for x in m[0::2]) % P == f2
    xi = O.nif2_root(2 * h)
    acc, xk = 0, 1
    for k in range(2 * h):
        acc = (acc + int(m[k]) * xk) % P
        xk = xk * xi % P
    assert acc == 0
    O.set_threads(oracle_threads())
    for seed in (1, 2):
        assert O.nif2_verify(a, h, seed, m) == (True, f2)
        assert G().nif2_verify(at, h, seed, m) == (True, f2)
