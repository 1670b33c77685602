"""GPU F2 sum-check through the C ABI, bit-exact against the oracle."""
import numpy as np
import pytest

from gpu_util import say, device_tensor, oracle_threads
from oracle import oracle as O
import workloads as W

P = (1 << 61) - 1
pytestmark = pytest.mark.gpu


def G():
    import paper_1202_1350_amd as mod
    return mod


@pytest.mark.parametrize("logn", [0, 1, 2, 3, 4, 9, 10, 11, 17, 20])
def test_bit_exact_small(logn):
    a = W.f2sc_vector(1 << logn, 40 + logn)
    say("f2sc logn", logn)
    want_m, want_c = O.f2sc_prove(a, 7)
    for dev in (False, True):
        got_m, got_c = G().f2_sumcheck_prove(device_tensor(a) if dev else a, 7)
        assert np.array_equal(got_m, want_m)
        assert np.array_equal(got_c, want_c)
    assert G().f2_sumcheck_verify(a, 7, got_m) == (True, -1, 0)


def test_full_values_up_to_2_32():
    a = (W.splitmix64(3, 3, 1 << 12) >> np.uint64(32)).astype(np.uint32)
    a[:4] = np.array([0xFFFFFFFF, 0, 0xFFFFFFFF, 1], np.uint32)
    want_m, _ = O.f2sc_prove(a, 8)
    got_m, _ = G().f2_sumcheck_prove(a, 8)
    assert np.array_equal(got_m, want_m)


def test_rejections():
    a = W.f2sc_vector(1 << 8, 2)
    m, _ = G().f2_sumcheck_prove(a, 2)
    for k in range(len(m)):
        bad = m.copy()
        bad[k] = np.uint64((int(bad[k]) + 1) % P)
        got = G().f2_sumcheck_verify(a, 2, bad)
        assert got == O.f2sc_verify(a, 2, bad), k
        assert not got[0]
    assert G().f2_sumcheck_verify(a, 2, m[:-1])[2] == 1


def test_c2_f2sc_2p26_full_bit_exact():
    a, seed = W.c2_f2sc()
    say("f2sc 2^26 oracle")
    O.set_threads(oracle_threads())
    want_m, want_c = O.f2sc_prove(a, seed)
    say("f2sc 2^26 gpu")
    ta = device_tensor(a)
    got_m, got_c = G().f2_sumcheck_prove(ta, seed)
    assert np.array_equal(got_m, want_m) and np.array_equal(got_c, want_c)
    assert int(got_m[0]) == int((a.astype(np.int64) ** 2).sum()) % P
    assert G().f2_sumcheck_verify(ta, seed, got_m)[0]
