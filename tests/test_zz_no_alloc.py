"""f2_sumcheck_prove_noalloc (scratch in the library's static device array,
no allocation in the call) against f2_sumcheck_prove and the oracle: two
calls in a row, the second smaller, so the second runs on what the first
left in the array; host and device inputs; the size limit."""
import numpy as np
import pytest

from gpu_util import say, device_tensor
from oracle import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def G():
    import paper_1202_1350_amd as mod
    return mod


@pytest.mark.parametrize("on_device", [True, False])
def test_noalloc_equals_allocating_entry_point(on_device):
    for logn, seed in ((22, 11), (13, 12), (1, 13), (0, 14), (17, 15)):
        a = W.f2sc_vector(1 << logn, seed)
        arg = device_tensor(a) if on_device else a
        say("noalloc F2 sum-check, log n", logn, "seed", seed, "device" if on_device else "host")
        m, c = G().f2_sumcheck_prove_noalloc(arg, seed)
        m_ref, c_ref = G().f2_sumcheck_prove(arg, seed)
        assert np.array_equal(m, m_ref), (logn, np.nonzero(m != m_ref)[0][:5])
        assert np.array_equal(c, c_ref)
        if logn <= 17:
            om, oc = O.f2sc_prove(a, seed)
            assert np.array_equal(m, om) and np.array_equal(c, oc)
        assert G().f2_sumcheck_verify(arg, seed, m)[0]


def test_noalloc_rejects_sizes_above_its_limit():
    a = device_tensor(np.zeros(1 << 23, np.uint32))
    with pytest.raises(G().GkrError) as e:
        G().f2_sumcheck_prove_noalloc(a, 1)
    assert e.value.code == G().GKR_ERR_NOMEM
