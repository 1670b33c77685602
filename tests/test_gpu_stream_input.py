"""The verifiers' input extension over host inputs, streamed in chunks of
2^23 values on a copy stream: verdicts equal those on device inputs,
over several chunks with a ragged last one, a changed input in a later
chunk is caught by the final check (the inputs' extension, Sec. 4.1.2), and
a value not below p is an error."""
import numpy as np
import pytest

from gpu_util import say, device_tensor
import workloads as W

P = (1 << 61) - 1
pytestmark = pytest.mark.gpu
CHUNK = 1 << 23


def G():
    import paper_1202_1350_amd as mod
    return mod


def test_gkr_verify_host_inputs_stream_over_chunks():
    n = 3 * CHUNK + 5  # four chunks, the last of 5 values
    circ = W.f2_circuit(n)
    x = W.f2_inputs(n, 11)
    gc = G().Circuit.from_workload(circ)
    xt = device_tensor(x)
    say("stream input: prove F2 n", n)
    m, _ = G().gkr_prove(gc, xt, 11, want_chals=False)
    say("stream input: verify host and device inputs")
    assert G().gkr_verify(gc, x, 11, m) == (True, -1, -1, 0)
    assert G().gkr_verify(gc, xt, 11, m) == (True, -1, -1, 0)
    for pos in (2 * CHUNK + 17, n - 1, 0):
        y = x.copy()
        y[pos] = np.uint64((int(y[pos]) + 1) % P)
        say("stream input: changed input at", pos)
        host = G().gkr_verify(gc, y, 11, m)
        dev = G().gkr_verify(gc, device_tensor(y), 11, m)
        assert host == dev and not host[0] and host[3] == 5, (pos, host, dev)
    y = x.copy()
    y[n - 2] = np.uint64(P)
    for on_dev in (False, True):
        say("stream input: value p, device", on_dev)
        with pytest.raises(G().GkrError) as e:
            G().gkr_verify(gc, device_tensor(y) if on_dev else y, 11, m)
        assert e.value.code == G().GKR_ERR_RANGE
    say("stream input: honest again after the error")
    assert G().gkr_verify(gc, x, 11, m)[0]


def test_f2_sumcheck_verify_host_vector_streams_over_chunks():
    a = W.f2sc_vector(1 << 25, 12)  # four chunks
    at = device_tensor(a)
    say("stream input: F2 sum-check prove 2^25")
    fm, _ = G().f2_sumcheck_prove(at, 12)
    say("stream input: F2 sum-check verify host and device")
    assert G().f2_sumcheck_verify(a, 12, fm)[0]
    assert G().f2_sumcheck_verify(at, 12, fm)[0]
    b = a.copy()
    b[3 * CHUNK + 99] ^= np.uint32(1)
    host = G().f2_sumcheck_verify(b, 12, fm)
    dev = G().f2_sumcheck_verify(device_tensor(b), 12, fm)
    assert host == dev and not host[0], (host, dev)
