"""Device field module (Sec. 6.1) against Python big integers."""
import random

import numpy as np
import pytest

from gpu_util import say, device_tensor

P = (1 << 61) - 1
pytestmark = pytest.mark.gpu


def test_field_ops_match_integers():
    import torch
    import paper_1202_1350_amd as G
    rng = random.Random(3)
    edge = [0, 1, 2, P - 1, P - 2, 1 << 60, (1 << 32) - 1, 1 << 32, (1 << 32) + 1, (1 << 61) - 3]
    a = [x for x in edge for _ in edge] + [rng.randrange(P) for _ in range(100000)]
    b = [y for _ in edge for y in edge] + [rng.randrange(P) for _ in range(100000)]
    ta = device_tensor(np.array(a, np.uint64))
    tb = device_tensor(np.array(b, np.uint64))
    out = torch.zeros_like(ta)
    for op, f in ((0, lambda x, y: (x + y) % P), (1, lambda x, y: (x - y) % P),
                  (2, lambda x, y: x * y % P)):
        say("field op", op, len(a))
        G.gkr_field_op(op, ta, tb, out)
        got = out.cpu().view(torch.int64).numpy().view(np.uint64)
        want = np.array([f(x, y) for x, y in zip(a, b)], np.uint64)
        assert np.array_equal(got, want), op


def test_lazy_sums_match_integers():
    """64 products summed in 128 bits and reduced once, including the
    largest sums (every factor p - 1)."""
    import torch
    import paper_1202_1350_amd as G
    rng = random.Random(4)
    n = 4096
    a = [P - 1] * 200 + [rng.randrange(P) for _ in range(n - 200)]
    b = [P - 1] * 200 + [rng.randrange(P) for _ in range(n - 200)]
    a[300:310] = [0, 1, 2, 1 << 60, P - 2, 0, 0, 1, P - 1, 3]
    ta = device_tensor(np.array(a, np.uint64))
    tb = device_tensor(np.array(b, np.uint64))
    out = torch.zeros_like(ta)
    say("lazy sums", n)
    G.gkr_field_op(3, ta, tb, out)
    got = out.cpu().view(torch.int64).numpy().view(np.uint64)
    want = np.array([sum(a[(k + j) % n] * b[(k + j) % n] for j in range(64)) % P
                     for k in range(n)], np.uint64)
    assert np.array_equal(got, want)


def test_product_chains_match_integers():
    import torch
    import paper_1202_1350_amd as G
    rng = random.Random(5)
    a = [0, 1, P - 1, 2] + [rng.randrange(P) for _ in range(2000)]
    b = [P - 1, P - 1, P - 1, 2] + [rng.randrange(P) for _ in range(2000)]
    ta = device_tensor(np.array(a, np.uint64))
    tb = device_tensor(np.array(b, np.uint64))
    out = torch.zeros_like(ta)
    say("product chains", len(a))
    G.gkr_field_op(4, ta, tb, out)
    got = out.cpu().view(torch.int64).numpy().view(np.uint64)
    want = np.array([x * pow(y, 256, P) % P for x, y in zip(a, b)], np.uint64)
    assert np.array_equal(got, want)
