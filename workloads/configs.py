"""Seeded synthetic workloads of the benchmark configurations.

The paper generated its data at random (Sec. 5.2.5, unverifiable F2); these
are uniform integers drawn from SplitMix64 streams (see prng.py), with the
sizes of the workloads measured:
  F2 GKR:       n inputs uniform in [0, 2^20), seed s, purpose 1
  F2 sum-check: n values uniform in [0, 2^16), purpose 3
  MatMult:      A then B (row-major) uniform in [0, 2^10), purpose 1
  PM:           text uniform in [0, 256), purpose 1; pattern = the q symbols
                of the text at a position drawn from purpose 6, so at least
                one occurrence exists
"""
import math

import numpy as np

from .circuits import f2_circuit, matmult_circuit, pm_circuit
from .prng import splitmix64, uniform_bits

P = (1 << 61) - 1


def f2_inputs(n: int, seed: int, bits: int = 20) -> np.ndarray:
    return uniform_bits(seed, 1, n, bits).astype(np.uint64)


def matmult_inputs(N: int, seed: int, bits: int = 10) -> np.ndarray:
    return uniform_bits(seed, 1, 2 * N * N, bits).astype(np.uint64)


def pm_inputs(n: int, seed: int, q: int = 8):
    """(input vector, text, pattern)."""
    text = uniform_bits(seed, 1, n, 8).astype(np.uint64)
    pos = int(splitmix64(seed, 6, 1)[0] % np.uint64(n - q + 1))
    pat = text[pos:pos + q].copy()
    neg = (np.uint64(P) - pat) % np.uint64(P)
    return np.concatenate([text, neg]).astype(np.uint64), text, pat


def f2sc_vector(n: int, seed: int, bits: int = 16) -> np.ndarray:
    return uniform_bits(seed, 3, n, bits).astype(np.uint32)


def c1_f2():
    """F2 GKR, n = 2^10, seed 1."""
    return f2_circuit(1 << 10), f2_inputs(1 << 10, 1), 1


def c2_f2(log_n: int = 22):
    """F2 GKR, n = 2^22, seed 2."""
    n = 1 << log_n
    return f2_circuit(n), f2_inputs(n, 2), 2


def c2_f2sc(log_n: int = 26):
    """F2 sum-check on a length-2^26 vector, seed 2."""
    return f2sc_vector(1 << log_n, 2), 2


def c3_matmult(N: int = 256):
    """MatMult N = 256, seed 3."""
    return matmult_circuit(N), matmult_inputs(N, 3), 3


def batch_mix(seed: int = 4, count: int = 64, f2_range=(12, 20), pm_range=(14, 18), q=8):
    """Uneven batch: proof k even is F2 with n = floor(2^u), u ~ U[12, 20];
    k odd is PM with text length floor(2^u), u ~ U[14, 18].  Per-proof seeds
    and the u draws come from purpose 5 of `seed`.  Returns a list of
    (kind, circuit, inputs, proof_seed)."""
    draws = splitmix64(seed, 5, 2 * count)
    out = []
    for k in range(count):
        u01 = float(draws[2 * k] >> np.uint64(11)) / float(1 << 53)
        pseed = int(draws[2 * k + 1] >> np.uint64(8))
        if k % 2 == 0:
            lo, hi = f2_range
            n = int(math.floor(2.0 ** (lo + (hi - lo) * u01)))
            out.append(("F2", f2_circuit(n), f2_inputs(n, pseed), pseed))
        else:
            lo, hi = pm_range
            n = int(math.floor(2.0 ** (lo + (hi - lo) * u01)))
            inp, _, _ = pm_inputs(n, pseed, q)
            out.append(("PM", pm_circuit(n, q), inp, pseed))
    return out
