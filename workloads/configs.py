"""Seeded synthetic workloads of the benchmark configurations.

The paper generated its data at random (Sec. 6.2.4, unverifiable F2); these
are uniform integers drawn from SplitMix64 streams (see prng.py), with the
sizes of the workloads measured:
  F2 GKR:       n inputs uniform in [0, 2^20), seed s, purpose 1
  F2 sum-check: n values uniform in [0, 2^16), purpose 3
  MatMult:      A then B (row-major) uniform in [0, 2^10), purpose 1
  PM:           text uniform in [0, 256), purpose 1; pattern = the q symbols
                of the text at a position drawn from purpose 6, so at least
                one occurrence exists
  F0:           n frequencies uniform in [0, 16), purpose 1 (about one in
                sixteen is zero)
  MatMult-check: A, B as MatMult; C = AB, then `bad` entries (positions
                from purpose 7) increased by one; inputs A, B, -C mod p
"""
import math

import numpy as np

from .circuits import (f2_circuit, matmult_circuit, pm_circuit, f0_circuit, pm_f0_circuit,
                       matmult_check_circuit)
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


def f0_inputs(n: int, seed: int, bits: int = 4) -> np.ndarray:
    return uniform_bits(seed, 1, n, bits).astype(np.uint64)


def matmult_check_inputs(N: int, seed: int, bad: int = 0):
    """(input vector A, B, -C mod p; the number of entries where C != AB).
    C = AB exactly (entries below 2^28), then `bad` distinct entries + 1."""
    ab = matmult_inputs(N, seed)
    A = ab[:N * N].reshape(N, N).astype(np.int64)
    B = ab[N * N:].reshape(N, N).astype(np.int64)
    C = (A @ B).reshape(-1)
    wrong = 0
    if bad:
        pos = np.unique(splitmix64(seed, 7, 4 * bad) % np.uint64(N * N))[:bad].astype(np.int64)
        C[pos] += 1
        wrong = len(pos)
    negC = (np.uint64(P) - C.astype(np.uint64)) % np.uint64(P)
    return np.concatenate([ab, negC]).astype(np.uint64), wrong


# Table 2's other three problems, built on the F0 (Fermat) stage.
def f1_f0(log_n: int = 21):
    """F0 GKR, n = 2^21 (Table 2: 2.1 million inputs), seed 6."""
    n = 1 << log_n
    return f0_circuit(n), f0_inputs(n, 6), 6


def f1_pm_f0(log_n: int = 19, q: int = 8):
    """Pattern matching with the F0 count, text 2^19 (Table 2: 524,288), q = 8, seed 7."""
    n = 1 << log_n
    return pm_f0_circuit(n, q), pm_inputs(n, 7, q)[0], 7


def f1_matmult_check(N: int = 256):
    """MatMult with the C = AB check, N = 256 (Table 2: 65,536 entries), seed 8."""
    return matmult_check_circuit(N), matmult_check_inputs(N, 8)[0], 8
