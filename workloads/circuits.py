"""Wiring of the layered fan-in-2 circuits the paper benchmarks (Sec. 5.2.1).

Layers are numbered 0 = output ... d = input.  Layer i < d has gate type
(0 = ADD, 1 = MUL) and two wires into layer i+1 per gate; a wire may name a
zero padding slot of layer i+1 (index < 2^ceil(log2 S_{i+1})).
"""
from dataclasses import dataclass, field
from typing import List

import numpy as np

ADD, MUL = 0, 1


@dataclass
class Circuit:
    sizes: List[int]                      # [d+1], sizes[0] = output layer
    types: List[np.ndarray] = field(default_factory=list)   # [d] uint8
    in1: List[np.ndarray] = field(default_factory=list)     # [d] uint32
    in2: List[np.ndarray] = field(default_factory=list)     # [d] uint32
    name: str = ""

    @property
    def depth(self) -> int:
        return len(self.sizes) - 1

    @property
    def gates(self) -> int:
        """All gates including the input layer (how Table 2 counts)."""
        return int(sum(self.sizes))


def _sum_tree(sizes, types, in1, in2, width):
    """Binary ADD tree from `width` values down to one: gate g adds 2g, 2g+1.
    An odd tail reads the zero padding slot.  Layers are prepended (they sit
    nearer the output)."""
    while width > 1:
        half = (width + 1) // 2
        g = np.arange(half, dtype=np.uint32)
        sizes.insert(0, half)
        types.insert(0, np.zeros(half, np.uint8))
        in1.insert(0, 2 * g)
        in2.insert(0, 2 * g + 1)
        width = half


def f2_circuit(n: int) -> Circuit:
    """F2 = sum_i a_i^2: a layer of MUL gates squaring each input, then a
    binary ADD tree (the paper's single large-fan-in sum gate, Sec. 5.2.1,
    written as fan-in-2 adds).  n = 2^k gives 3n - 1 gates."""
    assert n >= 1
    g = np.arange(n, dtype=np.uint32)
    sizes, types, in1, in2 = [n, n], [np.ones(n, np.uint8)], [g.copy()], [g.copy()]
    _sum_tree(sizes, types, in1, in2, n)
    return Circuit(sizes, types, in1, in2, name=f"F2 n={n}")


def matmult_circuit(N: int) -> Circuit:
    """C = AB for N x N matrices (N a power of two).  Inputs: A row-major
    (index i*N+k) then B row-major (N^2 + k*N + j).  MUL gate (i*N+j)*N+k
    forms A_ik B_kj; log2 N ADD layers sum over k; output gate i*N+j is C_ij."""
    assert N >= 1 and N & (N - 1) == 0
    idx = np.arange(N ** 3, dtype=np.uint64)
    i, j, k = idx // (N * N), (idx // N) % N, idx % N
    sizes = [N ** 3, 2 * N * N]
    types = [np.ones(N ** 3, np.uint8)]
    in1 = [(i * N + k).astype(np.uint32)]
    in2 = [(N * N + k * N + j).astype(np.uint32)]
    _sum_tree_rows(sizes, types, in1, in2, N * N, N)
    return Circuit(sizes, types, in1, in2, name=f"MatMult N={N}")


def _sum_tree_rows(sizes, types, in1, in2, rows, width):
    """rows independent ADD trees over `width` adjacent values each."""
    while width > 1:
        half = width // 2
        g = np.arange(rows * half, dtype=np.uint32)
        sizes.insert(0, rows * half)
        types.insert(0, np.zeros(rows * half, np.uint8))
        in1.insert(0, 2 * g)
        in2.insert(0, 2 * g + 1)
        width = half


def pm_circuit(n: int, q: int = 8) -> Circuit:
    """Pattern matching distances: for each shift i < M = n - q + 1,
    D_i = sum_j (t_{i+j} - p_j)^2, zero exactly where the pattern occurs.
    Inputs: text t_0..t_{n-1}, then the negated pattern (p - p_j) mod p, so an
    ADD gate forms t_{i+j} - p_j; a MUL gate squares it; log2 q ADD layers sum
    over j.  q must be a power of two."""
    assert q >= 1 and q & (q - 1) == 0 and n >= q
    M = n - q + 1
    g = np.arange(M * q, dtype=np.uint64)
    i, j = g // q, g % q
    sizes = [M * q, M * q, n + q]
    types = [np.ones(M * q, np.uint8), np.zeros(M * q, np.uint8)]
    in1 = [g.astype(np.uint32), (i + j).astype(np.uint32)]
    in2 = [g.astype(np.uint32), (n + j).astype(np.uint32)]
    _sum_tree_rows(sizes, types, in1, in2, M, q)
    return Circuit(sizes, types, in1, in2, name=f"PM n={n} q={q}")
