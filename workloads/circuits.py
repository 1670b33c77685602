"""Wiring of the layered fan-in-2 circuits the paper benchmarks (Sec. 6.2.1).

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
    binary ADD tree (the paper's single large-fan-in sum gate, Sec. 6.2.1,
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


# ----------------------------------------------------------------------
# F0 (Sec. 6.2.1): Fermat's little theorem sends x to x^(p-1) = 1 for x != 0
# and 0 for x = 0, so summing x^(p-1) counts the non-zero values.  p - 1 =
# 2^61 - 2 = 2 + 4 + ... + 2^60.  Two tracks of MUL gates per value: s_L =
# x^(2^L) squares itself; the accumulator a starts one layer later as
# s_1 + s_1 (an ADD gate, so no constant or copy gate is needed) and
# multiplies in s_{L-1} on every layer, a_L = 2 x^(2^L - 2), so a_61 =
# 2 x^(p-1): the circuit's output is 2 F0.  Per value: 1 + 2*59 + 1 gates,
# with the input and the sum tree 122 per input, as in Table 2.

F0_SQUARINGS = 61  # layers of the Fermat stage


def _fermat_stage(sizes, types, in1, in2, n, base=0):
    """Prepend the Fermat stage over n values at indices base.. of the
    current top layer; leaves 2 x^(p-1) of value e at index e of the new top
    layer (n gates)."""
    e = np.arange(n, dtype=np.uint32)
    # layer 1: s_1 = x * x
    sizes.insert(0, n)
    types.insert(0, np.ones(n, np.uint8))
    in1.insert(0, (base + e).astype(np.uint32))
    in2.insert(0, (base + e).astype(np.uint32))
    for L in range(2, F0_SQUARINGS):
        # s_L = s_{L-1}^2 at [0, n); a_L at [n, 2n): s_1 + s_1 (L = 2),
        # else a_{L-1} * s_{L-1}
        sizes.insert(0, 2 * n)
        t = np.ones(2 * n, np.uint8)
        if L == 2:
            t[n:] = 0
            a_in = e
        else:
            a_in = n + e
        types.insert(0, t)
        in1.insert(0, np.concatenate([e, a_in]).astype(np.uint32))
        in2.insert(0, np.concatenate([e, e]).astype(np.uint32))
    # layer 61: a_61 = a_60 * s_60
    sizes.insert(0, n)
    types.insert(0, np.ones(n, np.uint8))
    in1.insert(0, (n + e).astype(np.uint32))
    in2.insert(0, e.copy())


def f0_circuit(n: int) -> Circuit:
    """2 F0 = 2 |{i : a_i != 0}| of n values: the Fermat stage, then a
    binary ADD tree.  122 n - 1 gates."""
    assert n >= 1
    sizes, types, in1, in2 = [n], [], [], []
    _fermat_stage(sizes, types, in1, in2, n)
    _sum_tree(sizes, types, in1, in2, n)
    return Circuit(sizes, types, in1, in2, name=f"F0 n={n}")


def pm_f0_circuit(n: int, q: int = 8) -> Circuit:
    """Pattern matching with one output: the distances D_i of pm_circuit
    (zero exactly where the pattern occurs), then the Fermat stage and a sum:
    the output is 2 |{i : D_i != 0}|, twice the number of shifts where the
    pattern does not occur.  About 145 gates per input for q = 8."""
    c = pm_circuit(n, q)  # its top layer holds the M distances
    M = n - q + 1
    sizes, types, in1, in2 = list(c.sizes), list(c.types), list(c.in1), list(c.in2)
    _fermat_stage(sizes, types, in1, in2, M)
    _sum_tree(sizes, types, in1, in2, M)
    return Circuit(sizes, types, in1, in2, name=f"PM-F0 n={n} q={q}")


def matmult_check_circuit(N: int) -> Circuit:
    """One output that is zero iff C = AB, for N x N matrices (N a power of
    two, N >= 2).  Inputs: A row-major (i*N+k), B row-major (N^2 + k*N + j),
    then -C mod p row-major (2 N^2 + i*N + j).  The product layer and the
    ADD tree of matmult_circuit, each layer also carrying -C_ij up in N^2
    gates that add a zero padding slot of the layer below; then D_ij =
    (AB)_ij - C_ij, the Fermat stage over the N^2 values D, and a sum: the
    output is 2 |{(i, j) : (AB)_ij != C_ij}|."""
    assert N >= 2 and N & (N - 1) == 0
    NN = N * N
    idx = np.arange(N ** 3, dtype=np.uint64)
    i, j, k = idx // NN, (idx // N) % N, idx % N
    m = np.arange(NN, dtype=np.uint32)
    # product layer + carried -C (zero slot 3 N^2 of the input layer)
    sizes = [N ** 3 + NN, 3 * NN]
    types = [np.concatenate([np.ones(N ** 3, np.uint8), np.zeros(NN, np.uint8)])]
    in1 = [np.concatenate([(i * N + k).astype(np.uint32), 2 * NN + m])]
    in2 = [np.concatenate([(NN + k * N + j).astype(np.uint32), np.full(NN, 3 * NN, np.uint32)])]
    width = N
    while width > 1:
        half = width // 2
        below = NN * width + NN  # size of the layer below; its -C copies start at NN * width
        g = np.arange(NN * half, dtype=np.uint32)
        sizes.insert(0, NN * half + NN)
        types.insert(0, np.zeros(NN * half + NN, np.uint8))
        in1.insert(0, np.concatenate([2 * g, NN * width + m]).astype(np.uint32))
        in2.insert(0, np.concatenate([2 * g + 1, np.full(NN, below, np.uint32)]).astype(np.uint32))
        width = half
    # D = (AB) + (-C): the top layer holds AB at [0, NN), -C at [NN, 2 NN)
    sizes.insert(0, NN)
    types.insert(0, np.zeros(NN, np.uint8))
    in1.insert(0, m.copy())
    in2.insert(0, NN + m)
    _fermat_stage(sizes, types, in1, in2, NN)
    _sum_tree(sizes, types, in1, in2, NN)
    return Circuit(sizes, types, in1, in2, name=f"MatMult-check N={N}")
