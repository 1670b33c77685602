"""ctypes binding of the CPU oracle (gkr_oracle.c).

TEST INFRASTRUCTURE ONLY: the slow reference the GPU path is checked
against.  Only the tests, the smoke entry point and the benchmark's
CPU-baseline leg may import this module.  It imports nothing from the GPU
package.
"""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gkr_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
P = (1 << 61) - 1

u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11 + pthreads)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC",
                               "-pthread", SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        for name in ("or_field_add", "or_field_sub", "or_field_mul"):
            getattr(L, name).restype = C.c_uint64
            getattr(L, name).argtypes = [C.c_uint64, C.c_uint64]
        L.or_field_inv.restype = C.c_uint64
        L.or_field_inv.argtypes = [C.c_uint64]
        L.or_field_reduce_u128.restype = C.c_uint64
        L.or_field_reduce_u128.argtypes = [C.c_uint64, C.c_uint64]
        L.or_splitmix_raw.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, u64p]
        L.or_splitmix_field.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, u64p]
        L.or_set_threads.argtypes = [C.c_int]
        L.or_log2ceil.restype = C.c_uint32
        L.or_log2ceil.argtypes = [C.c_uint64]
        L.or_mle.restype = C.c_uint64
        L.or_mle.argtypes = [u64p, C.c_uint32, u64p]
        L.or_eq_table.argtypes = [u64p, C.c_uint32, u64p]
        L.or_lagrange.restype = C.c_uint64
        L.or_lagrange.argtypes = [u64p, C.c_uint32, C.c_uint64]
        L.or_transcript_size.argtypes = [C.c_uint32, u32p, C.POINTER(C.c_uint64),
                                         C.POINTER(C.c_uint64)]
        L.or_nif2_root.restype = C.c_uint64
        L.or_nif2_root.argtypes = [C.c_uint64]
        L.or_nif2_prove.argtypes = [u64p, C.c_uint64, C.c_uint64, u64p]
        L.or_nif2_verify.argtypes = [u64p, C.c_uint64, C.c_uint64, C.c_uint64, u64p, C.c_uint64,
                                     C.POINTER(C.c_int), C.POINTER(C.c_uint64)]
        _circ = [C.c_uint32, u32p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_check_circuit.argtypes = _circ
        L.or_evaluate.argtypes = _circ + [u64p, C.c_void_p]
        L.or_prove.argtypes = _circ + [u64p, C.c_uint64, u64p, u64p]
        L.or_verify.argtypes = _circ + [u64p, C.c_uint64, u64p, C.c_uint64,
                                        C.POINTER(C.c_int), C.POINTER(C.c_int),
                                        C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.or_f2sc_prove.argtypes = [u32p, C.c_uint64, C.c_uint64, u64p, u64p]
        L.or_f2sc_verify.argtypes = [u32p, C.c_uint64, C.c_uint64, u64p, C.c_uint64,
                                     C.POINTER(C.c_int), C.POINTER(C.c_int),
                                     C.POINTER(C.c_int)]
        _lib = L
    return _lib


def set_threads(t: int):
    lib().or_set_threads(int(t))


# ------------------------------------------------------------ field + PRNG
def add(a, b): return int(lib().or_field_add(a, b))
def sub(a, b): return int(lib().or_field_sub(a, b))
def mul(a, b): return int(lib().or_field_mul(a, b))
def inv(a): return int(lib().or_field_inv(a))
def reduce128(x: int) -> int: return int(lib().or_field_reduce_u128(x >> 64, x & ((1 << 64) - 1)))


def splitmix_raw(seed, purpose, n):
    out = np.zeros(n, np.uint64)
    lib().or_splitmix_raw(seed, purpose, n, out)
    return out


def splitmix_field(seed, purpose, n):
    out = np.zeros(n, np.uint64)
    lib().or_splitmix_field(seed, purpose, n, out)
    return out


def log2ceil(n): return int(lib().or_log2ceil(n))


def mle(table, point):
    table = np.ascontiguousarray(table, np.uint64)
    point = np.ascontiguousarray(point, np.uint64)
    s = len(point)
    assert len(table) == 1 << s
    return int(lib().or_mle(table, s, point if s else np.zeros(1, np.uint64)))


def eq_table(point):
    point = np.ascontiguousarray(point, np.uint64)
    s = len(point)
    E = np.zeros(1 << s, np.uint64)
    lib().or_eq_table(point if s else np.zeros(1, np.uint64), s, E)
    return E


def lagrange(y, x):
    y = np.ascontiguousarray(y, np.uint64)
    return int(lib().or_lagrange(y, len(y) - 1, x))


# ----------------------------------------------------------------- circuits
class _Marshal:
    """Keeps the per-layer arrays alive and exposes pointer arrays."""

    def __init__(self, circ):
        self.S = np.ascontiguousarray(circ.sizes, np.uint32)
        self.L = len(circ.sizes)
        self.keep = []
        d = self.L - 1
        self.types = (C.c_void_p * max(d, 1))()
        self.in1 = (C.c_void_p * max(d, 1))()
        self.in2 = (C.c_void_p * max(d, 1))()
        for i in range(d):
            t = np.ascontiguousarray(circ.types[i], np.uint8)
            a = np.ascontiguousarray(circ.in1[i], np.uint32)
            b = np.ascontiguousarray(circ.in2[i], np.uint32)
            self.keep += [t, a, b]
            self.types[i] = t.ctypes.data
            self.in1[i] = a.ctypes.data
            self.in2[i] = b.ctypes.data

    def args(self):
        return (self.L, self.S, C.cast(self.types, C.c_void_p), C.cast(self.in1, C.c_void_p),
                C.cast(self.in2, C.c_void_p))


def transcript_size(circ):
    S = np.ascontiguousarray(circ.sizes, np.uint32)
    m, c = C.c_uint64(), C.c_uint64()
    lib().or_transcript_size(len(S), S, C.byref(m), C.byref(c))
    return m.value, c.value


def check_circuit(circ) -> bool:
    return lib().or_check_circuit(*_Marshal(circ).args()) == 0


def evaluate(circ, inputs):
    """All layer tables, each zero-padded to a power of two."""
    M = _Marshal(circ)
    V = [np.zeros(1 << log2ceil(S), np.uint64) for S in circ.sizes]
    ptrs = (C.c_void_p * len(V))(*[v.ctypes.data for v in V])
    rc = lib().or_evaluate(*M.args(), np.ascontiguousarray(inputs, np.uint64),
                           C.cast(ptrs, C.c_void_p))
    if rc:
        raise ValueError("malformed circuit")
    return V


def prove(circ, inputs, seed):
    M = _Marshal(circ)
    nm, nc = transcript_size(circ)
    msgs = np.zeros(max(nm, 1), np.uint64)
    chals = np.zeros(max(nc, 1), np.uint64)
    rc = lib().or_prove(*M.args(), np.ascontiguousarray(inputs, np.uint64), seed, msgs, chals)
    if rc:
        raise ValueError(f"or_prove failed ({rc})")
    return msgs[:nm], chals[:nc]


def verify(circ, inputs, seed, msgs):
    """(accepted, layer, round, check)."""
    M = _Marshal(circ)
    msgs = np.ascontiguousarray(msgs, np.uint64)
    acc, wl, wr, wc = C.c_int(), C.c_int(), C.c_int(), C.c_int()
    buf = msgs if len(msgs) else np.zeros(1, np.uint64)
    rc = lib().or_verify(*M.args(), np.ascontiguousarray(inputs, np.uint64), seed, buf,
                         len(msgs), C.byref(acc), C.byref(wl), C.byref(wr), C.byref(wc))
    if rc:
        raise ValueError(f"or_verify failed ({rc})")
    return bool(acc.value), wl.value, wr.value, wc.value


def f2sc_prove(freq, seed):
    freq = np.ascontiguousarray(freq, np.uint32)
    n = len(freq)
    l = log2ceil(n)
    msgs = np.zeros(1 + 3 * l, np.uint64)
    chals = np.zeros(max(l, 1), np.uint64)
    rc = lib().or_f2sc_prove(freq, n, seed, msgs, chals)
    if rc:
        raise ValueError("n must be a power of two")
    return msgs, chals[:l]


def f2sc_verify(freq, seed, msgs):
    freq = np.ascontiguousarray(freq, np.uint32)
    msgs = np.ascontiguousarray(msgs, np.uint64)
    acc, wr, wc = C.c_int(), C.c_int(), C.c_int()
    rc = lib().or_f2sc_verify(freq, len(freq), seed, msgs, len(msgs), C.byref(acc),
                              C.byref(wr), C.byref(wc))
    if rc:
        raise ValueError("n must be a power of two")
    return bool(acc.value), wr.value, wc.value


# Non-interactive F2 (Sec. 3.2): a v x h grid, proof g at 2h points.
def nif2_root(N):
    """Generator of the order-N subgroup of F_p^* (0 if N does not divide p - 1)."""
    return int(lib().or_nif2_root(N))


def nif2_prove(a, h):
    a = np.ascontiguousarray(a, np.uint64)
    msgs = np.zeros(2 * h, np.uint64)
    if lib().or_nif2_prove(a, len(a), h, msgs) != 0:
        raise ValueError("h must be odd and divide (p - 1) / 2")
    return msgs


def nif2_verify(a, h, seed, msgs):
    """(accepted, F2 read from the proof)."""
    a = np.ascontiguousarray(a, np.uint64)
    m = np.ascontiguousarray(msgs, np.uint64)
    acc, f2 = C.c_int(), C.c_uint64()
    if lib().or_nif2_verify(a, len(a), h, seed, m, len(m), C.byref(acc), C.byref(f2)) != 0:
        raise ValueError("h must be odd and divide (p - 1) / 2")
    return bool(acc.value), int(f2.value)
