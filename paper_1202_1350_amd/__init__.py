"""MI355X GKR prover / verifier over F_p, p = 2^61 - 1.

Thin ctypes binding of libgkr.so (include/gkr.h): argument marshalling only,
every step of the proof runs in the library's HIP kernels.  Device buffers
are torch tensors on a ROCm device; host buffers are numpy arrays.  The
binding raises if the library is missing -- there is no CPU fallback.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgkr.so")
P = (1 << 61) - 1

GKR_OK, GKR_ERR_INVALID, GKR_ERR_RANGE, GKR_ERR_NOMEM, GKR_ERR_DEVICE, GKR_ERR_BUFSIZE = \
    0, -1, -2, -3, -4, -5
GKR_OMEGA_GATES, GKR_OMEGA_TABLES, GKR_OMEGA_TABLES_STEPWISE = 0, 1, 2
GKR_BATCH_GRAPH = 1
GKR_MEM_RESIDENT, GKR_MEM_LAYER, GKR_MEM_MESSAGE, GKR_MEM_AUTO = 0, 1, 2, 3
CHECKS = {1: "malformed", 2: "round", 3: "wiring", 4: "line", 5: "input"}


class GkrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gkr error {code}: {msg}")
        self.code = code


class RejectInfo(C.Structure):
    _fields_ = [("layer", C.c_int32), ("round", C.c_int32), ("check", C.c_int32)]


_lib = None

# (name, restype, argtypes) for every entry point of include/gkr.h
_SIGS = [
    ("gkr_circuit_create", C.c_int, [C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.POINTER(C.c_void_p)]),
    ("gkr_circuit_destroy", None, [C.c_void_p]),
    ("gkr_circuit_set_algorithm", C.c_int, [C.c_void_p, C.c_int]),
    ("gkr_memory_need", C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    ("gkr_circuit_set_memory", C.c_int, [C.c_void_p, C.c_int, C.c_uint64, C.POINTER(C.c_int)]),
    ("gkr_transcript_size", C.c_int, [C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    ("gkr_circuit_info", C.c_int, [C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                   C.POINTER(C.c_uint32)]),
    ("gkr_prove", C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_uint64, C.c_void_p, C.c_void_p,
                            C.c_void_p]),
    ("gkr_verify", C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_uint64, C.c_void_p, C.c_uint64,
                             C.POINTER(C.c_int), C.POINTER(RejectInfo), C.c_void_p]),
    ("gkr_circuit_wiring", C.c_int, [C.c_void_p, C.c_uint32, C.POINTER(C.c_int)]),
    ("gkr_verify_closed_forms", C.c_int, [C.c_int]),
    ("f2_sumcheck_prove", C.c_int, [C.c_void_p, C.c_uint64, C.c_int, C.c_uint64, C.c_void_p,
                                    C.c_void_p, C.c_void_p]),
    ("f2_sumcheck_prove_noalloc", C.c_int, [C.c_void_p, C.c_uint64, C.c_int, C.c_uint64, C.c_void_p,
                                            C.c_void_p, C.c_void_p]),
    ("f2_sumcheck_verify", C.c_int, [C.c_void_p, C.c_uint64, C.c_int, C.c_uint64, C.c_void_p,
                                     C.c_uint64, C.POINTER(C.c_int), C.POINTER(RejectInfo),
                                     C.c_void_p]),
    ("nif2_prove", C.c_int, [C.c_void_p, C.c_uint64, C.c_uint32, C.c_int, C.c_void_p, C.c_void_p]),
    ("nif2_verify", C.c_int, [C.c_void_p, C.c_uint64, C.c_uint32, C.c_int, C.c_uint64, C.c_void_p,
                              C.c_uint64, C.POINTER(C.c_int), C.POINTER(C.c_uint64), C.c_void_p]),
    ("gkr_batch_prove", C.c_int, [C.c_uint32, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p,
                                  C.c_void_p, C.c_int, C.c_void_p]),
    ("gkr_server_create", C.c_int, [C.c_uint64, C.c_uint32, C.POINTER(C.c_void_p)]),
    ("gkr_server_submit", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64,
                                    C.POINTER(C.c_uint64)]),
    ("gkr_server_poll", C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p, C.POINTER(C.c_int),
                                  C.POINTER(C.c_double)]),
    ("gkr_server_stats", C.c_int, [C.c_void_p, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                   C.POINTER(C.c_uint64)]),
    ("gkr_server_destroy", None, [C.c_void_p]),
    ("gkr_autotune", C.c_int, [C.c_uint32, C.c_void_p, C.c_void_p, C.c_int, C.c_uint32, C.c_void_p]),
    ("gkr_tune_get", C.c_int, [C.c_void_p, C.POINTER(C.c_uint32)]),
    ("gkr_tune_set", C.c_int, [C.c_void_p, C.c_uint32]),
    ("gkr_field_op", C.c_int, [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64,
                               C.c_void_p]),
    ("gkr_profile_enable", C.c_int, [C.c_int]),
    ("gkr_profile_read", C.c_int, [C.POINTER(C.c_uint32), C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p]),
    ("gkr_profile_launches", C.c_int, [C.POINTER(C.c_uint64), C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p]),
    ("gkr_last_error", C.c_char_p, []),
]
EXPORTS = [s[0] for s in _SIGS]


def lib():
    """Load libgkr.so (built by paper_1202_1350_amd/build.py); raise if absent."""
    global _lib
    if _lib is None:
        # torch's bundled HIP runtime carries the same soname as ROCm's
        # (libamdhip64.so.7): loading torch first makes libgkr.so bind to that
        # one copy, so torch tensors and this library share one runtime.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python paper_1202_1350_amd/build.py` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != GKR_OK:
        raise GkrError(rc, lib().gkr_last_error().decode())


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _ptr(x, dtype):
    """(pointer, on_device, keepalive) for a numpy array or torch tensor."""
    if _is_torch(x):
        import torch
        want = {np.uint64: torch.uint64, np.uint32: torch.uint32}[dtype]
        if x.dtype != want or not x.is_contiguous():
            raise TypeError(f"expected a contiguous {want} tensor")
        return x.data_ptr(), int(x.is_cuda), x
    a = np.ascontiguousarray(x, dtype)
    return a.ctypes.data, 0, a


def _stream(dev, stream):
    if stream is not None:
        return C.c_void_p(stream)
    if dev:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return None


class Circuit:
    """Device-resident layered circuit (gkr_circuit_create)."""

    def __init__(self, sizes, types, in1, in2):
        sizes = np.ascontiguousarray(sizes, np.uint32)
        d = len(sizes) - 1
        self._keep = [np.ascontiguousarray(t, np.uint8) for t in types] + \
                     [np.ascontiguousarray(a, np.uint32) for a in in1] + \
                     [np.ascontiguousarray(b, np.uint32) for b in in2]
        tp = (C.c_void_p * max(d, 1))(*[a.ctypes.data for a in self._keep[:d]])
        ap = (C.c_void_p * max(d, 1))(*[a.ctypes.data for a in self._keep[d:2 * d]])
        bp = (C.c_void_p * max(d, 1))(*[a.ctypes.data for a in self._keep[2 * d:]])
        h = C.c_void_p()
        _check(lib().gkr_circuit_create(len(sizes), sizes.ctypes.data, C.cast(tp, C.c_void_p),
                                        C.cast(ap, C.c_void_p), C.cast(bp, C.c_void_p),
                                        C.byref(h)))
        self._keep = None
        self.handle = h
        self.sizes = sizes
        m, c = C.c_uint64(), C.c_uint64()
        _check(lib().gkr_transcript_size(h, C.byref(m), C.byref(c)))
        self.n_msgs, self.n_chals = m.value, c.value
        g, r, nl = C.c_uint64(), C.c_uint64(), C.c_uint32()
        _check(lib().gkr_circuit_info(h, C.byref(g), C.byref(r), C.byref(nl)))
        self.gates, self.rounds = g.value, r.value

    @classmethod
    def from_workload(cls, circ, omega_algo=None):
        c = cls(circ.sizes, circ.types, circ.in1, circ.in2)
        if omega_algo is not None:
            c.set_algorithm(omega_algo)
        return c

    def set_algorithm(self, omega_algo: int):
        """GKR_OMEGA_TABLES (default), GKR_OMEGA_TABLES_STEPWISE or GKR_OMEGA_GATES;
        same transcript."""
        _check(lib().gkr_circuit_set_algorithm(self.handle, int(omega_algo)))

    def memory_need(self, mode: int):
        """(device bytes, pinned host bytes) of one proof in a GKR_MEM_* mode."""
        d, h = C.c_uint64(), C.c_uint64()
        _check(lib().gkr_memory_need(self.handle, int(mode), C.byref(d), C.byref(h)))
        return d.value, h.value

    def set_memory(self, mode: int, device_budget_bytes: int = 0) -> int:
        """Place the proofs' data (GKR_MEM_RESIDENT, _LAYER, _MESSAGE or
        _AUTO within the budget); returns the mode chosen."""
        chosen = C.c_int(-1)
        _check(lib().gkr_circuit_set_memory(self.handle, int(mode), int(device_budget_bytes),
                                            C.byref(chosen)))
        return chosen.value

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.gkr_circuit_destroy(h)
            self.handle = None


def gkr_circuit_create(sizes, types, in1, in2) -> Circuit:
    return Circuit(sizes, types, in1, in2)


def gkr_prove(circ: Circuit, inputs, seed: int, want_chals: bool = True, stream=None):
    """(msgs, chals) as uint64 numpy arrays."""
    p, dev, keep = _ptr(inputs, np.uint64)
    msgs = np.zeros(max(circ.n_msgs, 1), np.uint64)
    chals = np.zeros(max(circ.n_chals, 1), np.uint64) if want_chals else None
    _check(lib().gkr_prove(circ.handle, p, dev, seed, msgs.ctypes.data,
                           chals.ctypes.data if want_chals else None, _stream(dev, stream)))
    return msgs[:circ.n_msgs], (chals[:circ.n_chals] if want_chals else None)


def gkr_verify(circ: Circuit, inputs, seed: int, msgs, stream=None):
    """(accepted, layer, round, check)."""
    p, dev, keep = _ptr(inputs, np.uint64)
    m = np.ascontiguousarray(msgs, np.uint64)
    acc = C.c_int()
    why = RejectInfo()
    _check(lib().gkr_verify(circ.handle, p, dev, seed, m.ctypes.data if len(m) else None, len(m),
                            C.byref(acc), C.byref(why), _stream(dev, stream)))
    return bool(acc.value), why.layer, why.round, why.check


GKR_WIRING_GATES, GKR_WIRING_TREE, GKR_WIRING_SQUARE, GKR_WIRING_MATMULT = 0, 1, 2, 3


def gkr_circuit_wiring(circ: Circuit, layer: int) -> int:
    """Wiring shape of a layer (GKR_WIRING_*)."""
    f = C.c_int()
    _check(lib().gkr_circuit_wiring(circ.handle, layer, C.byref(f)))
    return f.value


def gkr_verify_closed_forms(enable: bool) -> bool:
    """Closed-form wiring in gkr_verify on or off; returns the previous setting."""
    return bool(lib().gkr_verify_closed_forms(1 if enable else 0))


def gkr_batch_prove(circs, inputs, seeds, graph: bool = True, stream=None):
    """Prove len(circs) proofs together; inputs are device tensors (uint64).
    Returns the list of transcripts."""
    n = len(circs)
    if n == 0:
        return []
    keep = [_ptr(x, np.uint64) for x in inputs]
    if not all(dev for _, dev, _ in keep):
        raise TypeError("batched inputs must be device tensors")
    hs = (C.c_void_p * n)(*[c.handle.value for c in circs])
    ins = (C.c_void_p * n)(*[p for p, _, _ in keep])
    sd = np.ascontiguousarray(seeds, np.uint64)
    outs = [np.zeros(max(c.n_msgs, 1), np.uint64) for c in circs]
    ms = (C.c_void_p * n)(*[o.ctypes.data for o in outs])
    _check(lib().gkr_batch_prove(n, C.cast(hs, C.c_void_p), C.cast(ins, C.c_void_p), 1,
                                 sd.ctypes.data, C.cast(ms, C.c_void_p),
                                 GKR_BATCH_GRAPH if graph else 0, _stream(1, stream)))
    return [o[:c.n_msgs] for o, c in zip(outs, circs)]


def gkr_autotune(circs, inputs, reps: int = 2, stream=None):
    """Pick launch shapes by timing proofs of circs (inputs: all host arrays
    or all device tensors)."""
    n = len(circs)
    keep = [_ptr(x, np.uint64) for x in inputs]
    ondev = {bool(dev) for _, dev, _ in keep}
    if len(ondev) != 1:
        raise TypeError("inputs must be all host arrays or all device tensors")
    hs = (C.c_void_p * n)(*[c.handle.value for c in circs])
    ins = (C.c_void_p * n)(*[p for p, _, _ in keep])
    dev = ondev.pop()
    _check(lib().gkr_autotune(n, C.cast(hs, C.c_void_p), C.cast(ins, C.c_void_p), int(dev),
                              int(reps), _stream(1 if dev else 0, stream)))


def gkr_tune_get() -> bytes:
    """The launch-shape table (to restore with gkr_tune_set)."""
    n = C.c_uint32(0)
    _check(lib().gkr_tune_get(None, C.byref(n)))
    buf = (C.c_uint8 * n.value)()
    _check(lib().gkr_tune_get(buf, C.byref(n)))
    return bytes(buf)


def gkr_tune_set(table):
    """Restore a table from gkr_tune_get; None restores the defaults."""
    if table is None:
        _check(lib().gkr_tune_set(None, 0))
    else:
        b = (C.c_uint8 * len(table)).from_buffer_copy(table)
        _check(lib().gkr_tune_set(b, len(table)))


class Server:
    """Continuous-batching proof server (gkr_server_*)."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int):
        h = C.c_void_p()
        _check(lib().gkr_server_create(int(hbm_budget_bytes), int(max_slots), C.byref(h)))
        self.handle = h
        self._circ = {}

    def submit(self, circ: Circuit, inputs, seed: int) -> int:
        x = np.ascontiguousarray(inputs, np.uint64)
        rid = C.c_uint64()
        _check(lib().gkr_server_submit(self.handle, circ.handle, x.ctypes.data, int(seed),
                                       C.byref(rid)))
        self._circ[rid.value] = circ
        return rid.value

    def poll(self, rid: int):
        """(done, msgs or None, latency_s); raises on a failed request."""
        circ = self._circ[rid]
        out = np.zeros(max(circ.n_msgs, 1), np.uint64)
        done, lat = C.c_int(), C.c_double()
        try:
            _check(lib().gkr_server_poll(self.handle, rid, out.ctypes.data, C.byref(done),
                                         C.byref(lat)))
        except GkrError:
            self._circ.pop(rid, None)
            raise
        if not done.value:
            return False, None, None
        self._circ.pop(rid, None)
        return True, out[:circ.n_msgs], lat.value

    def stats(self):
        r, q, u = C.c_uint32(), C.c_uint32(), C.c_uint64()
        _check(lib().gkr_server_stats(self.handle, C.byref(r), C.byref(q), C.byref(u)))
        return r.value, q.value, u.value

    def close(self):
        if self.handle:
            lib().gkr_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            self.close()


def f2_sumcheck_prove(freq, seed: int, stream=None):
    p, dev, keep = _ptr(freq, np.uint32)
    n = freq.numel() if _is_torch(freq) else len(keep)
    l = int(n).bit_length() - 1
    msgs = np.zeros(1 + 3 * l, np.uint64)
    chals = np.zeros(max(l, 1), np.uint64)
    _check(lib().f2_sumcheck_prove(p, n, dev, seed, msgs.ctypes.data, chals.ctypes.data,
                                   _stream(dev, stream)))
    return msgs, chals[:l]


def f2_sumcheck_prove_noalloc(freq, seed: int, stream=None):
    """f2_sumcheck_prove with its scratch in the library's static device
    array (no allocation inside the call; n <= 2^22)."""
    p, dev, keep = _ptr(freq, np.uint32)
    n = freq.numel() if _is_torch(freq) else len(keep)
    l = int(n).bit_length() - 1
    msgs = np.zeros(1 + 3 * l, np.uint64)
    chals = np.zeros(max(l, 1), np.uint64)
    _check(lib().f2_sumcheck_prove_noalloc(p, n, dev, seed, msgs.ctypes.data, chals.ctypes.data,
                                           _stream(dev, stream)))
    return msgs, chals[:l]


def f2_sumcheck_verify(freq, seed: int, msgs, stream=None):
    p, dev, keep = _ptr(freq, np.uint32)
    n = freq.numel() if _is_torch(freq) else len(keep)
    m = np.ascontiguousarray(msgs, np.uint64)
    acc = C.c_int()
    why = RejectInfo()
    _check(lib().f2_sumcheck_verify(p, n, dev, seed, m.ctypes.data if len(m) else None, len(m),
                                    C.byref(acc), C.byref(why), _stream(dev, stream)))
    return bool(acc.value), why.round, why.check


def nif2_prove(a, h: int, stream=None):
    """Proof (2h words) of the non-interactive F2 protocol for the values a
    (uint64 array or device tensor, each below p) on a v x h grid."""
    p, dev, keep = _ptr(a, np.uint64)
    n = a.numel() if _is_torch(a) else len(keep)
    msgs = np.zeros(2 * h, np.uint64)
    _check(lib().nif2_prove(p, n, h, dev, msgs.ctypes.data, _stream(dev, stream)))
    return msgs


def nif2_verify(a, h: int, seed: int, msgs, stream=None):
    """(accepted, F2 read from the proof)."""
    p, dev, keep = _ptr(a, np.uint64)
    n = a.numel() if _is_torch(a) else len(keep)
    m = np.ascontiguousarray(msgs, np.uint64)
    acc, f2 = C.c_int(), C.c_uint64()
    _check(lib().nif2_verify(p, n, h, dev, seed, m.ctypes.data if len(m) else None, len(m),
                             C.byref(acc), C.byref(f2), _stream(dev, stream)))
    return bool(acc.value), int(f2.value)


def gkr_field_op(op: int, a, b, out, stream=None):
    """Field op on device tensors (0 add, 1 sub, 2 mul, 3 lazy sum of 64
    products, 4 a * b^256 by successive products)."""
    pa, _, _ = _ptr(a, np.uint64)
    pb, _, _ = _ptr(b, np.uint64)
    po, dev, _ = _ptr(out, np.uint64)
    _check(lib().gkr_field_op(op, pa, pb, po, out.numel(), _stream(dev, stream)))


def gkr_profile_enable(flag):
    """0 off, 1 per-class totals, 2 totals and per-launch records."""
    _check(lib().gkr_profile_enable(int(flag)))


def gkr_profile_read():
    """{kernel class: (ms, launches, algorithmic bytes, algorithmic modular
    products)}; resets the totals."""
    n = C.c_uint32(32)
    names = (C.c_char_p * 32)()
    ms = (C.c_double * 32)()
    cnt = (C.c_uint64 * 32)()
    by = (C.c_double * 32)()
    mo = (C.c_double * 32)()
    _check(lib().gkr_profile_read(C.byref(n), C.cast(names, C.c_void_p), C.cast(ms, C.c_void_p),
                                  C.cast(cnt, C.c_void_p), C.cast(by, C.c_void_p),
                                  C.cast(mo, C.c_void_p)))
    return {names[k].decode(): (ms[k], cnt[k], by[k], mo[k]) for k in range(n.value)}


def gkr_profile_launches():
    """Per-launch records kept under gkr_profile_enable(2): a list of
    (class name, size class, ms, bytes, products); drops them."""
    n = C.c_uint64(0)
    _check(lib().gkr_profile_launches(C.byref(n), None, None, None, None, None))
    k = n.value
    cls = (C.c_int32 * max(k, 1))()
    sc = (C.c_int32 * max(k, 1))()
    ms = (C.c_float * max(k, 1))()
    by = (C.c_double * max(k, 1))()
    mo = (C.c_double * max(k, 1))()
    _check(lib().gkr_profile_launches(C.byref(n), C.cast(cls, C.c_void_p), C.cast(sc, C.c_void_p),
                                      C.cast(ms, C.c_void_p), C.cast(by, C.c_void_p),
                                      C.cast(mo, C.c_void_p)))
    names = list(gkr_profile_class_names())
    return [(names[cls[i]], sc[i], ms[i], by[i], mo[i]) for i in range(min(k, n.value))]


def gkr_profile_class_names():
    n = C.c_uint32(64)
    names = (C.c_char_p * 64)()
    _check(lib().gkr_profile_read(C.byref(n), C.cast(names, C.c_void_p), None, None, None, None))
    return [names[k].decode() for k in range(n.value)]
