"""The C-ABI library loads and exports every function include/gkr.h declares
(no compute calls: this runs without a GPU)."""
import os
import re

import pytest

import paper_1202_1350_amd as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in os.listdir(inc):
        if not f.endswith(".h"):
            continue
        text = open(os.path.join(inc, f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[\w\s\*]+?\b(\w+)\s*\(", text, flags=re.M):
            if m.group(1) not in ("if", "while", "for", "sizeof", "return"):
                names.add(m.group(1))
    return names


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert {"gkr_circuit_create", "gkr_prove", "gkr_verify", "f2_sumcheck_prove"} <= names
    L = G.lib()
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_header():
    assert declared_functions() == set(G.EXPORTS)


def test_no_oracle_in_product_path():
    """The GPU package and its sources never reference the oracle."""
    pkg = os.path.join(ROOT, "paper_1202_1350_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower(), os.path.join(dirpath, f)


def test_tune_table_round_trip_and_rejects():
    """The shape table is host state: get/set round-trip, reset, and
    malformed tables rejected, without touching a GPU."""
    import paper_1202_1350_amd as G
    G.gkr_tune_set(None)
    t0 = G.gkr_tune_get()
    assert t0[0] == 1 and len(t0) == 4 + t0[1] * t0[2]
    assert set(t0[4:]) == {0xFF}
    t1 = bytearray(t0)
    t1[4] = 5
    G.gkr_tune_set(bytes(t1))
    assert G.gkr_tune_get() == bytes(t1)
    for bad in (bytes(t1[:-1]), bytes([2]) + bytes(t1[1:]), bytes(t1[:4]) + bytes([16]) + bytes(t1[5:])):
        with pytest.raises(G.GkrError):
            G.gkr_tune_set(bad)
    assert G.gkr_tune_get() == bytes(t1)
    G.gkr_tune_set(None)
    assert G.gkr_tune_get() == t0
