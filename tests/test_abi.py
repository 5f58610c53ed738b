"""The C-ABI library builds, loads without a GPU, and exports every function
that include/vmo.h declares (no compute call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "vmo.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vmo_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for want in ["vmo_create", "vmo_destroy", "vmo_layout", "vmo_bisect", "vmo_order_sbd", "vmo_order_bbd",
                 "vmo_cut", "vmo_order_batch", "vmo_dual", "vmo_model", "vmo_components", "vmo_order_border",
                 "vmo_order_schur", "vmo_match", "vmo_order_matched", "vmo_matched_perms", "vmo_finegrain",
                 "vmo_refine_kl"]:
        assert want in names


def test_library_exports_every_declared_symbol():
    import paper_1105_4490_amd as P
    if not os.path.exists(P.LIB_PATH):
        from paper_1105_4490_amd import build
        build.build()
    L = ctypes.CDLL(P.LIB_PATH)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_refuses_without_library(tmp_path, monkeypatch):
    import paper_1105_4490_amd as P
    monkeypatch.setattr(P, "LIB_PATH", str(tmp_path / "none.so"))
    monkeypatch.setattr(P, "_lib", None)
    with pytest.raises(ImportError):
        P.lib()


def test_batch_job_records_match_the_c_layout():
    """The numpy records order_batch fills are byte-identical to ctypes vmo_job structs."""
    import ctypes as C
    import numpy as np
    import paper_1105_4490_amd as P
    vals = []
    arr = np.zeros(3, dtype=P._job_dtype())
    cj = (P.Job * 3)()
    for i in range(3):
        h = P.Hypergraph(10 + i, 20 + i, 0x1000 + i, 0x2000 + i, 0, 0x3000 + i)
        o = P.OrderOut(0x4000 + i, 0, 0x5000 + i, 0x6000 + i, 0x7000 + i, 0, 0x8000 + i, 0x9000 + i)
        cj[i] = P.Job(h, i % 2, 1 - i % 2, 0xA000 + i, 7 + i, 99 + i, 5 + i, o)
        arr[i] = (10 + i, 20 + i, 0x1000 + i, 0x2000 + i, 0, 0x3000 + i, i % 2, 1 - i % 2, 0xA000 + i, 7 + i,
                  99 + i, 5 + i, 0x4000 + i, 0, 0x5000 + i, 0x6000 + i, 0x7000 + i, 0, 0x8000 + i, 0x9000 + i)
    assert arr.tobytes() == C.string_at(cj, C.sizeof(cj))
