"""CPU checks of the boundary: the HIP library loads and exports every entry
point the C header declares, and the binding declares exactly those."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mortar_mi355x.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mt_\w+)\s*\(", txt)))


def test_header_declares_entry_points():
    names = declared()
    for n in ("mt_create", "mt_upload", "mt_build_pairs", "mt_csr_pattern", "mt_integrate", "mt_backward",
              "mt_batch_forward", "mt_batch_backward", "mt_batch_autotune"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2202_03933_amd import _capi
    if not os.path.exists(_capi.LIB_PATH):
        pytest.fail("HIP library not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_capi.LIB_PATH)  # loading runs no GPU code
    for n in declared():
        assert hasattr(lib, n), n
    assert sorted(_capi.SIGNATURES) == declared()


def test_binding_refuses_missing_library(tmp_path, monkeypatch):
    from paper_2202_03933_amd import _capi
    monkeypatch.setattr(_capi, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_capi, "_lib", None)
    with pytest.raises(RuntimeError):
        _capi.lib()
