"""Host-side checks of the C ABI: the library loads without a GPU and exports every
function include/hsma.h declares; the binding refuses to run without its library."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hsma.h")
LIB = os.path.join(ROOT, "paper_1907_01724_amd", "libhsma.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(hsma_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_core_entry_points():
    names = declared_functions()
    for n in ("hsma_plan", "hsma_plan_ex", "hsma_plan_destroy", "hsma_potential", "hsma_energy",
              "hsma_workspace_bytes", "hsma_stream_check", "hsma_status_string"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhsma.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhsma.so not built")
def test_status_strings_and_defaults():
    import paper_1907_01724_amd as hs
    L = hs.load_library()
    assert L.hsma_status_string(0).decode() == "ok"
    assert "cavity" in L.hsma_status_string(2).decode()
    o = L.hsma_plan_opts_default()
    assert o.p < 0 and abs(o.tau - 0.1) < 1e-15 and o.pair_prec == hs.HSMA_PAIR_FP32_COMP


def test_binding_fails_loudly_without_library(tmp_path):
    import paper_1907_01724_amd as hs
    with pytest.raises(RuntimeError):
        hs.load_library.__wrapped__ if False else None
        saved = hs._lib
        try:
            hs._lib = None
            hs.load_library(str(tmp_path / "missing.so"))
        finally:
            hs._lib = saved
