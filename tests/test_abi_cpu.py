"""CPU checks of the C ABI: the library is built for gfx950 and exports every
function that include/citron.h declares (no compute call without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "citron.h")
LIB = os.path.join(ROOT, "paper_2112_10913_amd", "libcitron.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(citron_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["citron_load_csr", "citron_order", "citron_count", "citron_count_batch",
                     "citron_get_dag", "citron_free", "citron_last_error",
                     "citron_server_create", "citron_server_submit", "citron_server_poll"]:
        assert required in names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libcitron.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_library_holds_gfx950_code():
    # the clang offload bundles embedded by hipcc name their device targets as
    # text ("hipv4-amdgcn-amd-amdhsa--<arch>"): every one must be gfx950
    with open(LIB, "rb") as f:
        blob = f.read()
    targets = set(re.findall(rb"hipv4-amdgcn-amd-amdhsa--(gfx[0-9a-z]+)", blob))
    assert targets == {b"gfx950"}, targets


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_2112_10913_amd._lib as L
    monkeypatch.setattr(L, "_LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(ImportError):
        L.load_library()


def test_null_arguments_are_rejected_without_a_gpu(lib):
    lib.citron_count.restype = ctypes.c_uint64
    st = ctypes.c_int32(-1)
    assert lib.citron_count(None, 3, ctypes.byref(st)) == 0
    assert st.value == 1
    lib.citron_free(None)
    lib.citron_last_error.restype = ctypes.c_char_p
    assert b"NULL" in lib.citron_last_error()


def test_vertex_count_limit_is_checked_before_any_device_call(lib):
    import numpy as np
    rp = np.zeros(2, np.int32)
    out = ctypes.c_void_p()
    lib.citron_load_csr.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_uint32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    lib.citron_last_error.restype = ctypes.c_char_p
    for n in (1 << 26, -1):
        assert lib.citron_load_csr(n, 0, rp.ctypes.data, None, 0, None, ctypes.byref(out)) == 1
        assert out.value is None
        assert b"2^26" in lib.citron_last_error()
