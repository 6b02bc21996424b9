"""The C ABI library loads and exports every symbol include/qdwf.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qdwf.h")
LIB = os.path.join(ROOT, "paper_2112_01852_amd", "libqdwf.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qdwf_[a-zA-Z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libqdwf.so not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_expected_calls():
    names = declared()
    for must in ["qdwf_create", "qdwf_destroy", "qdwf_set_gauge", "qdwf_apply_D",
                 "qdwf_apply_Mee", "qdwf_apply_Deo", "qdwf_apply_Mpc", "qdwf_apply_MdagM",
                 "qdwf_solve", "qdwf_pack_spinor", "qdwf_unpack_spinor", "qdwf_dot",
                 "qdwf_geometry_tables", "qdwf_workspace_bytes", "qdwf_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    from paper_2112_01852_amd import qdwf
    assert set(declared()) <= set(qdwf.declared_symbols())


def test_null_arguments_are_rejected_without_a_device(lib):
    lib.qdwf_create.restype = ctypes.c_int
    lib.qdwf_last_error.restype = ctypes.c_char_p
    assert lib.qdwf_create(None, 0, None) == 1          # QDWF_EINVAL
    assert lib.qdwf_last_error().decode() != ""
    lib.qdwf_apply_D.restype = ctypes.c_int
    assert lib.qdwf_apply_D(None, None, None, 0, 1, 1, 1, None) == 1
