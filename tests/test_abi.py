"""C-ABI library checks that need no GPU: it loads, exports every symbol the
header declares, and refuses to run without a device (no CPU fallback)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sp_engine.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sp_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_1901_11350_amd as pk

    if not os.path.exists(pk.LIB_PATH):
        pytest.fail("libsp_engine.so is not built (run __graft_entry__.build())")
    return pk.lib()


def test_library_exports_every_declared_symbol(lib):
    import paper_1901_11350_amd as pk

    declared = header_functions()
    assert len(declared) >= 20
    assert sorted(pk.EXPORTS) == declared
    raw = ctypes.CDLL(os.path.join(ROOT, "paper_1901_11350_amd", "libsp_engine.so"))
    for name in declared:
        assert hasattr(raw, name), name


def test_version_string(lib):
    assert lib.sp_version().decode().startswith("sp_engine")


def test_null_engine_arguments_are_rejected(lib):
    import paper_1901_11350_amd as pk

    assert lib.sp_create(None, 0, 0, None) == pk.SP_E_ARG
    h = ctypes.c_void_p()
    assert lib.sp_create(ctypes.byref(h), 0, 7, None) == pk.SP_E_ARG
    assert lib.sp_num_sites(None) == 0
    lib.sp_destroy(None)


def test_engine_creation_fails_loudly_without_gpu(lib):
    from conftest import gpu_available
    import paper_1901_11350_amd as pk

    if gpu_available():
        pytest.skip("a GPU is present")
    with pytest.raises(pk.SpError):
        pk.Engine(0, "f32")
