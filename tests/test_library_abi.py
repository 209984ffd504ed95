"""CPU-side checks of the C ABI: the library loads and exports every symbol
the header declares; the Python binding covers each of them.  No compute
calls are made here (there is no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "femasm.h")
LIB = os.path.join(ROOT, "paper_1401_3301_amd", "libfemasm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fem_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1401_3301_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("fem_assemble_symbolic", "fem_assemble_numeric", "fem_assemble_backward",
                 "fem_batch_create", "fem_batch_numeric", "fem_plan_slot_map"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_1401_3301_amd import femasm
    assert sorted(femasm.EXPORTED) == declared_functions()
    for n in declared_functions():
        assert callable(getattr(femasm, n))


def test_status_strings(lib):
    lib.fem_status_str.restype = ctypes.c_char_p
    lib.fem_status_str.argtypes = [ctypes.c_int]
    assert lib.fem_status_str(0) == b"FEM_OK"
    assert lib.fem_status_str(3) == b"FEM_ERR_DEGENERATE"
    assert lib.fem_status_str(99) == b"FEM_ERR_UNKNOWN"


def test_binding_refuses_without_gpu():
    import torch
    from paper_1401_3301_amd import femasm
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    femasm._lib = None
    with pytest.raises(femasm.FemasmUnavailable):
        femasm.load_library()
