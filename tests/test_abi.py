"""The C-ABI library loads on any host and exports every call declared in
include/eft.h; the binding mirrors the header's structs.  No GPU needed."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eft.h")
LIB = os.path.join(ROOT, "paper_2402_10348_amd", "_libeft.so")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:eft_status|const char \*)\s*(eft_\w+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2402_10348_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_hot_path():
    names = declared()
    for n in ("eft_create", "eft_destroy", "eft_assemble", "eft_spmv", "eft_fgmres", "eft_transport_solids",
              "eft_step", "eft_bands_build", "eft_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_export():
    from paper_2402_10348_amd import eft
    assert sorted(eft.EXPORTS) == declared()


def test_struct_layouts_match_header():
    """Sizes of the ABI structs computed by ctypes follow the C layout rules
    the header implies (x86-64 LP64)."""
    from paper_2402_10348_amd import eft
    assert ctypes.sizeof(eft.Phase) == 32
    assert ctypes.sizeof(eft.Materials) == 40
    assert ctypes.sizeof(eft.Params) == 8 * 7 + 4 * 2 + 8 + 4 * 4 + 8 + 4 * 2 + 4 + 4 + 8
    assert ctypes.sizeof(eft.State) == 8 * 8
    assert ctypes.sizeof(eft.StepInfo) == 16 + 8 * 129 + 24
    assert ctypes.sizeof(eft.TransportInfo) == 8 + 8 * 64 * 4 + 4 * 128 + 8 * 128


def test_null_arguments_are_rejected(lib):
    lib.eft_create.restype = ctypes.c_int
    out = ctypes.c_void_p()
    assert lib.eft_create(None, None, None, None, ctypes.byref(out)) == 1   # EFT_EINVAL
    lib.eft_destroy.restype = ctypes.c_int
    assert lib.eft_destroy(None) == 1
