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


PAIRS = [("Mesh", "eft_mesh"), ("Phase", "eft_phase"), ("Materials", "eft_materials"), ("Params", "eft_params"),
         ("State", "eft_state"), ("Iterate", "eft_iterate"), ("SolveInfo", "eft_solve_info"),
         ("TransportInfo", "eft_transport_info"), ("StepInfo", "eft_step_info"), ("TuneInfo", "eft_tune_info"),
         ("KernelTime", "eft_kernel_time")]


def test_struct_layouts_match_header(tmp_path):
    """Every ctypes struct of the binding has the size and field offsets that
    a C compiler gives the header's struct of the same role."""
    import shutil
    import subprocess
    from paper_2402_10348_amd import eft
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "eft.h"', 'int main(void) {']
    for py, c in PAIRS:
        lines.append(f'printf("{py} size %zu\\n", sizeof({c}));')
        for f in getattr(eft, py)._fields_:
            lines.append(f'printf("{py} {f[0]} %zu\\n", offsetof({c}, {f[0]}));')
    lines += ["return 0; }"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for py, _ in PAIRS:
        cls = getattr(eft, py)
        assert got[(py, "size")] == ctypes.sizeof(cls), py
        for f in cls._fields_:
            assert got[(py, f[0])] == getattr(cls, f[0]).offset, (py, f[0])


def test_null_arguments_are_rejected(lib):
    lib.eft_create.restype = ctypes.c_int
    out = ctypes.c_void_p()
    assert lib.eft_create(None, None, None, None, ctypes.byref(out)) == 1   # EFT_EINVAL
    lib.eft_destroy.restype = ctypes.c_int
    assert lib.eft_destroy(None) == 1
    lib.eft_time_kernel.restype = ctypes.c_int
    assert lib.eft_time_kernel(None, 1) == 1
    lib.eft_kernel_time_read.restype = ctypes.c_int
    assert lib.eft_kernel_time_read(None, 1, None) == 1
    lib.eft_center_of_mass.restype = ctypes.c_int
    assert lib.eft_center_of_mass(None, None, None, None) == 1
    lib.eft_track_particles.restype = ctypes.c_int
    lib.eft_track_particles.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.eft_track_particles(None, None, 1, 0.1, 1e-10, None, None) == 1
