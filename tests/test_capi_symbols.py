"""libsymx.so loads on the CPU host and exports every function of include/symx.h.

No compute call is made here (there is no GPU); the GPU tests exercise them.
"""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "symx.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(symx_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2303_02156_amd import symx
    if not os.path.exists(symx.LIBPATH):
        from paper_2303_02156_amd import build
        build.build_generator()
        build.build_hip_library()
    return symx.load()


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("symx_mesh_create", "symx_eval_derivatives", "symx_assemble_bsr",
                     "symx_newton_step"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2303_02156_amd import symx
    names = _declared()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(symx.EXPORTS), set(names) ^ set(symx.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", symx.LIBPATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r" T (symx_[a-z0-9_]+)", out))
    assert set(names) <= exported


def test_status_strings(lib):
    for s in range(9):
        assert lib.symx_status_string(s)
    assert lib.symx_status_string(99) == b"unknown status"


def test_struct_sizes_match_c_layout():
    import ctypes as C
    from paper_2303_02156_amd import symx
    # sizes implied by include/symx.h on x86-64 (natural alignment)
    assert C.sizeof(symx.EnergyDesc) == 4 + 4 + 8 * 8
    assert C.sizeof(symx.MeshDesc) == 8 + 8 + 8 + 8 + 8 + 8
    assert C.sizeof(symx.BsrView) == 8 * 5 + 8
    assert C.sizeof(symx.StepParams) == 8 * 5 + 4 * 7 + 4
    assert C.sizeof(symx.StepReport) == 4 * 6 + 8 * 8
    assert C.sizeof(symx.ServerStats) == 8 * 8 + 4 * 3 + 4


def test_null_arguments_rejected_without_gpu(lib):
    import ctypes as C
    from paper_2303_02156_amd import symx
    h = C.c_void_p()
    assert lib.symx_mesh_create(None, C.byref(h)) == 1
    assert lib.symx_mesh_get_info(None, None) == 1
    assert lib.symx_newton_step(None, None, None, None, None) == 1
    assert lib.symx_server_create(0, 4, C.byref(h)) == 1
    assert lib.symx_server_create(1 << 30, 0, C.byref(h)) == 1
    assert lib.symx_server_poll(None, 1, 0, None, None, None, None) == 1
    assert b"null" in lib.symx_last_error() or lib.symx_last_error()
    assert symx.STATUS[1] == "INVALID_ARG"
