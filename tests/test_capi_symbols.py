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


def test_struct_sizes_match_c_layout(tmp_path):
    """The ctypes structures have the sizes and field offsets the C compiler
    gives the structs of include/symx.h."""
    import ctypes as C
    import subprocess
    from paper_2303_02156_amd import symx
    pairs = {"symx_energy_desc": symx.EnergyDesc, "symx_mesh_desc": symx.MeshDesc,
             "symx_bsr_view": symx.BsrView, "symx_step_params": symx.StepParams,
             "symx_step_report": symx.StepReport, "symx_server_stats": symx.ServerStats,
             "symx_mesh_info": symx.MeshInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "symx.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("  return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = dict(line.rsplit(" ", 1) for line in
               subprocess.run([str(exe)], capture_output=True, text=True,
                              check=True).stdout.split("\n") if line)
    for cname, py in pairs.items():
        assert C.sizeof(py) == int(out[cname]), cname
        for f, _ in py._fields_:
            assert getattr(py, f).offset == int(out[f"{cname}.{f}"]), (cname, f)


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
