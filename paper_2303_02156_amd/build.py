"""Build steps for the native parts of the package.

1. symx_gen (C++ host tool, g++) -> generated element functions under
   csrc/generated/ (HIP templates, a test-only C variant and an op census).
2. libsymx.so: the HIP kernels and the C-ABI, compiled for gfx950 with hipcc.
3. libsymx_gen_cpu.so: the generated C variant compiled with gcc, used only by
   CPU tests that check the generator against the FP64 oracle.

Everything is built in-tree so the shared objects travel with the source tree.
"""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
GEN_OUT = os.path.join(CSRC, "generated")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libsymx.so")
GEN_EXE = os.path.join(BUILD, "symx_gen")
CPU_TESTLIB = os.path.join(BUILD, "libsymx_gen_cpu.so")

HIP_SOURCES = ["symx_mesh.cpp", "symx_kernels.hip", "symx_newton.cpp", "symx_capi.cpp",
               "symx_profile.cpp", "symx_server.cpp", "symx_memory.cpp", "symx_contact.cpp",
               "symx_contact_pattern.hip", "symx_noalloc.hip", "symx_batch.cpp"]
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-Wno-unknown-warning-option",
]


def _run(cmd, cwd=None):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r.stdout


def build_generator():
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(GEN_OUT, exist_ok=True)
    src = [os.path.join(CSRC, "gen", f) for f in ("expr.cpp", "symx_gen.cpp")]
    _run(["g++", "-O2", "-std=c++17", "-Wall", "-Wextra", *src, "-o", GEN_EXE])
    _run([GEN_EXE, GEN_OUT])


def build_cpu_testlib():
    _run(["gcc", "-O2", "-fPIC", "-shared", os.path.join(GEN_OUT, "symx_generated_cpu.c"),
          "-o", CPU_TESTLIB, "-lm"])


def build_hip_library(jobs: int = 4):
    """Compile each source to an object in parallel, then link libsymx.so."""
    os.makedirs(BUILD, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", GEN_OUT]
    procs = []
    objs = []
    for s in HIP_SOURCES:
        obj = os.path.join(BUILD, s + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if s.endswith(".hip") else []
        cmd = [hipcc, *[f for f in HIP_FLAGS if f != "-shared"], "-c", *inc, *lang,
               os.path.join(CSRC, s), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                            text=True)))
    errors = []
    for cmd, p in procs:
        out, err = p.communicate()
        if p.returncode != 0:
            errors.append(f"{' '.join(cmd)}\n{out}\n{err}")
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errors))
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)


def build_all():
    build_generator()
    build_cpu_testlib()
    build_hip_library()
