"""Builds liblbm.so (HIP for gfx950 + the C-ABI host code) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
SOURCES = [os.path.join(CSRC, "lbm_kernels.hip"), os.path.join(CSRC, "lbm_adjoint.hip"),
           os.path.join(CSRC, "lbm_api.cpp")]
OBJDIR = os.path.join(HERE, "_build")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # a multiply and an add are fused only within one source expression: the rounding of every
    # value is then a property of the source, the same in every kernel that evaluates it (fusing
    # across statements depends on how often a product is used in the surrounding kernel); the
    # temperature kernels opt back into cross-statement fusion with a pragma
    "-ffp-contract=on",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # the kernel arguments arrive preloaded in scalar registers: one dependent memory round trip
    # fewer before a workgroup's first loads (its tile entry, then its run's parameters)
    "-mllvm", "-amdgpu-kernarg-preload-count=8",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel), then link liblbm.so."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJDIR, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
        cmd = [hipcc, *HIPCC_FLAGS, "-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd))
        procs.append((subprocess.Popen(cmd), src))
        objs.append(obj)
    failed = [src for p, src in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, f"hipcc {failed}")
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


C_EXAMPLE_SRC = os.path.join(ROOT, "tests", "c_abi_example.c")
C_EXAMPLE_BIN = os.path.join(ROOT, "tests", "c_abi_example.bin")


def build_c_example(verbose: bool = False) -> str:
    """The plain C consumer of the C ABI used by the tests (gcc, C99, linked against liblbm.so and the
    HIP runtime; finds liblbm.so next to the package through its run path)."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(rocm, "include"),
           "-I", os.path.join(ROOT, "include"), C_EXAMPLE_SRC, "-L", HERE, "-llbm", "-L", os.path.join(rocm, "lib"),
           "-lamdhip64", "-Wl,-rpath," + os.path.join(rocm, "lib"), "-Wl,-rpath,$ORIGIN/../paper_1912_02018_amd",
           "-o", C_EXAMPLE_BIN]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return C_EXAMPLE_BIN


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_c_example(verbose=True))
