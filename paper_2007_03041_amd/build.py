"""Build the gfx950 shared library ``libsc.so`` in-tree with hipcc.

Usage: ``python -m paper_2007_03041_amd.build`` (also called by ``__graft_entry__.build()``).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsc.so")
# the line-pass units first: they take longest
SOURCES = ["sc_lp_f64_o4.hip", "sc_lp_f64_o6.hip", "sc_lp_f32_o4.hip", "sc_lp_f32_o6.hip", "sc_lp_f64_o4_full.hip",
           "sc_lp_f64_o6_full.hip", "sc_lp_f32_o4_full.hip", "sc_lp_f32_o6_full.hip", "sc_api.cpp", "sc_batch.cpp",
           "sc_coeffs.cpp", "sc_hj.cpp", "sc_hj_kernels.hip", "sc_kernels.hip", "sc_noalloc.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = [
    "-O3", "-std=c++17", "-fPIC", "-Wall",
    f"--offload-arch={ARCH}",
    # no packed FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every unit (in parallel, one hipcc per unit) and link ``libsc.so``."""
    obj_dir = os.path.join(HERE, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1, 8)
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(obj_dir, os.path.splitext(src)[0] + ".o")
        cmds.append([HIPCC, *COMMON, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    running, failed = [], []
    pending = list(cmds)
    while pending or running:
        while pending and len(running) < jobs:
            cmd = pending.pop(0)
            if verbose:
                print(" ".join(cmd), flush=True)
            running.append((cmd, subprocess.Popen(cmd)))
        cmd, proc = running.pop(0)
        if proc.wait() != 0:
            failed.append(cmd[-3])
    if failed:
        raise RuntimeError(f"hipcc failed on {failed}")
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


# the units holding only host code (validation, planning, launches): the sanitizer build
# instruments these and links them with the kernel units of the last build()
HOST_UNITS = ["sc_api.cpp", "sc_batch.cpp", "sc_coeffs.cpp", "sc_hj.cpp", "sc_noalloc.hip"]
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]


def build_sanitized(out_dir: str) -> str:
    """``libsc_asan.so`` in out_dir: the host units built with AddressSanitizer and
    UndefinedBehaviorSanitizer (host code only), linked with the kernel objects of build().  Load it
    with SC_LIBRARY_PATH and the clang ASan runtime preloaded (see ``asan_runtime``)."""
    obj_dir = os.path.join(HERE, "_build")
    kernels = [os.path.join(obj_dir, os.path.splitext(s)[0] + ".o") for s in SOURCES if s not in HOST_UNITS]
    if not all(os.path.exists(k) for k in kernels):
        build()
    os.makedirs(out_dir, exist_ok=True)
    procs, objs = [], []
    for src in HOST_UNITS:
        obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, *COMMON, *SANITIZE, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stderr=subprocess.DEVNULL)))
        objs.append(obj)
    failed = [src for src, p in procs if p.wait() != 0]
    if failed:
        raise RuntimeError(f"hipcc failed on {failed}")
    lib = os.path.join(out_dir, "libsc_asan.so")
    subprocess.check_call([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-fsanitize=address",
                           "-shared-libsan", "-o", lib, *objs, *kernels], stderr=subprocess.DEVNULL)
    return lib


def asan_runtime() -> str:
    """The clang AddressSanitizer runtime that ``libsc_asan.so`` needs preloaded."""
    out = subprocess.run([HIPCC.replace("hipcc", "amdclang++"), "-print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(out) or not os.path.exists(out):
        import glob

        cands = glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        out = cands[0] if cands else ""
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
