"""Build libmgemm.so (the HIP kernels and the C-ABI host layer) for gfx950.

Usage: python -m paper_2305_18236_amd.build [--asm]

Each ``csrc/*.hip`` file is compiled by hipcc into an object in ``_build/``
and the objects are linked into ``libmgemm.so`` next to this file.  ``--asm``
also writes the gfx950 assembly of each file to ``_build/<name>.s`` (our own
code only) for register and spill inspection.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libmgemm.so")
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"),
                 shutil.which("hipcc") or ""):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the ROCm toolchain is required to build mgemm")


# Packed-FP32 VALU instructions are disabled for all device code.  Private
# arrays (staging registers) are never moved into LDS behind our back: the
# kernels size their LDS explicitly.
DEVICE_FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-mllvm", "-disable-promote-alloca-to-lds",
                "-Wall", "-Wno-unused-function"]


def build(asm: bool = False, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    procs = []
    objs = []
    for src in srcs:
        name = os.path.splitext(os.path.basename(src))[0]
        obj = os.path.join(BUILD, name + ".o")
        objs.append(obj)
        cmd = [cc, *DEVICE_FLAGS, "-c", src, "-o", obj]
        procs.append((src, cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if asm:
            s_out = os.path.join(BUILD, name + ".s")
            acmd = [cc, *DEVICE_FLAGS, "--cuda-device-only", "-S", src, "-o", s_out]
            procs.append((src + " (asm)", acmd,
                          subprocess.Popen(acmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, cmd, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            failed.append(src)
            sys.stderr.write(f"--- {src}\n{' '.join(cmd)}\n{text}\n")
        elif verbose and text.strip():
            sys.stderr.write(f"--- {src}\n{text}\n")
    if failed:
        raise RuntimeError("hipcc failed for: " + ", ".join(failed))
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(asm="--asm" in sys.argv, verbose="-v" in sys.argv))
