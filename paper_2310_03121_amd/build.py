"""Builds the HIP engine (libnnp.so) for gfx950, in tree.

Every ``csrc/*.hip`` source is compiled with hipcc for gfx950 and linked into
``paper_2310_03121_amd/libnnp.so`` (object files under ``_build/``).  The
benchmark's ceiling microbenchmarks (``ceilings/ceilings.hip``) become
``libnnp_ceilings.so``, built with MFMA operands kept in vector registers so
the issue loops are free of accumulator copies.  Run:
python -m paper_2310_03121_amd.build
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libnnp.so")
CEIL_SRC = os.path.join(PKG, "ceilings", "ceilings.hip")
CEIL_LIB = os.path.join(PKG, "libnnp_ceilings.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc() -> str:
    for p in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if p and os.path.exists(p):
            return p
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("build failed: " + " ".join(cmd) + "\n" + out)
    return out


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    objs = [os.path.join(BUILD, os.path.basename(s)[:-4] + ".o") for s in srcs]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        futs = [ex.submit(_run, [cc, *HIPCC_FLAGS, "-c", s, "-o", o]) for s, o in zip(srcs, objs)]
        for f in futs:
            out = f.result()
            if verbose and out.strip():
                print(out)
    tmp = LIB + ".tmp"
    _run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    tmp = CEIL_LIB + ".tmp"
    _run([cc, *HIPCC_FLAGS, "-mllvm", "-amdgpu-mfma-vgpr-form", "-shared", CEIL_SRC, "-o", tmp])
    os.replace(tmp, CEIL_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
