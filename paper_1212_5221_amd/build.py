"""Build libgf.so (HIP, gfx950) in-tree.

    python -m paper_1212_5221_amd.build        # or build() from Python

Every .hip / .cpp under csrc/ is compiled with hipcc for gfx950 (the SU(3)
half-sweep table gf_sweep_inst.hip once per gauge and storage) and linked
into paper_1212_5221_amd/libgf.so.  Packed-FP32 instructions are disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgf.so")
ARCH = os.environ.get("GF_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(os.path.dirname(HERE), "include")]

SOURCES = ["gf_api.cpp", "gf_kernels.hip", "gf_sweep_su2.hip", "gf_stream.hip"]
# the SU(3) half-sweep variants: gf_sweep_inst.hip once per gauge (Landau,
# Coulomb, MAG) and storage (FP64-18, FP64-12, FP32-12, single precision)
INST = [("gf_sweep_inst.hip", "gf_sweep_g%d_s%d.o" % (g, st), ["-DGF_GAUGE=%d" % g, "-DGF_STORAGE=%d" % st])
        for g in range(3) for st in range(4)]


def _compile(job) -> str:
    src, objname, defs = job if isinstance(job, tuple) else (job, os.path.splitext(job)[0] + ".o", [])
    obj = os.path.join(BUILD, objname)
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = [HIPCC] + FLAGS + defs + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, out))
    return obj


def build(jobs: int | None = None, verbose: bool = True) -> str:
    """Compile all sources (always) and link libgf.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    work = INST + SOURCES  # the long instantiation units first
    jobs = jobs or min(len(work), os.cpu_count() or 4, 16)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, work))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
