"""Build libmgx.so (all HIP kernels + the C-ABI) for gfx950 with hipcc.

Every translation unit is compiled in parallel, then linked into one shared
library next to this file.  Usage: ``python -m paper_1210_7774_amd.build``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmgx.so")
BUILD = os.path.join(ROOT, "_build")

SOURCES = ["mg_host.hip", "k_generic.hip", "k_tail.hip", "k_march2d_f64.hip", "k_march2d_f32.hip",
           "k_march2d_bf16.hip", "k_learned.hip", "k_tile2d.hip", "k_rb3.hip", "k_jacobi5.hip", "k_march3d.hip",
           "k_march3dw.hip", "ve_host.hip"]

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
         "-Wno-unused-variable", "-Wno-unused-but-set-variable",
         # no packed FP32 instructions (v_pk_*_f32) in any kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


# run-time compilation of the vector engine's generated kernels
LIBS = ["-L/opt/rocm/lib", "-lhiprtc"]


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc") or ""):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build libmgx.so)")


# per-file code generation options: the learned kernels keep MFMA results in
# VGPRs (they feed VALU packing right away; AGPR results cost a copy each)
FILE_FLAGS = {"k_learned.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def _compile(src: str, extra=(), tag="") -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + tag + ".o")
    cmd = [hipcc()] + FLAGS + FILE_FLAGS.get(src, []) + list(extra) + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr))
    return obj


def build(verbose: bool = True, out: str = OUT, defines=()) -> str:
    """Compile and link; `defines` (e.g. ["-DMGX_MARCH_MINW=4"]) and `out`
    allow variant builds for tuning."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = min(len(SOURCES), max(1, os.cpu_count() or 1))
    tag = "" if out == OUT else "_" + os.path.basename(out).replace(".", "_")
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, defines, tag), SOURCES))
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + LIBS
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr)
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build()
    sys.exit(0)
