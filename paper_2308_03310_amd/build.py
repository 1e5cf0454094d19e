"""Build libletkf.so (gfx950) in-tree with hipcc.

Each HIP translation unit compiles in its own process (the unrolled
eigensolver sweeps make the 64-row variant the slowest), then one link step
produces ``paper_2308_03310_amd/libletkf.so``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libletkf.so")

SOURCES = ["k_fused64.hip", "k_fused32.hip", "k_fused16.hip", "k_xf64.hip", "k_xf32.hip",
           "k_xf16.hip", "k_evd64.hip", "k_evd32.hip", "k_evd16.hip", "k_gram.hip", "k_gram_lp.hip",
           "k_prep.hip", "k_lbm.hip", "k_nsqrt.hip", "api.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
MAX_SCRATCH = 256   # bytes of private memory per lane a kernel may use
# The fused kernels build without any: a spilled register's reload waits for
# every memory operation the wavefront has in flight, its scattered ensemble
# stores included.
MAX_SCRATCH_OF = {f"k_fused{k}.hip": 0 for k in (16, 32, 64)}
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed-FP32 instructions in any device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]


# Per-source additions.  The fused kernels' persistent item loop: machine
# loop-invariant code motion would hoist the per-lane arithmetic of the whole
# loop body (Gram and eigensolve) out of it and keep it live throughout
# (register spills); the sources also make the lane index opaque for the same
# reason at the IR level.
EXTRA = {f"k_fused{k}.hip": ["-mllvm", "-disable-machine-licm"] for k in (16, 32, 64)}
# The k = 64 unit (every width from 33 to 64): LLVM's iterative scheduler
# that keeps the occupancy (two wavefronts per SIMD) and then minimizes
# latency.  Measured on the 1024^2, k = 64 analysis: 102.1 -> 99.5 ms (FP32
# form), 121.2 -> 116.1 ms (FP64), bitwise the same results; the
# instruction-level-parallelism and memory-clause strategies, and turning off
# either of its rescheduling stages, were no faster, and the
# register-minimizing strategy was 11 % slower.
EXTRA["k_fused64.hip"] += ["-mllvm", "-amdgpu-sched-strategy=iterative-maxocc"]
# The same for the split form's k = 64 eigensolve and update (1024^2, k = 64:
# 102.0 -> 101.0 ms FP32 form, 124.0 -> 120.2 ms FP64, bitwise the same); at
# k = 32 it made no difference and the default stays.
EXTRA["k_xf64.hip"] = ["-mllvm", "-amdgpu-sched-strategy=iterative-maxocc"]
# And for the standalone eigensolver's k = 64 unit (16,384 matrices: 3.00 ->
# 2.89 ms at k = 48, 3.48 -> 3.35 ms at k = 64, bitwise the same).
EXTRA["k_evd64.hip"] = ["-mllvm", "-amdgpu-sched-strategy=iterative-maxocc"]


def _compile(src: str, force: bool) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    if not force and os.path.exists(obj):
        newest = max(os.path.getmtime(os.path.join(CSRC, f)) for f in os.listdir(CSRC)
                     if f.endswith((".h", ".inc")))
        newest = max(newest, os.path.getmtime(path),
                     os.path.getmtime(os.path.join(ROOT, "include", "letkf.h")))
        if os.path.getmtime(obj) >= newest:
            return obj
    cmd = [HIPCC] + FLAGS + EXTRA.get(src, []) + ["-Rpass-analysis=kernel-resource-usage", "-c",
                                                  path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-4000:]}")
    _check_scratch(src, r.stderr)
    return obj


def _check_scratch(src: str, remarks: str) -> None:
    """Every kernel is written to live in registers and LDS: a kernel that
    spills more than MAX_SCRATCH bytes per lane is a build error (a large
    private segment also makes the runtime's scratch allocation fail)."""
    name = None
    for line in remarks.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            continue
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        limit = MAX_SCRATCH_OF.get(src, MAX_SCRATCH)
        if m and int(m.group(1)) > limit:
            raise RuntimeError(f"{src}: kernel {name} spills {m.group(1)} bytes per lane "
                               f"(limit {limit})")


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile every source for gfx950 and link the shared library; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(lambda s: _compile(s, force), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(force="--force" in sys.argv, verbose=True)
