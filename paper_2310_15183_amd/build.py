"""Build libgrtrace.so (HIP, gfx950) in-tree with hipcc.

Every translation unit is compiled with -ffp-contract=off (the binary64
tracer's operation sequence is fixed; fused products are explicit fma calls)
and with packed FP32 instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgrtrace.so")
ARCH = os.environ.get("GRTRACE_ARCH", "gfx950")

SOURCES = ["api.hip", "trace_fp64.hip", "trace_mixed.hip", "trace_mn.hip", "shade.hip",
           "redshift.hip", "order.hip", "mlp.hip", "mlp_api.hip", "surrogate.hip", "diag.hip"]
HEADERS = ["grmath.h", "internal.h", "step_fp64.h", "mlp_internal.h", "surrogate_internal.h"]

# Per-source options.  The binary64 tracers' steps are long blocks of
# arithmetic whose three metric evaluations per stage are independent; where
# few waves are left (the trapped Manko-Novikov rays at the end of a frame,
# the short fallback lists of the surrogate) the frame time is one wave's
# latency, and LLVM's instruction-level-parallel scheduler, which interleaves
# the independent chains, shortens it.  Throughput-bound launches are not
# slower with it; the mixed-precision tracer is, and keeps the default.
EXTRA = {src: ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]
         for src in ("trace_fp64.hip", "trace_mn.hip")}

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", f"-I{INCLUDE}", f"-I{CSRC}"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed ({r.returncode})")
    return r


def build(verbose: bool = False) -> str:
    """Compile every source and link libgrtrace.so (always rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        cmd = [HIPCC, *FLAGS, *EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd))
        cmds.append(cmd)
        objs.append(obj)
    # one hipcc per source, a few at a time
    with ThreadPoolExecutor(max_workers=max(1, min(8, os.cpu_count() or 1))) as pool:
        list(pool.map(_run, cmds))
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
