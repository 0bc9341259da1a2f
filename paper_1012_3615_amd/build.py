"""Build the HIP library libbri.so for gfx950 (in-tree, no JIT cache).

    python -m paper_1012_3615_amd.build            # compile every source
    python paper_1012_3615_amd/build.py --jobs 8

Each .hip source is compiled to an object with hipcc, then linked into
paper_1012_3615_amd/libbri.so.  Packed FP32 instructions are disabled for
device code (-packed-fp32-ops).  Floating-point contraction is off: the
kernels write every fused multiply-add explicitly, so all launch
configurations of an operation round identically.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libbri.so")
OBJDIR = os.path.join(HERE, "_build")
ARCH = os.environ.get("BRI_OFFLOAD_ARCH", "gfx950")

SOURCES = ["abi.hip", "abi_prod.hip", "apply.hip", "apply_f64.hip", "apply_f32.hip", "apply_f16.hip", "apply_f16h.hip",
           "apply_prod_f64.hip", "apply_prod_f32.hip", "apply_prod_f16.hip", "apply_prod_f16h.hip",
           "build.hip", "production.hip", "overlap.hip", "pack.hip", "blas.hip", "solve.hip", "grad.hip", "wilson.hip", "mfma.hip"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(HERE, "..", "include"),
]


def hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def compile_one(src, extra):
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + FLAGS + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj, r.stderr


def build(jobs=None, extra=None, verbose=False):
    extra = list(extra or [])
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda s: compile_one(s, extra), SOURCES))
    for _, err in results:
        if verbose and err.strip():
            print(err, file=sys.stderr)
    objs = [o for o, _ in results]
    tmp = OUT + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--extra", nargs="*", default=[])
    a = ap.parse_args()
    print(build(a.jobs, a.extra, a.verbose))
