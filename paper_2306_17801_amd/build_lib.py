"""Build step for the HIP library: compiles csrc/*.hip for gfx950 into
libapcg.so next to this file (in-tree, so it travels with the source).

Each source is compiled to its own object in parallel (under _build/ at the
repository root), then the objects are linked into the shared library."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["runtime.hip", "blas.hip", "pcg.hip", "batched.hip", "learn.hip", "fcg.hip", "batched_fcg.hip",
           "tfqmr.hip", "intent.hip", "expr.hip", "persist.hip", "tune.hip"]
LIB = os.path.join(HERE, "libapcg.so")
OBJDIR = os.path.join(ROOT, "_build")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result", "-Wno-unused-value",
]


def _jobs() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16, len(SOURCES)))


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = [os.path.join(HERE, "csrc", s) for s in SOURCES]
    objs = [os.path.join(OBJDIR, os.path.splitext(s)[0] + ".o") for s in SOURCES]

    def compile_one(pair):
        src, obj = pair
        cmd = [hipcc, *HIPCC_FLAGS, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        return subprocess.run(cmd, capture_output=True, text=True)

    with ThreadPoolExecutor(_jobs()) as ex:
        results = list(ex.map(compile_one, zip(srcs, objs)))
    failed = False
    for src, r in zip(srcs, results):
        msg = "\n".join(l for l in (r.stderr or "").splitlines() if "packed-fp32-ops" not in l)
        if msg.strip():
            print(msg, file=sys.stderr)
        if r.returncode != 0:
            print(f"build_lib: compiling {os.path.basename(src)} failed", file=sys.stderr)
            failed = True
    if failed:
        raise RuntimeError("HIP compilation failed")
    tmp = LIB + ".tmp"
    subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
