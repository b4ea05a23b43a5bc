"""Build librpyfmm.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1711_02976_amd.build          # or build() from Python
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "librpyfmm.so")
SOURCES = ["tree.hip", "fmm.hip", "p2e.hip", "eval.hip", "m2l_rot.hip", "nearfield.hip", "krylov.hip", "api.hip"]
ARCH = os.environ.get("RPYFMM_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    # packed FP32 arithmetic stays disabled in every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # hardware FP64 atomic add on (coarse-grained) device memory
    "-munsafe-fp-atomics",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


HEADERS = [os.path.join(CSRC, h) for h in ("common.h", "fmm.h")]
ABI_HEADER = os.path.join(os.path.dirname(HERE), "include", "rpyfmm.h")


def _stale(src_path: str, obj: str) -> bool:
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [src_path, *HEADERS] + ([ABI_HEADER] if src_path.endswith("api.hip") else [])
    return any(os.path.getmtime(f) > t for f in deps if os.path.exists(f))


def _compile(src: str, force: bool = True) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    if not force and not _stale(os.path.join(CSRC, src), obj):
        return obj
    cmd = [HIPCC, *CFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    if r.stderr.strip():
        sys.stderr.write(r.stderr)
    return obj


def build(verbose: bool = False, force: bool = True) -> str:
    """Compile every source (force) or only stale objects, then link."""
    os.makedirs(OBJDIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(6, len(SOURCES))) as ex:
        objs = list(ex.map(lambda f: _compile(f, force), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, force="--incremental" not in sys.argv)
