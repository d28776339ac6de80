"""Build the HIP library libtq.so for gfx950 (MI355X) in-tree.

    python -m paper_2506_00528_amd.build

Every source in csrc/ is compiled by hipcc into _build/ and linked into
paper_2506_00528_amd/libtq.so, which the Python binding loads.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libtq.so")
ARCH = os.environ.get("TQ_OFFLOAD_ARCH", "gfx950")

# (source, plane width): the matrix-core kernels are compiled once per plane
# width (16-byte chunks per plane, 1..8) so their instantiations build in
# parallel; every other source is compiled once.  Slowest first.
SOURCES = [("mfma_kernels.hip", nc) for nc in range(8, 0, -1)] + \
          [("scan.hip", 0), ("batched_kernels.hip", 0), ("encode.hip", 0), ("layout.hip", 0), ("rerank.hip", 0), ("masked.hip", 0), ("sparse.hip", 0), ("noalloc.hip", 0),
           ("api.cpp", 0), ("search.cpp", 0), ("batched.cpp", 0), ("serve.cpp", 0)]

CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-result",
    # never let the compiler form packed fp32 instructions (v_pk_*_f32)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(item: tuple, verbose: bool) -> str:
    src, nc = item
    obj = os.path.join(BUILD, os.path.basename(src) + (f".nc{nc}" if nc else "") + ".o")
    lang = [] if src.endswith(".hip") else ["-x", "hip"]
    defs = [f"-DTQ_NC={nc}"] if nc else []
    cmd = [hipcc()] + lang + CFLAGS + defs + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{msg}")
    if msg.strip() and verbose:
        print(msg, file=sys.stderr)
    return obj


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s[0]))]
    jobs = jobs or min(len(srcs), max(1, min(16, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
