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
          [("scan.hip", 0), ("batched_kernels.hip", 0), ("encode.hip", 0), ("layout.hip", 0), ("rerank.hip", 0), ("masked.hip", 0), ("sparse.hip", 0), ("noalloc.hip", 0), ("clock.hip", 0),
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


# Host sources rebuilt with AddressSanitizer and UndefinedBehaviorSanitizer on
# their host code only (each -fsanitize after -Xarch_host); the device kernels
# keep their normal objects.
SAN_SOURCES = ["api.cpp", "search.cpp", "batched.cpp", "serve.cpp"]
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
SAN_LIB = os.path.join(BUILD, "san", "libtq_san.so")


def asan_runtime() -> str:
    """The compiler's shared AddressSanitizer runtime (to preload into a
    process that loads the sanitizer build)."""
    out = subprocess.run([hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = out.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("AddressSanitizer runtime not found")
    return path


def build_sanitized(verbose: bool = False) -> str:
    """libtq_san.so: the library with its host code instrumented, for tests
    of the host-side paths; load it with asan_runtime() preloaded."""
    if not all(os.path.exists(os.path.join(BUILD, s + (f".nc{nc}" if nc else "") + ".o"))
               for s, nc in SOURCES if s.endswith(".hip")):
        build(verbose)
    san = os.path.dirname(SAN_LIB)
    os.makedirs(san, exist_ok=True)

    def one(src):
        obj = os.path.join(san, src + ".o")
        cmd = [hipcc(), "-x", "hip"] + [f for f in CFLAGS if f != "-O3"] + ["-O1", "-g"] + SAN_FLAGS + \
              ["-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc (sanitizer build) failed on {src}:\n{r.stdout}{r.stderr}")
        return obj

    with cf.ThreadPoolExecutor(len(SAN_SOURCES)) as ex:
        objs = list(ex.map(one, SAN_SOURCES))
    objs += [os.path.join(BUILD, s + (f".nc{nc}" if nc else "") + ".o") for s, nc in SOURCES if s.endswith(".hip")]
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", SAN_LIB + ".tmp"] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed (sanitizer build):\n{r.stdout}{r.stderr}")
    os.replace(SAN_LIB + ".tmp", SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
