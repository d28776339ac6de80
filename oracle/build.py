"""Build the CPU oracle (oracle.c) with gcc into oracle/liboracle.so.

Test infrastructure; see oracle/__init__.py.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(HERE, "oracle.c")


def library_path(mutant: int = 0, out_dir: str | None = None, sanitize: bool = False) -> str:
    name = "liboracle.so" if mutant == 0 else f"liboracle_mutant{mutant}.so"
    if sanitize:
        name = name.replace(".so", "_san.so")
    return os.path.join(out_dir or HERE, name)


# AddressSanitizer + UndefinedBehaviorSanitizer (gcc): a process that loads
# the sanitized library needs gcc's libasan preloaded (asan_runtime()).
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined", "-g"]


def asan_runtime() -> str:
    out = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True, check=True)
    return out.stdout.strip()


def build(mutant: int = 0, out_dir: str | None = None, verbose: bool = False, sanitize: bool = False) -> str:
    out = library_path(mutant, out_dir, sanitize)
    cmd = ["gcc", "-std=c11", "-O1" if sanitize else "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           f"-DORACLE_MUTANT={int(mutant)}"] + (SAN_FLAGS if sanitize else []) + [SOURCE, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
