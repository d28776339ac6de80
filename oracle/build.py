"""Build the CPU oracle (oracle.c) with gcc into oracle/liboracle.so.

Test infrastructure; see oracle/__init__.py.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(HERE, "oracle.c")


def library_path(mutant: int = 0, out_dir: str | None = None) -> str:
    name = "liboracle.so" if mutant == 0 else f"liboracle_mutant{mutant}.so"
    return os.path.join(out_dir or HERE, name)


def build(mutant: int = 0, out_dir: str | None = None, verbose: bool = False) -> str:
    out = library_path(mutant, out_dir)
    cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           f"-DORACLE_MUTANT={int(mutant)}", SOURCE, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
