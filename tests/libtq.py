"""Locate the HIP library for the tests; it is built only where none exists
yet (a library already built is loaded as it is)."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tq.h")


def ensure_built():
    from paper_2506_00528_amd import tq
    if not os.path.exists(tq.LIB_PATH):
        from paper_2506_00528_amd.build import build
        build()
    return tq


def declared_functions():
    """Names of the functions declared in include/tq.h."""
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tq_[a-z_0-9]+)\s*\(", src)))
