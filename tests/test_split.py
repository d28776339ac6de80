"""The batched split's buffer and coverage invariants, checked on the host.

batch_split (paper_2506_00528_amd/csrc/tq_batched.h) sizes the (query tile,
database part) items of every batched and served scan; the list buffers and
the merge are sized from batch_max_lists / batch_max_parts.  The check program
(tests/split_invariants.cpp) includes the header with the host compiler and
sweeps query counts, query tiles, grids and database sizes."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(os.path.join(ROCM, "include", "hip")),
                    reason="needs g++ and the HIP headers")
def test_split_invariants(tmp_path):
    exe = tmp_path / "split_invariants"
    cmd = ["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include",
           "-I" + os.path.join(ROOT, "paper_2506_00528_amd", "csrc"), "-I" + os.path.join(ROOT, "include"),
           os.path.join(HERE, "split_invariants.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0 and out.stdout.startswith("OK"), out.stdout + out.stderr
