"""The oracle and the library's host-side paths under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).  Each runs in a child process with the
sanitizer runtime preloaded: the oracle's pins on a sanitizer build of
oracle.c, and the host-side argument checks of the C ABI on a build of the
library whose host code is instrumented.  Any report fails the child."""
import os
import subprocess
import sys
import textwrap

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:exitcode=86",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1:exitcode=87"}


def run_child(code, preload):
    env = dict(os.environ, LD_PRELOAD=preload, **SAN_ENV)
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    r = subprocess.run([sys.executable, "-c", textwrap.dedent(code)], env=env, capture_output=True, text=True,
                       timeout=600, cwd=ROOT)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "Sanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


def test_oracle_pins_under_sanitizers(tmp_path):
    from oracle.build import asan_runtime, build
    lib = build(out_dir=str(tmp_path), sanitize=True)
    out = run_child(f"""
        import oracle
        from tests import pins
        o = oracle.Oracle(oracle.load({lib!r}))
        for check in pins.ALL_CHECKS:
            check(o)
        print("pins", len(pins.ALL_CHECKS))
        """, asan_runtime())
    assert "pins" in out


def test_abi_host_paths_under_sanitizers():
    from paper_2506_00528_amd.build import asan_runtime, build_sanitized
    lib = build_sanitized()
    out = run_child(f"""
        import ctypes
        from paper_2506_00528_amd._abi import declare
        from tests import abi_host_checks
        abi_host_checks.run(declare(ctypes.CDLL({lib!r})))
        print("host checks done")
        """, asan_runtime())
    assert "host checks done" in out
