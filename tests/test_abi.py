"""The C ABI library loads, exports every declared call, and rejects bad
arguments on the host before touching a GPU (runs without a GPU)."""
import ctypes
import subprocess

import pytest

from tests.libtq import HEADER, declared_functions, ensure_built


@pytest.fixture(scope="module")
def tq():
    return ensure_built()


def test_every_declared_symbol_is_exported(tq):
    names = declared_functions()
    assert len(names) >= 20
    out = subprocess.run(["nm", "-D", "--defined-only", tq.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, f"declared in {HEADER} but not exported: {missing}"
    assert sorted(tq.EXPORTS) == names, "binding and header disagree"
    L = tq.lib()
    for n in names:
        assert getattr(L, n) is not None


def test_status_strings(tq):
    assert tq.status_str(0) == "TQ_OK"
    assert tq.status_str(-1) == "TQ_ERR_INVALID"
    assert tq.status_str(-6) == "TQ_ERR_STATE"
    assert tq.status_str(-99) == "TQ_ERR_UNKNOWN"


def test_code_words(tq):
    assert tq.tq_code_words(1) == 1
    assert tq.tq_code_words(32) == 1
    assert tq.tq_code_words(33) == 2
    assert tq.tq_code_words(1024) == 32
    for bad in (0, -3, tq.TQ_MAX_D + 1):
        with pytest.raises(tq.TQError):
            tq.tq_code_words(bad)


def test_host_validation_without_gpu(tq):
    """Every call with invalid arguments is rejected on the host, before any
    GPU work (the checks are shared with the sanitizer run)."""
    from tests import abi_host_checks
    abi_host_checks.run(tq.lib())


def test_default_x_against_the_oracle(tq):
    """The library's closed form against the oracle's brute force over exact
    big-integer vertex counts, for every supported d."""
    import oracle
    for d in range(1, tq.TQ_MAX_D + 1):
        assert tq.tq_default_x(d) == oracle.default_x(d), d
    for bad in (0, -1, tq.TQ_MAX_D + 1):
        with pytest.raises(tq.TQError):
            tq.tq_default_x(bad)
