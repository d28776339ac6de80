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
    L = tq.lib()
    p = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first
    assert L.tq_encode(p, -1, 8, 2, p, None) == tq.TQ_ERR_INVALID
    assert L.tq_encode(p, 4, 0, 1, p, None) == tq.TQ_ERR_INVALID
    assert L.tq_encode(p, 4, 8, 0, p, None) == tq.TQ_ERR_INVALID
    assert L.tq_encode(p, 4, 8, 9, p, None) == tq.TQ_ERR_INVALID
    assert "x=9" in tq.last_error()
    assert L.tq_encode(None, 4, 8, 2, p, None) == tq.TQ_ERR_INVALID
    assert L.tq_encode(None, 0, 8, 2, None, None) == tq.TQ_OK  # nothing to do
    out = ctypes.c_void_p()
    assert L.tq_db_create(None, 10, 8, 2, None, ctypes.byref(out)) == tq.TQ_ERR_INVALID
    assert L.tq_db_create(p, 0, 8, 2, None, ctypes.byref(out)) == tq.TQ_ERR_INVALID
    assert L.tq_db_create(p, 2 ** 31, 8, 2, None, ctypes.byref(out)) == tq.TQ_ERR_INVALID
    assert L.tq_db_create(p, 10, 8, 2, None, None) == tq.TQ_ERR_INVALID
    assert L.tq_search_knn(None, p, 1, 1, p, p, None, None) == tq.TQ_ERR_INVALID
    assert L.tq_db_export(None, p, None) == tq.TQ_ERR_INVALID
    assert L.tq_delta_dump(None, p, 1, p, None) == tq.TQ_ERR_INVALID
    assert L.tq_db_destroy(None) == tq.TQ_OK
    assert L.tq_serve_destroy(None) == tq.TQ_OK
    assert L.tq_timing_read(7, None, None, 0) == tq.TQ_ERR_INVALID


def test_rerank_host_validation_without_gpu(tq):
    L = tq.lib()
    p = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first
    assert L.tq_rerank(None, 10, 8, p, 1, p, 4, 2, p, p, None) == tq.TQ_ERR_INVALID
    assert L.tq_rerank(p, 0, 8, p, 1, p, 4, 2, p, p, None) == tq.TQ_ERR_INVALID
    assert L.tq_rerank(p, 10, 0, p, 1, p, 4, 2, p, p, None) == tq.TQ_ERR_INVALID
    assert L.tq_rerank(p, 10, tq.TQ_MAX_D + 1, p, 1, p, 4, 2, p, p, None) == tq.TQ_ERR_INVALID
    assert L.tq_rerank(p, 10, 8, p, -1, p, 4, 2, p, p, None) == tq.TQ_ERR_INVALID
    assert L.tq_rerank(p, 10, 8, p, 1, p, 0, 1, p, p, None) == tq.TQ_ERR_INVALID
    assert L.tq_rerank(p, 10, 8, p, 1, p, tq.TQ_MAX_RERANK + 1, 2, p, p, None) == tq.TQ_ERR_INVALID
    assert L.tq_rerank(p, 10, 8, p, 1, p, 4, 5, p, p, None) == tq.TQ_ERR_INVALID
    assert "k=5" in tq.last_error()
    assert L.tq_rerank(p, 10, 8, p, 1, p, 4, 0, p, p, None) == tq.TQ_ERR_INVALID
    assert L.tq_rerank(p, 10, 8, p, 0, p, 4, 2, p, p, None) == tq.TQ_OK  # nothing to do


def test_masked_host_validation_without_gpu(tq):
    L = tq.lib()
    p = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first
    assert L.tq_search_masked(None, p, 1, 1, p, p, None, None) == tq.TQ_ERR_INVALID
    assert L.tq_timing_read(3, None, None, 0) == tq.TQ_OK  # index-list scan family
    assert L.tq_timing_read(4, None, None, 0) == tq.TQ_ERR_INVALID


def test_default_x_against_the_oracle(tq):
    """The library's closed form against the oracle's brute force over exact
    big-integer vertex counts, for every supported d."""
    import oracle
    for d in range(1, tq.TQ_MAX_D + 1):
        assert tq.tq_default_x(d) == oracle.default_x(d), d
    for bad in (0, -1, tq.TQ_MAX_D + 1):
        with pytest.raises(tq.TQError):
            tq.tq_default_x(bad)
