"""Calls of the C ABI that must be rejected (or need no GPU) on the host,
before any GPU work: argument validation, status strings, sizes.  Takes a
ctypes library declared by paper_2506_00528_amd._abi.declare, so it runs on
the normal build and, in a separate process, on the sanitizer build of the
host code; it imports no torch."""
import ctypes

OK, INVALID = 0, -1
MAX_D, MAX_K, MAX_RERANK = 1024, 512, 1024


def run(L):
    p = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first
    err = lambda: L.tq_last_error().decode()
    # sizes and names
    assert L.tq_code_words(1) == 1 and L.tq_code_words(33) == 2 and L.tq_code_words(1024) == 32
    assert L.tq_code_words(0) == INVALID and L.tq_code_words(MAX_D + 1) == INVALID
    assert L.tq_default_x(500) == 333 and L.tq_default_x(768) == 512 and L.tq_default_x(0) == INVALID
    assert L.tq_status_str(-2) == b"TQ_ERR_NOMEM" and L.tq_status_str(-99) == b"TQ_ERR_UNKNOWN"
    # encode
    assert L.tq_encode(p, -1, 8, 2, p, None) == INVALID
    assert L.tq_encode(p, 4, 0, 1, p, None) == INVALID
    assert L.tq_encode(p, 4, 8, 0, p, None) == INVALID
    assert L.tq_encode(p, 4, 8, 9, p, None) == INVALID
    assert "x=9" in err()
    assert L.tq_encode(None, 4, 8, 2, p, None) == INVALID
    assert L.tq_encode(None, 0, 8, 2, None, None) == OK  # nothing to do
    assert L.tq_encode_b158(p, -1, 8, p, None) == INVALID
    assert L.tq_encode_b158(p, 4, MAX_D + 1, p, None) == INVALID
    # database
    out = ctypes.c_void_p()
    assert L.tq_db_create(None, 10, 8, 2, None, ctypes.byref(out)) == INVALID
    assert L.tq_db_create(p, 0, 8, 2, None, ctypes.byref(out)) == INVALID
    assert L.tq_db_create(p, 2 ** 31, 8, 2, None, ctypes.byref(out)) == INVALID
    assert L.tq_db_create(p, 10, 8, 9, None, ctypes.byref(out)) == INVALID
    assert L.tq_db_create(p, 10, 8, 2, None, None) == INVALID
    assert L.tq_db_export(None, p, None) == INVALID
    assert L.tq_db_info(None, None, None, None, None) == INVALID
    assert L.tq_db_destroy(None) == OK
    # search
    assert L.tq_search_knn(None, p, 1, 1, p, p, None, None) == INVALID
    assert L.tq_search_knn_noalloc(None, p, 1, 1, p, p, None, None) == INVALID
    assert L.tq_search_masked(None, p, 1, 1, p, p, None, None) == INVALID
    assert L.tq_delta_dump(None, p, 1, p, None) == INVALID
    assert L.tq_autotune(None, 8, None, 0, None) == INVALID
    # refinement
    assert L.tq_rerank(None, 10, 8, p, 1, p, 4, 2, p, p, None) == INVALID
    assert L.tq_rerank(p, 0, 8, p, 1, p, 4, 2, p, p, None) == INVALID
    assert L.tq_rerank(p, 10, 0, p, 1, p, 4, 2, p, p, None) == INVALID
    assert L.tq_rerank(p, 10, MAX_D + 1, p, 1, p, 4, 2, p, p, None) == INVALID
    assert L.tq_rerank(p, 10, 8, p, -1, p, 4, 2, p, p, None) == INVALID
    assert L.tq_rerank(p, 10, 8, p, 1, p, 0, 1, p, p, None) == INVALID
    assert L.tq_rerank(p, 10, 8, p, 1, p, MAX_RERANK + 1, 2, p, p, None) == INVALID
    assert L.tq_rerank(p, 10, 8, p, 1, p, 4, 5, p, p, None) == INVALID
    assert "k=5" in err()
    assert L.tq_rerank(p, 10, 8, p, 1, p, 4, 0, p, p, None) == INVALID
    assert L.tq_rerank(p, 10, 8, p, 0, p, 4, 2, p, p, None) == OK  # nothing to do
    # serving
    srv = ctypes.c_void_p()
    assert L.tq_serve_create(None, None, ctypes.byref(srv)) == INVALID
    assert L.tq_serve_create(p, None, None) == INVALID
    assert L.tq_serve_submit(None, p, 1, 1, None) == INVALID
    assert L.tq_serve_poll(None, 1, None, None, None) == INVALID
    assert L.tq_serve_cancel(None, 1) == INVALID
    assert L.tq_serve_destroy(None) == OK
    # measurement and memory bound
    assert L.tq_timing_read(7, None, None, 0) == INVALID
    assert L.tq_timing_read(3, None, None, 0) == OK  # index-list scan family
    assert L.tq_timing_read(4, None, None, 0) == INVALID
    held = ctypes.c_uint64()
    assert L.tq_device_bytes(None) == INVALID
    assert L.tq_clock_mhz(None, None) == INVALID
    assert L.tq_device_bytes(ctypes.byref(held)) == OK
    assert L.tq_set_device_limit(1 << 30) == OK and L.tq_set_device_limit(0) == OK
