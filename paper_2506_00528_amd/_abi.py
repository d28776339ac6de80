"""ctypes declarations of the C ABI in include/tq.h: the structures and the
argument / result types of every exported call.  No torch here, so a library
build can be loaded and driven on its own (e.g. a sanitizer build of the host
code); the torch binding (tq.py) uses the same declarations."""
from __future__ import annotations

import ctypes


class tq_search_opts(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int), ("check_queries", ctypes.c_int), ("grid", ctypes.c_int),
                ("qtile", ctypes.c_int), ("use_graph", ctypes.c_int), ("engine", ctypes.c_int),
                ("metric", ctypes.c_int), ("reserved", ctypes.c_int * 1)]


class tq_serve_cfg(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("max_slots", ctypes.c_int), ("max_k", ctypes.c_int),
                ("n_segments", ctypes.c_int), ("max_request_nq", ctypes.c_int), ("tick_timeout_us", ctypes.c_int),
                ("engine", ctypes.c_int), ("reserved", ctypes.c_int * 2)]


class tq_req_stats(ctypes.Structure):
    _fields_ = [("submit_ns", ctypes.c_uint64), ("admit_ns", ctypes.c_uint64),
                ("complete_ns", ctypes.c_uint64), ("nq", ctypes.c_int), ("k", ctypes.c_int),
                ("ticks", ctypes.c_int), ("reserved", ctypes.c_int)]


def declare(L: ctypes.CDLL) -> ctypes.CDLL:
    """Set argtypes / restype of every call on a loaded library; returns it."""
    vp, i32, i64, u64, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t
    P = ctypes.POINTER
    sig = {
        "tq_status_str": ([i32], ctypes.c_char_p),
        "tq_last_error": ([], ctypes.c_char_p),
        "tq_version": ([], i32),
        "tq_code_words": ([i32], i32),
        "tq_default_x": ([i32], i32),
        "tq_encode": ([vp, i64, i32, i32, vp, vp], i32),
        "tq_encode_b158": ([vp, i64, i32, vp, vp], i32),
        "tq_db_create": ([vp, i64, i32, i32, vp, P(vp)], i32),
        "tq_db_export": ([vp, vp, vp], i32),
        "tq_db_info": ([vp, P(i64), P(i32), P(i32), P(sz)], i32),
        "tq_db_destroy": ([vp], i32),
        "tq_search_knn": ([vp, vp, i32, i32, vp, vp, P(tq_search_opts), vp], i32),
        "tq_search_knn_noalloc": ([vp, vp, i32, i32, vp, vp, P(tq_search_opts), vp], i32),
        "tq_autotune": ([vp, i32, P(i32), i32, vp], i32),
        "tq_delta_dump": ([vp, vp, i32, vp, vp], i32),
        "tq_rerank": ([vp, i64, i32, vp, i32, vp, i32, i32, vp, vp, vp], i32),
        "tq_search_masked": ([vp, vp, i32, i32, vp, vp, P(tq_search_opts), vp], i32),
        "tq_sync": ([vp], i32),
        "tq_serve_create": ([vp, P(tq_serve_cfg), P(vp)], i32),
        "tq_serve_submit": ([vp, vp, i32, i32, P(u64)], i32),
        "tq_serve_poll": ([vp, u64, vp, vp, P(tq_req_stats)], i32),
        "tq_serve_wait": ([vp, u64, i32, vp, vp, P(tq_req_stats)], i32),
        "tq_serve_cancel": ([vp, u64], i32),
        "tq_serve_stats": ([vp, P(u64), P(u64), P(u64), P(u64)], i32),
        "tq_serve_destroy": ([vp], i32),
        "tq_timing_enable": ([i32], i32),
        "tq_set_device_limit": ([u64], i32),
        "tq_device_bytes": ([P(u64)], i32),
        "tq_clock_mhz": ([P(ctypes.c_double), vp], i32),
        "tq_timing_read": ([i32, P(ctypes.c_double), P(i64), i32], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L
