"""Thin Python binding of the C ABI in include/tq.h (libtq.so).

Argument marshalling only: every step of the search runs in the HIP library.
Functions keep the C names (``tq_encode``, ``tq_db_create``, ``tq_search_knn``,
``tq_serve_submit`` ...) and take torch tensors where the C call takes device
pointers; ``stream`` defaults to torch's current stream on the tensor's device.
Code tensors are ``torch.int32`` holding the canonical uint32 bit patterns.

The library must have been built (``python -m paper_2506_00528_amd.build``);
there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import torch  # imported first so libtq.so binds to the HIP runtime torch loaded

from ._abi import declare, tq_req_stats, tq_search_opts, tq_serve_cfg  # noqa: E402

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtq.so")

TQ_OK = 0
TQ_ERR_INVALID = -1
TQ_ERR_NOMEM = -2
TQ_ERR_DEVICE = -3
TQ_ERR_AGAIN = -4
TQ_ERR_NOTFOUND = -5
TQ_ERR_STATE = -6

TQ_PATH_AUTO = 0
TQ_PATH_PLAIN = 1
TQ_PATH_BATCHED = 2

TQ_ENGINE_AUTO = 0
TQ_ENGINE_POPCOUNT = 1
TQ_ENGINE_MATRIX = 2
TQ_ENGINE_SPARSE = 3

TQ_METRIC_DELTA = 0
TQ_METRIC_L2 = 1

TQ_MAX_D = 1024
TQ_MAX_K = 512

# Every function declared in include/tq.h (checked by the tests).
EXPORTS = (
    "tq_status_str", "tq_last_error", "tq_version", "tq_code_words", "tq_encode", "tq_db_create",
    "tq_db_export", "tq_db_info", "tq_db_destroy", "tq_search_knn", "tq_autotune", "tq_delta_dump", "tq_sync",
    "tq_serve_create", "tq_serve_submit", "tq_serve_poll", "tq_serve_wait", "tq_serve_cancel",
    "tq_serve_stats", "tq_serve_destroy", "tq_timing_enable", "tq_timing_read", "tq_rerank",
    "tq_search_masked", "tq_default_x", "tq_encode_b158", "tq_search_knn_noalloc", "tq_set_device_limit",
    "tq_device_bytes", "tq_clock_mhz",
)


class TQError(RuntimeError):
    def __init__(self, status: int, call: str, detail: str):
        super().__init__(f"{call}: {status_str(status)}: {detail}")
        self.status = status


_lib = None


def lib(path: Optional[str] = None):
    """The loaded libtq.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"HIP library {p} is not built; run python -m paper_2506_00528_amd.build first")
    L = declare(ctypes.CDLL(p))
    if path is None:
        _lib = L
    return L


def status_str(status: int) -> str:
    return lib().tq_status_str(int(status)).decode()


def last_error() -> str:
    return lib().tq_last_error().decode()


def _check(rc: int, call: str) -> int:
    if rc != TQ_OK:
        raise TQError(rc, call, last_error())
    return rc


def _stream(t: Optional[torch.Tensor], stream) -> int:
    if stream is not None:
        return int(stream.cuda_stream if hasattr(stream, "cuda_stream") else stream)
    dev = t.device if t is not None else torch.device("cuda", torch.cuda.current_device())
    return int(torch.cuda.current_stream(dev).cuda_stream)


def _dev(t: torch.Tensor, name: str, dtype: torch.dtype) -> int:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def tq_default_x(d: int) -> int:
    """x with the most {x,d} vertices (see tq.h)."""
    r = lib().tq_default_x(int(d))
    if r < 0:
        _check(r, "tq_default_x")
    return r


def tq_code_words(d: int) -> int:
    rc = lib().tq_code_words(int(d))
    if rc < 0:
        raise TQError(rc, "tq_code_words", last_error())
    return rc


def tq_encode(X: torch.Tensor, x: int, codes: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Nearest {x,d} EVP vertices of the rows of X (n x d float32, on the GPU),
    as canonical codes (n x 2W int32 holding uint32 bit patterns)."""
    if X.dim() != 2:
        raise ValueError("X must be n x d")
    n, d = X.shape
    W = tq_code_words(d)
    with torch.cuda.device(X.device):
        if codes is None:
            codes = torch.empty((n, 2 * W), dtype=torch.int32, device=X.device)
        if tuple(codes.shape) != (n, 2 * W):
            raise ValueError("codes has the wrong shape")
        _check(lib().tq_encode(_dev(X, "X", torch.float32), n, d, int(x), _dev(codes, "codes", torch.int32),
                               _stream(X, stream)), "tq_encode")
    return codes


def tq_encode_b158(X: torch.Tensor, codes: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """b1.58 (absmean) ternary codes of the rows of X (see tq.h)."""
    if X.dim() != 2:
        raise ValueError("X must be n x d")
    n, d = X.shape
    W = tq_code_words(d)
    with torch.cuda.device(X.device):
        if codes is None:
            codes = torch.empty((n, 2 * W), dtype=torch.int32, device=X.device)
        if tuple(codes.shape) != (n, 2 * W):
            raise ValueError("codes has the wrong shape")
        _check(lib().tq_encode_b158(_dev(X, "X", torch.float32), n, d, _dev(codes, "codes", torch.int32),
                                    _stream(X, stream)), "tq_encode_b158")
    return codes


def tq_sync(stream=None, device=None) -> None:
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    with torch.cuda.device(dev):
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        _check(lib().tq_sync(_stream(None, s)), "tq_sync")


class tq_db:
    """Owning handle of a resident database (tq_db_create / tq_db_destroy)."""

    def __init__(self, codes: torch.Tensor, d: int, x: int, stream=None):
        if codes.dim() != 2:
            raise ValueError("codes must be n x 2W")
        self.n, self.d, self.x = int(codes.shape[0]), int(d), int(x)
        self.W = tq_code_words(d)
        if codes.shape[1] != 2 * self.W:
            raise ValueError("code width does not match d")
        self.device = codes.device
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().tq_db_create(_dev(codes, "codes", torch.int32), self.n, self.d, self.x,
                                      _stream(codes, stream), ctypes.byref(self._h)), "tq_db_create")

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("database was destroyed")
        return self._h

    def info(self):
        n, d, x, b = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int(), ctypes.c_size_t()
        _check(lib().tq_db_info(self.handle, ctypes.byref(n), ctypes.byref(d), ctypes.byref(x), ctypes.byref(b)),
               "tq_db_info")
        return n.value, d.value, x.value, b.value

    def destroy(self):
        if self._h:
            with torch.cuda.device(self.device):
                torch.cuda.synchronize(self.device)
                _check(lib().tq_db_destroy(self._h), "tq_db_destroy")
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def tq_db_create(codes: torch.Tensor, d: int, x: int, stream=None) -> tq_db:
    return tq_db(codes, d, x, stream)


def tq_db_destroy(db: tq_db) -> None:
    db.destroy()


def tq_db_export(db: tq_db, codes: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    with torch.cuda.device(db.device):
        if codes is None:
            codes = torch.empty((db.n, 2 * db.W), dtype=torch.int32, device=db.device)
        _check(lib().tq_db_export(db.handle, _dev(codes, "codes", torch.int32), _stream(codes, stream)),
               "tq_db_export")
    return codes


def _opts(path=TQ_PATH_AUTO, check_queries=False, grid=0, qtile=0, use_graph=1, engine=TQ_ENGINE_AUTO,
          metric=TQ_METRIC_DELTA):
    o = tq_search_opts()
    o.path, o.check_queries, o.grid, o.qtile, o.use_graph = int(path), int(bool(check_queries)), int(grid), \
        int(qtile), int(use_graph)
    o.engine = int(engine)
    o.metric = int(metric)
    return o


def tq_search_knn(db: tq_db, qcodes: torch.Tensor, k: int, path: int = TQ_PATH_AUTO, check_queries: bool = False,
                  grid: int = 0, qtile: int = 0, use_graph: int = 1, engine: int = TQ_ENGINE_AUTO,
                  ids: Optional[torch.Tensor] = None,
                  scores: Optional[torch.Tensor] = None, stream=None,
                  metric: int = TQ_METRIC_DELTA) -> Tuple[torch.Tensor, torch.Tensor]:
    """Top-k (ids, scores) of every query code, nearest first (score desc, id
    asc); the score is Delta, or 2 Delta - nnz(v) with metric=TQ_METRIC_L2."""
    if qcodes.dim() != 2 or qcodes.shape[1] != 2 * db.W:
        raise ValueError("qcodes must be nq x 2W for the database's d")
    nq = int(qcodes.shape[0])
    with torch.cuda.device(db.device):
        if ids is None:
            ids = torch.empty((nq, k), dtype=torch.int32, device=db.device)
        if scores is None:
            scores = torch.empty((nq, k), dtype=torch.int32, device=db.device)
        o = _opts(path, check_queries, grid, qtile, use_graph, engine, metric)
        _check(lib().tq_search_knn(db.handle, _dev(qcodes, "qcodes", torch.int32), nq, int(k),
                                   _dev(ids, "ids", torch.int32), _dev(scores, "scores", torch.int32),
                                   ctypes.byref(o), _stream(qcodes, stream)), "tq_search_knn")
    return ids, scores


def tq_search_knn_noalloc(db: tq_db, qcodes: torch.Tensor, k: int, ids: torch.Tensor, scores: torch.Tensor,
                          path: int = TQ_PATH_PLAIN, grid: int = 0, engine: int = TQ_ENGINE_AUTO,
                          check_queries: bool = False, stream=None, metric: int = TQ_METRIC_DELTA) -> None:
    """tq_search_knn's plain path into caller-provided ids / scores, with the
    library's fixed scratch array (no device allocation in the call)."""
    if qcodes.dim() != 2 or qcodes.shape[1] != 2 * db.W:
        raise ValueError("qcodes must be nq x 2W for the database's d")
    nq = int(qcodes.shape[0])
    if tuple(ids.shape) != (nq, k) or tuple(scores.shape) != (nq, k):
        raise ValueError("ids and scores must be nq x k")
    with torch.cuda.device(db.device):
        o = _opts(path, check_queries, grid, 0, 1, engine, metric)
        _check(lib().tq_search_knn_noalloc(db.handle, _dev(qcodes, "qcodes", torch.int32), nq, int(k),
                                           _dev(ids, "ids", torch.int32), _dev(scores, "scores", torch.int32),
                                           ctypes.byref(o), _stream(qcodes, stream)), "tq_search_knn_noalloc")


def tq_autotune(db: tq_db, nq_max: int, ks, stream=None) -> None:
    """Pick the fastest batched / plain shapes per batch-size bucket and k."""
    arr = (ctypes.c_int * len(ks))(*[int(k) for k in ks])
    with torch.cuda.device(db.device):
        _check(lib().tq_autotune(db.handle, int(nq_max), arr, len(ks), _stream(None, stream)), "tq_autotune")


def tq_delta_dump(db: tq_db, qcodes: torch.Tensor, stream=None) -> torch.Tensor:
    nq = int(qcodes.shape[0])
    with torch.cuda.device(db.device):
        out = torch.empty((nq, db.n), dtype=torch.int32, device=db.device)
        _check(lib().tq_delta_dump(db.handle, _dev(qcodes, "qcodes", torch.int32), nq,
                                   _dev(out, "delta", torch.int32), _stream(qcodes, stream)), "tq_delta_dump")
    return out


def tq_search_masked(db: "tq_db", Q: torch.Tensor, k: int, grid: int = 0, ids: Optional[torch.Tensor] = None,
                     scores: Optional[torch.Tensor] = None, stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """k nearest database codes of each float query by masked addition
    (see tq.h); Q: nq x d float32 on the GPU."""
    nq = int(Q.shape[0])
    if Q.dim() != 2 or int(Q.shape[1]) != db.d:
        raise ValueError("Q must be nq x d")
    with torch.cuda.device(db.device):
        if ids is None:
            ids = torch.empty((nq, k), dtype=torch.int32, device=db.device)
        if scores is None:
            scores = torch.empty((nq, k), dtype=torch.float32, device=db.device)
        opts = tq_search_opts()
        opts.grid = int(grid)
        _check(lib().tq_search_masked(db.handle, _dev(Q, "Q", torch.float32), nq, int(k),
                                      _dev(ids, "ids", torch.int32), _dev(scores, "scores", torch.float32),
                                      ctypes.byref(opts), _stream(Q, stream)), "tq_search_masked")
    return ids, scores


TQ_MAX_RERANK = 1024


def tq_rerank(X: torch.Tensor, Q: torch.Tensor, cand: torch.Tensor, k: int, ids: Optional[torch.Tensor] = None,
              scores: Optional[torch.Tensor] = None, stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """The k best of each query's candidate ids by the float scalar product
    (double precision); see tq.h.  X: n x d float32, Q: nq x d float32,
    cand: nq x ncand int32, all on the GPU."""
    n, d = int(X.shape[0]), int(X.shape[1])
    nq, ncand = int(cand.shape[0]), int(cand.shape[1])
    if Q.shape[0] != nq or Q.shape[1] != d:
        raise ValueError("Q must be nq x d")
    with torch.cuda.device(X.device):
        if ids is None:
            ids = torch.empty((nq, k), dtype=torch.int32, device=X.device)
        if scores is None:
            scores = torch.empty((nq, k), dtype=torch.float64, device=X.device)
        _check(lib().tq_rerank(_dev(X, "X", torch.float32), n, d, _dev(Q, "Q", torch.float32), nq,
                               _dev(cand, "cand", torch.int32), ncand, int(k), _dev(ids, "ids", torch.int32),
                               _dev(scores, "scores", torch.float64), _stream(X, stream)), "tq_rerank")
    return ids, scores


def tq_set_device_limit(nbytes: int) -> None:
    """Bound on the device memory the library holds (0 = none)."""
    _check(lib().tq_set_device_limit(int(nbytes)), "tq_set_device_limit")


def tq_device_bytes() -> int:
    """Device bytes the library holds now."""
    v = ctypes.c_uint64()
    _check(lib().tq_device_bytes(ctypes.byref(v)), "tq_device_bytes")
    return int(v.value)


def tq_clock_mhz(stream=None) -> float:
    """Shader clock of the current device in MHz, measured under load."""
    v = ctypes.c_double()
    _check(lib().tq_clock_mhz(ctypes.byref(v), _stream(None, stream)), "tq_clock_mhz")
    return float(v.value)


def tq_timing_enable(on: bool = True) -> None:
    _check(lib().tq_timing_enable(int(bool(on))), "tq_timing_enable")


def tq_timing_read(which: int = 0, reset: bool = False) -> Tuple[float, int]:
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(lib().tq_timing_read(int(which), ctypes.byref(ms), ctypes.byref(n), int(bool(reset))), "tq_timing_read")
    return ms.value, n.value


class tq_server:
    """Continuous-batching server over a database (tq_serve_create / destroy).

    submit() takes host query codes (numpy uint32 / int32, nq x 2W) and returns
    a ticket; poll() / wait() return (ids, scores, stats) as numpy arrays once
    the request has finished, or None while it is pending."""

    def __init__(self, db: tq_db, budget_bytes: int = 0, max_slots: int = 0, max_k: int = 0, n_segments: int = 0,
                 max_request_nq: int = 0, tick_timeout_us: int = 0, engine: int = TQ_ENGINE_AUTO):
        import numpy as np  # noqa: F401
        self.db = db
        cfg = tq_serve_cfg()
        cfg.budget_bytes, cfg.max_slots, cfg.max_k = int(budget_bytes), int(max_slots), int(max_k)
        cfg.n_segments, cfg.max_request_nq = int(n_segments), int(max_request_nq)
        cfg.tick_timeout_us = int(tick_timeout_us)
        cfg.engine = int(engine)
        self._h = ctypes.c_void_p()
        self._k = {}
        with torch.cuda.device(db.device):
            _check(lib().tq_serve_create(db.handle, ctypes.byref(cfg), ctypes.byref(self._h)), "tq_serve_create")

    def submit(self, qcodes, k: int) -> int:
        import numpy as np
        q = np.ascontiguousarray(qcodes).view(np.uint32)
        if q.ndim != 2 or q.shape[1] != 2 * self.db.W:
            raise ValueError("qcodes must be nq x 2W")
        t = ctypes.c_uint64()
        _check(lib().tq_serve_submit(self._h, q.ctypes.data, q.shape[0], int(k), ctypes.byref(t)), "tq_serve_submit")
        self._k[t.value] = (q.shape[0], int(k))
        return t.value

    def _collect(self, fn, ticket, *extra):
        import numpy as np
        nq, k = self._k.get(ticket, (1, 1))
        ids = np.empty((nq, k), np.int32)
        sc = np.empty((nq, k), np.int32)
        st = tq_req_stats()
        rc = fn(self._h, ctypes.c_uint64(ticket), *extra, ids.ctypes.data, sc.ctypes.data, ctypes.byref(st))
        if rc == TQ_ERR_AGAIN:
            return None
        _check(rc, fn.__name__)
        self._k.pop(ticket, None)
        return ids, sc, st

    def poll(self, ticket: int):
        return self._collect(lib().tq_serve_poll, ticket)

    def wait(self, ticket: int, timeout_ms: int = -1):
        return self._collect(lib().tq_serve_wait, ticket, ctypes.c_int(int(timeout_ms)))

    def cancel(self, ticket: int) -> None:
        _check(lib().tq_serve_cancel(self._h, ctypes.c_uint64(ticket)), "tq_serve_cancel")
        self._k.pop(ticket, None)

    def stats(self):
        a, b, c, d = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().tq_serve_stats(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)),
               "tq_serve_stats")
        return dict(submitted=a.value, completed=b.value, ticks=c.value, bytes_in_use=d.value)

    def destroy(self) -> None:
        if self._h:
            _check(lib().tq_serve_destroy(self._h), "tq_serve_destroy")
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def tq_serve_create(db: tq_db, **cfg) -> tq_server:
    return tq_server(db, **cfg)
