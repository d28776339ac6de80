"""CPU oracle for the ternary EVP search path (arXiv 2506.00528).

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the GPU
library and never imports it.

The arithmetic lives in ``oracle.c`` (plain C + OpenMP, built with gcc); this
module only marshals numpy arrays (encode, pack, unpack, delta, knn, the
refinement of proxy candidates with the float vectors, rerank, and the
masked-addition search of float queries against ternary vectors,
masked_knn, the b1.58 quantisation of Sec. 4.3, encode_b158, and the search
by euclidean distance between ternary vectors that codes of varying non-zero
counts need, knn_l2), plus a few
pure-Python definitions:

* ``default_x(d)``     -- the x maximising the vertex count C(d,x)*2^x
                          (Sec. 5.1.1), by brute force over all x with exact
                          big-integer arithmetic;
* ``vertex_count(d,x)``-- C(d,x)*2^x, the number of {x,d} EVP vertices
                          (Sec. 2.3).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from .build import build as _build, library_path

_lib = None

EINVAL = -1
ENONFINITE = -2
ENOMEM = -3


class OracleError(RuntimeError):
    def __init__(self, rc: int, what: str):
        super().__init__(f"oracle {what} failed with status {rc}")
        self.rc = rc


def load(path: str | None = None):
    """Load (building first if needed) the oracle shared library."""
    global _lib
    if path is None and _lib is not None:
        return _lib
    p = path or library_path()
    if path is None and not os.path.exists(p):
        _build()
    lib = ctypes.CDLL(p)
    i64, i32, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
    lib.oracle_words_per_plane.argtypes = [i32]
    lib.oracle_encode.argtypes = [vp, i64, i32, i32, vp]
    lib.oracle_pack.argtypes = [vp, i64, i32, vp]
    lib.oracle_unpack.argtypes = [vp, i64, i32, vp]
    lib.oracle_delta.argtypes = [vp, i64, vp, i64, i32, vp]
    lib.oracle_knn.argtypes = [vp, i64, vp, i64, i32, i32, vp, vp]
    lib.oracle_knn_l2.argtypes = [vp, i64, vp, i64, i32, i32, vp, vp]
    lib.oracle_rerank.argtypes = [vp, i64, i32, vp, i64, vp, i32, i32, vp, vp]
    lib.oracle_masked_knn.argtypes = [vp, i64, vp, i64, i32, i32, vp, vp, vp]
    lib.oracle_encode_b158.argtypes = [vp, i64, i32, vp]
    lib.oracle_num_threads.restype = i32
    lib.oracle_set_num_threads.argtypes = [i32]
    if path is None:
        _lib = lib
    return lib


class Oracle:
    """numpy front end over one build of oracle.c (the normal one by default;
    the tests also build deliberately broken copies to prove the pins bite)."""

    def __init__(self, lib=None):
        self.lib = lib if lib is not None else load()

    # -- sizes ------------------------------------------------------------
    def words_per_plane(self, d: int) -> int:
        return int(self.lib.oracle_words_per_plane(int(d)))

    def num_threads(self) -> int:
        return int(self.lib.oracle_num_threads())

    def set_num_threads(self, t: int) -> None:
        self.lib.oracle_set_num_threads(int(t))

    # -- encode (Sec. 2.4) ------------------------------------------------
    def encode(self, X: np.ndarray, x: int) -> np.ndarray:
        X = np.ascontiguousarray(X, dtype=np.float32)
        if X.ndim == 1:
            X = X[None, :]
        n, d = X.shape
        V = np.empty((n, d), dtype=np.int8)
        rc = self.lib.oracle_encode(X.ctypes.data, n, d, int(x), V.ctypes.data)
        if rc != 0:
            raise OracleError(rc, "encode")
        return V

    # -- b1.58 quantisation (Sec. 4.3), per embedding --------------------
    def encode_b158(self, X: np.ndarray) -> np.ndarray:
        X = np.ascontiguousarray(X, dtype=np.float32)
        if X.ndim == 1:
            X = X[None, :]
        n, d = X.shape
        V = np.empty((n, d), dtype=np.int8)
        rc = self.lib.oracle_encode_b158(X.ctypes.data, n, d, V.ctypes.data)
        if rc != 0:
            raise OracleError(rc, "encode_b158")
        return V

    # -- bit planes (Sec. 5.1.2, Table 3) ---------------------------------
    def pack(self, V: np.ndarray) -> np.ndarray:
        V = np.ascontiguousarray(V, dtype=np.int8)
        if V.ndim == 1:
            V = V[None, :]
        n, d = V.shape
        W = self.words_per_plane(d)
        C = np.empty((n, 2 * W), dtype=np.uint32)
        rc = self.lib.oracle_pack(V.ctypes.data, n, d, C.ctypes.data)
        if rc != 0:
            raise OracleError(rc, "pack")
        return C

    def unpack(self, C: np.ndarray, d: int) -> np.ndarray:
        C = np.ascontiguousarray(C, dtype=np.uint32)
        if C.ndim == 1:
            C = C[None, :]
        n = C.shape[0]
        if C.shape[1] != 2 * self.words_per_plane(d):
            raise ValueError("code width does not match d")
        V = np.empty((n, d), dtype=np.int8)
        rc = self.lib.oracle_unpack(C.ctypes.data, n, int(d), V.ctypes.data)
        if rc != 0:
            raise OracleError(rc, "unpack")
        return V

    # -- Delta = b2sp (Sec. 5.1.2) ----------------------------------------
    def delta(self, Q: np.ndarray, V: np.ndarray) -> np.ndarray:
        Q = np.ascontiguousarray(Q, dtype=np.int8)
        V = np.ascontiguousarray(V, dtype=np.int8)
        if Q.ndim == 1:
            Q = Q[None, :]
        if V.ndim == 1:
            V = V[None, :]
        if Q.shape[1] != V.shape[1]:
            raise ValueError("dimension mismatch")
        D = np.empty((Q.shape[0], V.shape[0]), dtype=np.int32)
        rc = self.lib.oracle_delta(Q.ctypes.data, Q.shape[0], V.ctypes.data, V.shape[0],
                                   Q.shape[1], D.ctypes.data)
        if rc != 0:
            raise OracleError(rc, "delta")
        return D

    # -- exhaustive kNN in the proxy space ----------------------------------
    def knn(self, Q: np.ndarray, V: np.ndarray, k: int):
        Q = np.ascontiguousarray(Q, dtype=np.int8)
        V = np.ascontiguousarray(V, dtype=np.int8)
        if Q.ndim == 1:
            Q = Q[None, :]
        if Q.shape[1] != V.shape[1]:
            raise ValueError("dimension mismatch")
        nq = Q.shape[0]
        ids = np.empty((nq, k), dtype=np.int32)
        scores = np.empty((nq, k), dtype=np.int32)
        rc = self.lib.oracle_knn(Q.ctypes.data, nq, V.ctypes.data, V.shape[0], Q.shape[1],
                                 int(k), ids.ctypes.data, scores.ctypes.data)
        if rc != 0:
            raise OracleError(rc, "knn")
        return ids, scores

    # -- exhaustive kNN by euclidean distance of ternary vectors -----------
    def knn_l2(self, Q: np.ndarray, V: np.ndarray, k: int):
        """Nearest by squared l2 distance between the ternary vectors (for
        codes of varying non-zero counts, e.g. b1.58), ties to the lower id;
        scores are nnz(q) - distance (= 2 Delta - nnz(v))."""
        Q = np.ascontiguousarray(Q, dtype=np.int8)
        V = np.ascontiguousarray(V, dtype=np.int8)
        if Q.ndim == 1:
            Q = Q[None, :]
        if Q.shape[1] != V.shape[1]:
            raise ValueError("dimension mismatch")
        nq = Q.shape[0]
        ids = np.empty((nq, k), dtype=np.int32)
        scores = np.empty((nq, k), dtype=np.int32)
        rc = self.lib.oracle_knn_l2(Q.ctypes.data, nq, V.ctypes.data, V.shape[0], Q.shape[1],
                                    int(k), ids.ctypes.data, scores.ctypes.data)
        if rc != 0:
            raise OracleError(rc, "knn_l2")
        return ids, scores

    # -- refinement of proxy candidates (Sec. 5.3 k@n) ---------------------
    def rerank(self, X: np.ndarray, Q: np.ndarray, cand: np.ndarray, k: int):
        """The k best of each query's candidate ids by the double-precision
        scalar product of the float vectors (ties: lower id); ids outside
        [0, n) are skipped, missing results are id -1, score -inf."""
        X = np.ascontiguousarray(X, dtype=np.float32)
        Q = np.ascontiguousarray(Q, dtype=np.float32)
        cand = np.ascontiguousarray(cand, dtype=np.int32)
        if Q.ndim == 1:
            Q = Q[None, :]
        if cand.ndim == 1:
            cand = cand[None, :]
        if Q.shape[1] != X.shape[1] or cand.shape[0] != Q.shape[0]:
            raise ValueError("shape mismatch")
        nq, ncand = cand.shape
        ids = np.empty((nq, k), dtype=np.int32)
        scores = np.empty((nq, k), dtype=np.float64)
        rc = self.lib.oracle_rerank(X.ctypes.data, X.shape[0], X.shape[1], Q.ctypes.data, nq, cand.ctypes.data,
                                    ncand, int(k), ids.ctypes.data, scores.ctypes.data)
        if rc != 0:
            raise OracleError(rc, "rerank")
        return ids, scores


    # -- masked addition: float query vs ternary database (Sec. 5.1.2, 6) --
    def masked_knn(self, Q: np.ndarray, V: np.ndarray, k: int):
        """Top-k of each float query against ternary vectors V by masked
        addition: ids, float scores (the double sums rounded once) and the
        double sums themselves."""
        Q = np.ascontiguousarray(Q, dtype=np.float32)
        V = np.ascontiguousarray(V, dtype=np.int8)
        if Q.ndim == 1:
            Q = Q[None, :]
        if Q.shape[1] != V.shape[1]:
            raise ValueError("dimension mismatch")
        nq = Q.shape[0]
        ids = np.empty((nq, k), dtype=np.int32)
        scores = np.empty((nq, k), dtype=np.float32)
        exact = np.empty((nq, k), dtype=np.float64)
        rc = self.lib.oracle_masked_knn(Q.ctypes.data, nq, V.ctypes.data, V.shape[0], Q.shape[1], int(k),
                                        ids.ctypes.data, scores.ctypes.data, exact.ctypes.data)
        if rc != 0:
            raise OracleError(rc, "masked_knn")
        return ids, scores, exact


# -- pure-Python definitions ------------------------------------------------

def vertex_count(d: int, x: int) -> int:
    """Number of {x,d} EVP vertices: choose the x non-zero places, then a sign
    for each (Sec. 2.3)."""
    return math.comb(d, x) * 2 ** x


def default_x(d: int) -> int:
    """The x in 1..d with the most vertices (Sec. 5.1.1); on equal counts the
    smaller x (the reading that reproduces the paper's {333,500})."""
    best_x, best = 1, vertex_count(d, 1)
    for x in range(2, d + 1):
        c = vertex_count(d, x)
        if c > best:
            best_x, best = x, c
    return best_x


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def encode(X, x):
    return default().encode(X, x)


def pack(V):
    return default().pack(V)


def unpack(C, d):
    return default().unpack(C, d)


def delta(Q, V):
    return default().delta(Q, V)


def knn(Q, V, k):
    return default().knn(Q, V, k)


def knn_l2(Q, V, k):
    return default().knn_l2(Q, V, k)


def rerank(X, Q, cand, k):
    return default().rerank(X, Q, cand, k)


def masked_knn(Q, V, k):
    return default().masked_knn(Q, V, k)


def encode_b158(X):
    return default().encode_b158(X)
