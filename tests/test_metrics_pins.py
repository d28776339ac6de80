"""The recall ground truth (workloads/metrics.py) against brute force.

Sec. 5.3 measures k@n recall: how many of a query's k true nearest neighbours
(nearest in the original space) are among the first n results of the proxy
search.  The ground truth here is the top-k by the float64 scalar product of
the float32 vectors (cosine on l2-normalised vectors, Sec. 1.1), ties to the
lower id, accumulated one database chunk at a time.  Every recall figure the
benchmark reports rests on it, so it is pinned against things it does not
compute itself:

* scores: each product of two float32 values is exact in float64, and
  ``math.fsum`` rounds their sum correctly once, so the brute-force score is
  the exactly rounded scalar product; ranking: ``np.lexsort`` on (-score, id);
* exact ties: queries and rows with small dyadic coordinates have scalar
  products that every summation order computes exactly, and duplicate rows
  placed on both sides of chunk boundaries give equal scores that must go to
  the lower id;
* chunking: the rows arrive in uneven chunks (1, 7, 64, ... rows), so the
  running list must carry across every boundary;
* ``recall_at`` against hand-counted cases.

Three plausible mistakes (ties to the higher id, float32 accumulation, a
running list dropped between chunks) are planted in subclasses, and each must
fail the checks.
"""
import math

import numpy as np
import pytest
import torch

from workloads.metrics import ExactTopK, recall_at

CHUNKS = (1, 7, 64, 3, 100, 2, 77, 46)  # 300 rows


def brute_topk(Q: np.ndarray, X: np.ndarray, k: int):
    """Top-k of every query by the correctly rounded float64 scalar product."""
    Qd, Xd = Q.astype(np.float64), X.astype(np.float64)
    ids = np.arange(X.shape[0])
    out_i, out_s = [], []
    for q in Qd:
        s = np.array([math.fsum((q * x).tolist()) for x in Xd])
        order = np.lexsort((ids, -s))[:k]
        out_i.append(ids[order])
        out_s.append(s[order])
    return np.array(out_i), np.array(out_s)


def feed(cls, Q: np.ndarray, X: np.ndarray, k: int, chunks=CHUNKS):
    assert sum(chunks) == X.shape[0]
    gt = cls(torch.from_numpy(Q), k)
    r = 0
    for c in chunks:
        gt.add(torch.from_numpy(X[r:r + c]), r)
        r += c
    return gt.result()


def random_case(seed=1, nq=6, n=300, d=48):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d))
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    Q = rng.standard_normal((nq, d))
    Q /= np.linalg.norm(Q, axis=1, keepdims=True)
    return Q.astype(np.float32), X.astype(np.float32)


def tie_case(seed=2, nq=5, n=300, d=16):
    """Dyadic coordinates (multiples of 1/8 in [-1, 1]): every scalar product
    is exact in any order.  Rows are copied across chunk boundaries, so equal
    scores straddle chunks; each query also gets a group of equal best rows."""
    rng = np.random.default_rng(seed)
    X = rng.integers(-8, 9, size=(n, d)).astype(np.float32) / 8
    Q = rng.integers(-8, 9, size=(nq, d)).astype(np.float32) / 8
    bounds = np.cumsum(CHUNKS)[:-1]
    for b in bounds:  # the row after each boundary repeats a row before it
        X[b] = X[max(0, b - 3)]
    for qi in range(nq):  # five copies of a row equal to the query itself, spread out
        for j in range(5):
            X[(37 + 61 * j + 11 * qi) % n] = Q[qi]
    return Q, X


def check_exact_topk(cls):
    # random unit vectors: ids exactly, scores to the correctly rounded value
    Q, X = random_case()
    for k in (1, 10, 64):
        ei, es = brute_topk(Q, X, k)
        gi, gs = feed(cls, Q, X, k)
        assert np.array_equal(gi, ei), f"random case: ids differ at k={k}"
        assert np.allclose(gs, es, rtol=1e-13, atol=1e-15), f"random case: scores differ at k={k}"
    # exact ties across chunk boundaries: lower id first, every score exact
    Q, X = tie_case()
    for k in (1, 5, 12, 40):
        ei, es = brute_topk(Q, X, k)
        gi, gs = feed(cls, Q, X, k)
        assert np.array_equal(gs, es), f"tie case: scores differ at k={k}"
        assert np.array_equal(gi, ei), f"tie case: ids differ at k={k}"
    # one row per chunk and a single chunk give the same ids (the library
    # product may sum in another order per chunk shape, so scores to rounding)
    Q, X = random_case(seed=3, nq=3, n=40, d=20)
    a = feed(cls, Q, X, 8, chunks=(1,) * 40)
    b = feed(cls, Q, X, 8, chunks=(40,))
    assert np.array_equal(a[0], b[0]) and np.allclose(a[1], b[1], rtol=1e-13), "chunking changes the result"


class _TiesToHigherId(ExactTopK):
    def add(self, rows, first_id):
        s = self.q @ rows.to(dtype=torch.float64).T
        ids = torch.arange(first_id, first_id + rows.shape[0]).expand(s.shape[0], -1)
        cs, ci = torch.cat([self.scores, s], 1), torch.cat([self.ids, ids], 1)
        order = torch.sort(ci, dim=1, descending=True, stable=True).indices  # planted
        cs, ci = torch.gather(cs, 1, order), torch.gather(ci, 1, order)
        order = torch.sort(cs, dim=1, descending=True, stable=True).indices[:, : self.k]
        self.scores, self.ids = torch.gather(cs, 1, order), torch.gather(ci, 1, order)


class _Float32Accumulation(ExactTopK):
    def add(self, rows, first_id):
        q32 = self.q.to(torch.float32)
        s = (q32 @ rows.to(torch.float32).T).to(torch.float64)  # planted
        ids = torch.arange(first_id, first_id + rows.shape[0]).expand(s.shape[0], -1)
        cs, ci = torch.cat([self.scores, s], 1), torch.cat([self.ids, ids], 1)
        order = torch.sort(ci, dim=1, stable=True).indices
        cs, ci = torch.gather(cs, 1, order), torch.gather(ci, 1, order)
        order = torch.sort(cs, dim=1, descending=True, stable=True).indices[:, : self.k]
        self.scores, self.ids = torch.gather(cs, 1, order), torch.gather(ci, 1, order)


class _DropsRunningList(ExactTopK):
    def add(self, rows, first_id):
        s = self.q @ rows.to(dtype=torch.float64).T
        ids = torch.arange(first_id, first_id + rows.shape[0]).expand(s.shape[0], -1)
        # planted: the lists of earlier chunks are forgotten once a chunk fills k
        if s.shape[1] >= self.k:
            cs, ci = s, ids
        else:
            cs, ci = torch.cat([self.scores, s], 1), torch.cat([self.ids, ids], 1)
        order = torch.sort(ci, dim=1, stable=True).indices
        cs, ci = torch.gather(cs, 1, order), torch.gather(ci, 1, order)
        order = torch.sort(cs, dim=1, descending=True, stable=True).indices[:, : self.k]
        self.scores, self.ids = torch.gather(cs, 1, order), torch.gather(ci, 1, order)


def test_exact_topk_against_brute_force():
    check_exact_topk(ExactTopK)


@pytest.mark.parametrize("mutant", [_TiesToHigherId, _Float32Accumulation, _DropsRunningList],
                         ids=lambda c: c.__name__.strip("_"))
def test_planted_mistake_is_caught(mutant):
    with pytest.raises(AssertionError):
        check_exact_topk(mutant)


def test_recall_at_hand_counted():
    true_ids = np.array([[0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 90, 91],
                         [10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 92, 93]])
    # query 0: 3 of the true 10 among the first 10 found, 7 among the first 100
    f0 = [0, 50, 51, 52, 2, 53, 54, 9, 55, 56] + list(range(100, 190)) + [1, 3, 4, 5]
    f0[40], f0[41], f0[42], f0[43] = 1, 3, 4, 5
    # query 1: none among the first 10, all 10 among the first 100
    f1 = list(range(200, 210)) + [19, 18, 17, 16, 15, 14, 13, 12, 11, 10] + list(range(300, 384))
    found = np.array([f0[:104], f1[:104]])
    assert recall_at(true_ids, found, 10, 10) == pytest.approx((3 + 0) / 20)
    assert recall_at(true_ids, found, 10, 100) == pytest.approx((7 + 10) / 20)
    # k truncates the true list (90, 91, 92, 93 are not among the true 10)
    found2 = np.array([[90, 91] + [0] * 8, [92, 93] + [10] * 8])
    assert recall_at(true_ids, found2, 10, 10) == pytest.approx(2 / 20)
    assert recall_at(true_ids, found2, 12, 10) == pytest.approx((3 + 3) / 24)
    # 1@1 and a repeated id counts once
    assert recall_at(true_ids, np.array([[0, 0], [11, 10]]), 1, 1) == pytest.approx(0.5)
    assert recall_at(true_ids, np.array([[0, 0], [11, 10]]), 2, 2) == pytest.approx((1 + 2) / 4)
