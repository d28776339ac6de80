"""Refinement of proxy candidates with the float vectors (tq_rerank) against
the oracle.  Scores are double-precision scalar products summed in a
different order on each side, so they are compared to 1e-12 (relative to the
product of the norms); ids must match wherever the oracle's neighbouring
scores are further apart than that, and near-equal runs must hold the same
ids.  Exact ties (equal rows) must go to the lower id on both sides."""
import sys

import numpy as np
import pytest
import torch

import oracle
from tests.libtq import ensure_built
from workloads import datagen

pytestmark = pytest.mark.gpu

TOL = 1e-12


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stderr.flush()


@pytest.fixture(scope="module")
def tq():
    return ensure_built()


@pytest.fixture(scope="module")
def o():
    return oracle.default()


def compare(gi, gs, ei, es, scale):
    assert gi.shape == ei.shape and gs.shape == es.shape
    assert np.array_equal(np.isneginf(gs), np.isneginf(es))
    fin = ~np.isneginf(es)
    assert np.all(np.abs(gs[fin] - es[fin]) <= TOL * scale), np.max(np.abs(gs[fin] - es[fin]))
    assert np.array_equal(gi[~fin], ei[~fin])
    k = ei.shape[1]
    for q in range(ei.shape[0]):
        kf = int(np.sum(fin[q]))  # the empty (-inf) slots follow and are checked above
        j = 0
        while j < kf:  # runs of oracle scores within the tolerance of each other
            e = j + 1
            while e < kf and es[q, e - 1] - es[q, e] <= 2 * TOL * scale:
                e += 1
            if e - j == 1:
                assert gi[q, j] == ei[q, j], (q, j)
            else:
                assert set(gi[q, j:e]) == set(ei[q, j:e]) or e == k, (q, j, e)
            j = e


def run(tq, X, Q, cand, k):
    ids, sc = tq.tq_rerank(torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda(),
                           torch.from_numpy(cand).cuda(), k)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), sc.cpu().numpy()


@pytest.mark.parametrize("d", [1, 33, 64, 100, 384, 768, 1000, 1024])
@pytest.mark.parametrize("ncand,k", [(1, 1), (10, 10), (100, 10), (512, 100), (1000, 37), (1024, 1024)])
def test_rerank_vs_oracle(tq, o, d, ncand, k):
    rng = np.random.default_rng(d * 7 + ncand)
    n, nq = 3000, 9
    X = rng.standard_normal((n, d)).astype(np.float32)
    Q = rng.standard_normal((nq, d)).astype(np.float32)
    cand = np.stack([rng.permutation(n)[:ncand] for _ in range(nq)]).astype(np.int32)
    say(f"rerank d={d} ncand={ncand} k={k}")
    gi, gs = run(tq, X, Q, cand, k)
    ei, es = o.rerank(X, Q, cand, k)
    scale = float(np.max(np.linalg.norm(Q, axis=1)) * np.max(np.linalg.norm(X, axis=1)))
    compare(gi, gs, ei, es, scale)


def test_rerank_ties_invalid_and_short(tq, o):
    rng = np.random.default_rng(5)
    n, d, nq, ncand, k = 500, 96, 6, 40, 20
    X = rng.standard_normal((n, d)).astype(np.float32)
    X[11] = X[4]
    X[12] = X[4]
    Q = rng.standard_normal((nq, d)).astype(np.float32)
    Q[0] = X[4]
    cand = np.stack([rng.permutation(n)[:ncand] for _ in range(nq)]).astype(np.int32)
    cand[:, :3] = [12, 4, 11]
    cand[1, 5:] = -1  # query 1: only 5 candidates, so 15 empty results
    cand[2, 5] = n  # outside [0, n): ignored
    cand[2, 6] = 2 ** 31 - 1
    say("rerank ties / invalid ids / short lists")
    gi, gs = run(tq, X, Q, cand, k)
    ei, es = o.rerank(X, Q, cand, k)
    assert gi[0, :3].tolist() == [4, 11, 12] and ei[0, :3].tolist() == [4, 11, 12]
    assert np.all(gi[1, 5:] == -1) and np.all(np.isneginf(gs[1, 5:]))
    scale = float(np.max(np.linalg.norm(Q, axis=1)) * np.max(np.linalg.norm(X, axis=1)))
    compare(gi, gs, ei, es, scale)


def test_rerank_of_proxy_candidates_small_workload(tq, o):
    """The path end to end on the small workload: Delta top-100 candidates on
    the GPU, refined on the GPU, against the oracle refining the oracle's own
    top-100; and refining every id equals the exact ground truth."""
    w = datagen.WORKLOADS["small"]
    X = datagen.rows("small", datagen.DB, 0, w["n"]).numpy()
    Q = datagen.rows("small", datagen.QUERIES, 0, w["nq"]).numpy()
    V, VQ = o.encode(X, w["x"]), o.encode(Q, w["x"])
    db = tq.tq_db_create(torch.from_numpy(o.pack(V).view(np.int32).copy()).cuda(), w["d"], w["x"])
    say("rerank small workload: GPU Delta top-100 -> GPU refine")
    cand_g, _ = tq.tq_search_knn(db, torch.from_numpy(o.pack(VQ).view(np.int32).copy()).cuda(), 100)
    torch.cuda.synchronize()
    cand_o, _ = o.knn(VQ, V, 100)
    assert np.array_equal(cand_g.cpu().numpy(), cand_o)
    gi, gs = run(tq, X, Q, cand_o, 10)
    ei, es = o.rerank(X, Q, cand_o, 10)
    compare(gi, gs, ei, es, 1.0)
    db.destroy()
    allc = np.tile(np.arange(1000, dtype=np.int32), (w["nq"], 1))
    gi, gs = run(tq, X[:1000], Q, allc, 10)
    exact = np.argsort(-(Q.astype(np.float64) @ X[:1000].astype(np.float64).T), axis=1, kind="stable")[:, :10]
    assert np.array_equal(gi, exact)


def test_rerank_rejects(tq):
    X = torch.zeros((10, 8), dtype=torch.float32, device="cuda")
    Q = torch.zeros((2, 8), dtype=torch.float32, device="cuda")
    c = torch.zeros((2, 4), dtype=torch.int32, device="cuda")
    with pytest.raises(tq.TQError):
        tq.tq_rerank(X, Q, c, 5)
    with pytest.raises(tq.TQError):
        tq.tq_rerank(X, Q, torch.zeros((2, 1025), dtype=torch.int32, device="cuda"), 5)
