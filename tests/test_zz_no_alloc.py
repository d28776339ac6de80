"""tq_search_knn_noalloc (the plain search with the library's fixed scratch
array, for callers that cannot allocate) gives exactly tq_search_knn's plain
results, on two calls in a row with the second one smaller, and rejects what
cannot run without allocating before anything is queued."""
import sys

import pytest
import torch

from tests.libtq import ensure_built
from workloads import datagen

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stderr.flush()


@pytest.fixture(scope="module")
def tq():
    return ensure_built()


@pytest.fixture(scope="module")
def setup(tq):
    # 2 049 tiles of d = 1024 codes: more than the sample pass's minimum, so
    # the sample rows share the array too, and a ragged last tile
    n, d, x = 2048 * 64 + 37, 1024, 256
    dev = torch.device("cuda", 0)
    X = datagen.rows("large", datagen.DB, 0, n, dev)
    codes = tq.tq_encode(X, x)
    del X
    Q = datagen.rows("large", datagen.QUERIES, 0, 40, dev)
    qcodes = tq.tq_encode(Q, x)
    tq.tq_sync()
    db = tq.tq_db_create(codes, d, x)
    del codes
    yield db, qcodes
    db.destroy()


def run_noalloc(tq, db, qcodes, k, **kw):
    nq = qcodes.shape[0]
    ids = torch.full((nq, k), -7, dtype=torch.int32, device=qcodes.device)
    scores = torch.full((nq, k), -7, dtype=torch.int32, device=qcodes.device)
    tq.tq_search_knn_noalloc(db, qcodes, k, ids, scores, **kw)
    torch.cuda.synchronize()
    return ids, scores


def test_noalloc_equals_plain_two_calls(tq, setup):
    db, qcodes = setup
    # first call: 40 queries at k = 512 (2 MiB of lists per query, so the
    # queries run in several rounds through the array); second call smaller
    for nq, k in ((40, 512), (5, 10)):
        say(f"noalloc vs plain nq={nq} k={k}")
        ids, scores = run_noalloc(tq, db, qcodes[:nq], k)
        ei, es = tq.tq_search_knn(db, qcodes[:nq], k, path=tq.TQ_PATH_PLAIN)
        torch.cuda.synchronize()
        assert torch.equal(ids, ei) and torch.equal(scores, es), (nq, k)


def test_noalloc_engines_and_grids(tq, setup):
    db, qcodes = setup
    for k, grid, engine in ((100, 0, tq.TQ_ENGINE_POPCOUNT), (64, 300, tq.TQ_ENGINE_AUTO), (1, 2049, tq.TQ_ENGINE_AUTO)):
        say(f"noalloc k={k} grid={grid} engine={engine}")
        ids, scores = run_noalloc(tq, db, qcodes[:9], k, grid=grid, engine=engine)
        ei, es = tq.tq_search_knn(db, qcodes[:9], k, path=tq.TQ_PATH_PLAIN, grid=grid)
        torch.cuda.synchronize()
        assert torch.equal(ids, ei) and torch.equal(scores, es), (k, grid, engine)


def test_noalloc_rejects_before_queueing(tq, setup):
    db, qcodes = setup
    nq, k = 3, 512
    bad = (
        dict(grid=8192),  # 8192 x 512 keys = 32 MiB per query, more than the array
        dict(check_queries=True),
        dict(path=tq.TQ_PATH_BATCHED),
        dict(engine=tq.TQ_ENGINE_MATRIX),
        dict(engine=tq.TQ_ENGINE_SPARSE),  # x = 256 of d = 1024: no index-list copy
    )
    for kw in bad:
        ids = torch.full((nq, k), -7, dtype=torch.int32, device=qcodes.device)
        scores = torch.full((nq, k), -7, dtype=torch.int32, device=qcodes.device)
        with pytest.raises(tq.TQError) as e:
            tq.tq_search_knn_noalloc(db, qcodes[:nq], k, ids, scores, **kw)
        assert e.value.status == tq.TQ_ERR_INVALID, kw
        if "grid" in kw:
            assert "scratch" in str(e.value), str(e.value)
        torch.cuda.synchronize()
        assert bool((ids == -7).all()) and bool((scores == -7).all()), kw
