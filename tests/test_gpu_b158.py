"""b1.58 quantisation on the GPU (tq_encode_b158) against the oracle, bit for
bit, and searches over a database of such codes (x = 0: any number of
non-zeros) on every path against the oracle's exhaustive kNN."""
import sys

import numpy as np
import pytest
import torch

import oracle
from tests.libtq import ensure_built

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stderr.flush()


@pytest.fixture(scope="module")
def tq():
    return ensure_built()


@pytest.fixture(scope="module")
def o():
    return oracle.default()


def gpu_b158(tq, X):
    codes = tq.tq_encode_b158(torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda())
    tq.tq_sync()
    return codes.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("d", [1, 2, 31, 33, 64, 100, 129, 384, 500, 768, 1000, 1024])
def test_b158_encode_vs_oracle(tq, o, d):
    rng = np.random.default_rng(500 + d)
    X = rng.standard_normal((3000, d)).astype(np.float32)
    X[1] = 0.0
    X[2] = np.round(X[2] * 2) / 2  # many exact ties of |u| / gamma
    X[3] *= np.float32(1e-30)
    X[4] *= np.float32(1e30)
    X[5, : d // 2] = 0.0
    say(f"b1.58 encode d={d}")
    assert np.array_equal(gpu_b158(tq, X), o.pack(o.encode_b158(X)))


def test_b158_worked_rows(tq, o):
    X = np.array([[0.2, -0.5, 1.3, 0.0], [1.0, 3.0, -1.0, -3.0], [0.0, 0.0, 0.0, 0.0], [2.0, -2.0, 2.0, -2.0]],
                 dtype=np.float32)
    say("b1.58 worked rows")
    assert np.array_equal(o.unpack(gpu_b158(tq, X), 4),
                          np.array([[0, -1, 1, 0], [0, 1, 0, -1], [0, 0, 0, 0], [1, -1, 1, -1]], dtype=np.int8))


def test_b158_nonfinite(tq, o):
    X = np.ones((4, 50), dtype=np.float32)
    X[2, 7] = np.inf
    say("b1.58 with an infinite element")
    codes = tq.tq_encode_b158(torch.from_numpy(X).cuda())
    with pytest.raises(tq.TQError):
        tq.tq_sync()
    c = codes.cpu().numpy().view(np.uint32)
    assert np.all(c[2] == 0) and np.array_equal(c[[0, 1, 3]], o.pack(o.encode_b158(X[[0, 1, 3]])))


@pytest.mark.parametrize("d", [96, 384, 1024])
def test_b158_database_search(tq, o, d):
    """x = 0 databases: every path returns the oracle's exhaustive kNN over
    the b1.58 vectors (Delta = their ternary scalar product)."""
    rng = np.random.default_rng(600 + d)
    X = rng.standard_normal((5000, d)).astype(np.float32)
    Q = rng.standard_normal((70, d)).astype(np.float32)
    V, VQ = o.encode_b158(X), o.encode_b158(Q)
    codes = torch.from_numpy(o.pack(V).view(np.int32).copy()).cuda()
    db = tq.tq_db_create(codes, d, 0)
    qc = torch.from_numpy(o.pack(VQ).view(np.int32).copy()).cuda()
    for k in (1, 10, 100):
        ei, es = o.knn(VQ, V, k)
        for path, engine in ((tq.TQ_PATH_PLAIN, 0), (tq.TQ_PATH_BATCHED, tq.TQ_ENGINE_POPCOUNT),
                             (tq.TQ_PATH_BATCHED, tq.TQ_ENGINE_MATRIX)):
            say(f"b1.58 database d={d} k={k} path={path} engine={engine}")
            ids, sc = tq.tq_search_knn(db, qc, k, path=path, engine=engine)
            torch.cuda.synchronize()
            assert np.array_equal(ids.cpu().numpy(), ei) and np.array_equal(sc.cpu().numpy(), es)
    db.destroy()


def test_x0_database_still_checks_planes(tq, o):
    rng = np.random.default_rng(9)
    C = o.pack(o.encode_b158(rng.standard_normal((10, 100)).astype(np.float32)))
    bad = C.copy()
    bad[3, 0] |= np.uint32(1)
    bad[3, 4] |= np.uint32(1)  # coordinate 0 in both planes
    say("x = 0 database rejects a coordinate in both planes")
    with pytest.raises(tq.TQError):
        tq.tq_db_create(torch.from_numpy(bad.view(np.int32).copy()).cuda(), 100, 0)
    bad = C.copy()
    bad[5, 3] |= np.uint32(1 << 30)  # padding bit
    with pytest.raises(tq.TQError):
        tq.tq_db_create(torch.from_numpy(bad.view(np.int32).copy()).cuda(), 100, 0)


# ---------------------------------------------------------------------------
# the l2 order (TQ_METRIC_L2): codes of varying non-zero counts ranked by the
# euclidean distance between the ternary vectors, score 2 Delta - nnz(v)
# ---------------------------------------------------------------------------

def b158_set(o, rng, n, nq, d, dup=0):
    """b1.58 codes of Gaussian rows; with dup > 0 the database repeats dup
    distinct codes (many equal distances) and the first queries are members."""
    if dup:
        base = o.encode_b158(rng.standard_normal((dup, d)).astype(np.float32))
        V = base[rng.integers(0, dup, size=n)]
        VQ = np.concatenate([base[:nq // 2], o.encode_b158(rng.standard_normal((nq - nq // 2, d)).astype(np.float32))])
    else:
        V = o.encode_b158(rng.standard_normal((n, d)).astype(np.float32))
        VQ = o.encode_b158(rng.standard_normal((nq, d)).astype(np.float32))
    return V, VQ


def dev(o, V):
    return torch.from_numpy(o.pack(V).view(np.int32).copy()).cuda()


@pytest.mark.parametrize("d,n,dup", [(96, 5037, 0), (384, 5000, 40), (1000, 3001, 0), (1024, 4160, 25)])
def test_l2_search_vs_oracle(tq, o, d, n, dup):
    rng = np.random.default_rng(700 + d)
    V, VQ = b158_set(o, rng, n, 40, d, dup)
    db = tq.tq_db_create(dev(o, V), d, 0)
    qc = dev(o, VQ)
    for k in (1, 10, 100, 200, 512):
        ei, es = o.knn_l2(VQ, V, k)
        runs = [(tq.TQ_PATH_PLAIN, 0, 0), (tq.TQ_PATH_PLAIN, 0, 7), (tq.TQ_PATH_AUTO, 0, 0),
                (tq.TQ_PATH_BATCHED, 0, 0)]
        runs += [(tq.TQ_PATH_BATCHED, q, 0) for q in (2, 4, 8, 16) if q <= (16 if k <= 128 else 8 if k <= 256 else 4)]
        for path, qtile, grid in runs:
            say(f"l2 d={d} n={n} dup={dup} k={k} path={path} qtile={qtile} grid={grid}")
            ids, sc = tq.tq_search_knn(db, qc, k, path=path, qtile=qtile, grid=grid, metric=tq.TQ_METRIC_L2)
            torch.cuda.synchronize()
            assert np.array_equal(sc.cpu().numpy(), es) and np.array_equal(ids.cpu().numpy(), ei), \
                (k, path, qtile, grid)
    db.destroy()


def test_l2_sample_floor_and_bound(tq, o):
    """2 100 tiles of b1.58 codes with many duplicates: the plain path's
    sample pass (k = 200, 512) and the popcount engine's cross-part bound
    (k > 128) both prune by l2 keys."""
    rng = np.random.default_rng(77)
    n, d = 2100 * 64 + 9, 64
    V, VQ = b158_set(o, rng, n, 12, d, dup=3000)
    db = tq.tq_db_create(dev(o, V), d, 0)
    qc = dev(o, VQ)
    for k in (100, 200, 512):
        ei, es = o.knn_l2(VQ, V, k)
        for path in (tq.TQ_PATH_PLAIN, tq.TQ_PATH_BATCHED):
            say(f"l2 sample floor / bound n={n} k={k} path={path}")
            ids, sc = tq.tq_search_knn(db, qc, k, path=path, metric=tq.TQ_METRIC_L2)
            torch.cuda.synchronize()
            assert np.array_equal(sc.cpu().numpy(), es) and np.array_equal(ids.cpu().numpy(), ei), (k, path)
    db.destroy()


def test_l2_on_evp_codes_is_delta_order(tq, o):
    """{x,d} codes all have x non-zeros: the l2 order is the Delta order and
    the score 2 Delta - x."""
    rng = np.random.default_rng(78)
    d, x = 256, 85
    V = o.encode(rng.standard_normal((3000, d)).astype(np.float32), x)
    VQ = o.encode(rng.standard_normal((20, d)).astype(np.float32), x)
    db = tq.tq_db_create(dev(o, V), d, x)
    qc = dev(o, VQ)
    say("l2 on EVP codes")
    i2, s2 = tq.tq_search_knn(db, qc, 50, metric=tq.TQ_METRIC_L2)
    i1, s1 = tq.tq_search_knn(db, qc, 50)
    torch.cuda.synchronize()
    assert torch.equal(i1, i2) and torch.equal(2 * s1 - x, s2)
    db.destroy()


def test_l2_noalloc_and_rejections(tq, o):
    rng = np.random.default_rng(79)
    d = 128
    V, VQ = b158_set(o, rng, 2000, 6, d)
    db = tq.tq_db_create(dev(o, V), d, 0)
    qc = dev(o, VQ)
    ei, es = o.knn_l2(VQ, V, 30)
    say("l2 through the no-allocation entry point")
    ids = torch.empty((6, 30), dtype=torch.int32, device="cuda")
    sc = torch.empty((6, 30), dtype=torch.int32, device="cuda")
    tq.tq_search_knn_noalloc(db, qc, 30, ids, sc, metric=tq.TQ_METRIC_L2)
    torch.cuda.synchronize()
    assert np.array_equal(sc.cpu().numpy(), es) and np.array_equal(ids.cpu().numpy(), ei)
    say("l2 rejections: matrix engine, index-list engine, unknown metric")
    for kw in (dict(path=tq.TQ_PATH_BATCHED, engine=tq.TQ_ENGINE_MATRIX, metric=tq.TQ_METRIC_L2),
               dict(path=tq.TQ_PATH_BATCHED, qtile=64, metric=tq.TQ_METRIC_L2),
               dict(engine=tq.TQ_ENGINE_SPARSE, metric=tq.TQ_METRIC_L2),
               dict(metric=7)):
        with pytest.raises(tq.TQError) as e:
            tq.tq_search_knn(db, qc, 10, **kw)
        assert e.value.status == tq.TQ_ERR_INVALID, kw
    db.destroy()
