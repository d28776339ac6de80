"""The index-list engine of the plain path (TQ_ENGINE_SPARSE: Delta gathered
at each database code's listed non-zeros, kept for 8x <= d) against the CPU
oracle, bit-exact: the same ids and Delta as the definition, including ragged
tails, padding entries (x not a multiple of 8), the widest list (x = 128 at
d = 1024), heavy ties and every top-k list depth."""
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


def dev_codes(c):
    return torch.from_numpy(np.ascontiguousarray(c).view(np.int32).copy()).cuda()


def make(o, rng, n, d, x, nq):
    V = o.encode(rng.standard_normal((n, d)).astype(np.float32), x)
    VQ = o.encode(rng.standard_normal((nq, d)).astype(np.float32), x)
    return V, VQ


def search(tq, db, CQ, k, **kw):
    ids, sc = tq.tq_search_knn(db, dev_codes(CQ), k, **kw)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), sc.cpu().numpy()


SPARSE_SHAPES = [(1, 8, 1), (63, 64, 8), (65, 100, 12), (1000, 384, 7), (4097, 384, 24), (10000, 384, 48),
                 (3001, 768, 96), (2500, 1024, 128), (777, 1000, 3)]


@pytest.mark.parametrize("n,d,x,k", [(n, d, x, k) for (n, d, x) in SPARSE_SHAPES for k in (1, 10, 100, 512) if k <= n])
def test_sparse_vs_oracle(tq, o, n, d, x, k):
    rng = np.random.default_rng(n * 7 + d * 3 + x)
    V, VQ = make(o, rng, n, d, x, 13)
    say(f"sparse n={n} d={d} x={x} k={k}")
    db = tq.tq_db_create(dev_codes(o.pack(V)), d, x)
    ids, sc = search(tq, db, o.pack(VQ), k, path=tq.TQ_PATH_PLAIN, engine=tq.TQ_ENGINE_SPARSE)
    ei, es = o.knn(VQ, V, k)
    assert np.array_equal(sc, es) and np.array_equal(ids, ei)
    db.destroy()


@pytest.mark.parametrize("grid", [1, 7, 512, 2048])
def test_sparse_grids(tq, o, grid):
    rng = np.random.default_rng(91)
    n, d, x, k = 20000, 512, 32, 10
    V, VQ = make(o, rng, n, d, x, 5)
    say(f"sparse grid={grid}")
    db = tq.tq_db_create(dev_codes(o.pack(V)), d, x)
    ids, sc = search(tq, db, o.pack(VQ), k, path=tq.TQ_PATH_PLAIN, engine=tq.TQ_ENGINE_SPARSE, grid=grid)
    ei, es = o.knn(VQ, V, k)
    assert np.array_equal(sc, es) and np.array_equal(ids, ei)
    db.destroy()


def test_sparse_heavy_ties(tq, o):
    """Six distinct vectors repeated 20000 times: every score ties thousands of
    times, so the order is decided by the ids alone."""
    rng = np.random.default_rng(24)
    d, x = 256, 16
    base = o.encode(rng.standard_normal((6, d)).astype(np.float32), x)
    V = base[rng.integers(0, 6, size=20000)]
    VQ = np.concatenate([base[:3], o.encode(rng.standard_normal((10, d)).astype(np.float32), x)])
    say("sparse heavy ties")
    db = tq.tq_db_create(dev_codes(o.pack(V)), d, x)
    for k in (1, 10, 100, 512):
        ids, sc = search(tq, db, o.pack(VQ), k, path=tq.TQ_PATH_PLAIN, engine=tq.TQ_ENGINE_SPARSE)
        ei, es = o.knn(VQ, V, k)
        assert np.array_equal(sc, es) and np.array_equal(ids, ei), k
    db.destroy()


def test_sparse_same_as_bit_planes(tq, o):
    """Automatic choice (16x <= d takes the index list), the forced index list
    and the bit-plane scan give the same bits; every query is also in the
    database, so its own id comes first with Delta = x."""
    rng = np.random.default_rng(25)
    n, d, x, k = 30000, 1024, 32, 50
    V, _ = make(o, rng, n, d, x, 1)
    qi = rng.choice(n, size=9, replace=False)
    qi.sort()
    CQ = o.pack(V[qi])
    say("sparse vs bit planes, d=1024 x=32")
    db = tq.tq_db_create(dev_codes(o.pack(V)), d, x)
    a = search(tq, db, CQ, k, path=tq.TQ_PATH_PLAIN, engine=tq.TQ_ENGINE_SPARSE)
    b = search(tq, db, CQ, k, path=tq.TQ_PATH_PLAIN, engine=tq.TQ_ENGINE_POPCOUNT)
    c = search(tq, db, CQ, k, path=tq.TQ_PATH_PLAIN)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])
    # a query's own row: Delta = x; an earlier duplicate would come first
    for j, q in enumerate(qi):
        assert a[1][j, 0] == x
        assert q in a[0][j][a[1][j] == x]
    ei, es = o.knn(V[qi], V, k)
    assert np.array_equal(a[0], ei) and np.array_equal(a[1], es)
    db.destroy()


def test_sparse_copy_kept_only_for_small_x(tq, o):
    rng = np.random.default_rng(26)
    n, d = 500, 256
    sizes = {}
    for x in (32, 33):  # 8x <= d keeps the index list, 8x > d does not
        V, VQ = make(o, rng, n, d, x, 2)
        db = tq.tq_db_create(dev_codes(o.pack(V)), d, x)
        sizes[x] = db.info()[3]
        if x == 32:
            ids, sc = search(tq, db, o.pack(VQ), 5, engine=tq.TQ_ENGINE_SPARSE)  # AUTO path: plain
            ei, es = o.knn(VQ, V, 5)
            assert np.array_equal(sc, es) and np.array_equal(ids, ei)
            with pytest.raises(tq.TQError):
                tq.tq_search_knn(db, dev_codes(o.pack(VQ)), 5, path=tq.TQ_PATH_BATCHED, engine=tq.TQ_ENGINE_SPARSE)
        else:
            with pytest.raises(tq.TQError):
                tq.tq_search_knn(db, dev_codes(o.pack(VQ)), 5, path=tq.TQ_PATH_PLAIN, engine=tq.TQ_ENGINE_SPARSE)
        db.destroy()
    tiles = (n + 63) // 64
    planes = tiles * 64 * 2 * 16 * ((d // 32 + 3) // 4)
    assert sizes[33] == planes
    assert sizes[32] == planes + tiles * 64 * 16 * 4  # 4 chunks of 8 entries per vector


def test_sparse_rejects_any_count_database(tq, o):
    """x = 0 databases (any number of non-zeros per code) keep no index list."""
    rng = np.random.default_rng(27)
    d = 256
    V = o.encode_b158(rng.standard_normal((300, d)).astype(np.float32))
    db = tq.tq_db_create(dev_codes(o.pack(V)), d, 0)
    with pytest.raises(tq.TQError):
        tq.tq_search_knn(db, dev_codes(o.pack(V[:2])), 3, path=tq.TQ_PATH_PLAIN, engine=tq.TQ_ENGINE_SPARSE)
    db.destroy()


def test_sparse_timing_family(tq, o):
    rng = np.random.default_rng(28)
    V, VQ = make(o, rng, 5000, 512, 16, 3)
    db = tq.tq_db_create(dev_codes(o.pack(V)), 512, 16)
    tq.tq_timing_enable(True)
    tq.tq_timing_read(3, reset=True)
    search(tq, db, o.pack(VQ), 10, path=tq.TQ_PATH_PLAIN, engine=tq.TQ_ENGINE_SPARSE)
    ms, launches = tq.tq_timing_read(3, reset=True)
    tq.tq_timing_enable(False)
    assert launches == 3 and ms > 0
    db.destroy()
