"""HIP path against the CPU oracle, element by element (bit-exact: codes,
Delta and top-k ids/scores are integers).  Every call goes through the C ABI
(libtq.so via the ctypes binding).  Inputs are seeded; the same float32 bytes
go to both sides."""
import sys

import numpy as np
import pytest
import torch

import oracle
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
def o():
    return oracle.default()


def u32(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def gpu_codes(tq, X: np.ndarray, x: int) -> np.ndarray:
    Xg = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    codes = tq.tq_encode(Xg, x)
    tq.tq_sync()
    return u32(codes)


def oracle_codes(o, X, x):
    return o.pack(o.encode(X, x))


def make_db(tq, codes_u32: np.ndarray, d: int, x: int):
    t = torch.from_numpy(codes_u32.view(np.int32).copy()).cuda()
    return tq.tq_db_create(t, d, x)


def search(tq, db, qcodes_u32, k, **kw):
    q = torch.from_numpy(qcodes_u32.view(np.int32).copy()).cuda()
    ids, scores = tq.tq_search_knn(db, q, k, **kw)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), scores.cpu().numpy()


# ---------------------------------------------------------------------------
# encode
# ---------------------------------------------------------------------------

def test_encode_small_workload(tq, o):
    w = datagen.WORKLOADS["small"]
    say(f"encode small workload n={w['n']} d={w['d']} x={w['x']}")
    X = datagen.rows("small", datagen.DB, 0, w["n"]).numpy()
    Q = datagen.rows("small", datagen.QUERIES, 0, w["nq"]).numpy()
    for A in (X, Q):
        g = gpu_codes(tq, A, w["x"])
        assert np.array_equal(g, oracle_codes(o, A, w["x"]))


@pytest.mark.parametrize("d", [1, 2, 31, 32, 33, 63, 64, 65, 100, 127, 128, 129, 383, 384, 385, 500, 512, 640,
                               767, 768, 769, 1000, 1023, 1024])
def test_encode_dims(tq, o, d):
    rng = np.random.default_rng(1000 + d)
    xs = sorted({1, d, oracle.default_x(d), max(1, d // 4), int(rng.integers(1, d + 1))})
    n = 67
    X = rng.standard_normal((n, d)).astype(np.float32)
    # rows with many equal magnitudes, zeros of both signs and subnormals
    X[1] = np.round(X[1] * 2) / 2
    X[2, ::3] = 0.0
    X[2, 1::3] = -0.0
    X[3] = np.float32(1e-45) * rng.integers(-3, 4, size=d)
    X[4] = 0.0
    X[5] = -0.0
    for x in xs:
        say(f"encode d={d} n={n} x={x}")
        assert np.array_equal(gpu_codes(tq, X, x), oracle_codes(o, X, x)), f"d={d} x={x}"


def test_encode_ties(tq, o):
    rng = np.random.default_rng(5)
    d = 384
    X = (rng.integers(-3, 4, size=(300, d)) / 4).astype(np.float32)
    for x in (1, 7, 96, 200, 383, 384):
        say(f"encode ties d={d} x={x}")
        assert np.array_equal(gpu_codes(tq, X, x), oracle_codes(o, X, x))


def test_encode_rows_of_many_lengths(tq, o):
    rng = np.random.default_rng(6)
    for n in (1, 2, 3, 4, 5, 255, 1025):
        X = rng.standard_normal((n, 100)).astype(np.float32)
        say(f"encode n={n} d=100 x=67")
        assert np.array_equal(gpu_codes(tq, X, 67), oracle_codes(o, X, 67))


@pytest.mark.parametrize("d", [96, 384, 512, 768, 1024])
def test_encode_many_rows_per_wave(tq, o, d):
    """Enough rows that every wave encodes several in turn, so each search
    starts from the previous row's threshold: rows of one scale (a good guess),
    rows whose scales jump over many binades (the guess is far off, above and
    below), rows with heavy ties and rows with few non-zeros."""
    rng = np.random.default_rng(2000 + d)
    n = 40000
    X = rng.standard_normal((n, d)).astype(np.float32)
    kind = rng.integers(0, 4, size=n)
    X[kind == 1] *= (10.0 ** rng.uniform(-30, 30, size=(int((kind == 1).sum()), 1))).astype(np.float32)
    X[kind == 2] = np.round(X[kind == 2] * 2) / 2
    sparse = np.nonzero(kind == 3)[0]
    X[sparse[:, None], rng.integers(0, d, size=(sparse.size, d // 2))] = 0.0
    for x in sorted({1, d // 4, oracle.default_x(d), d}):
        say(f"encode many rows per wave n={n} d={d} x={x}")
        assert np.array_equal(gpu_codes(tq, X, x), oracle_codes(o, X, x)), f"d={d} x={x}"


@pytest.mark.parametrize("d", [100, 768, 1024])
def test_encode_outlier_rows(tq, o, d):
    """Rows with one huge coordinate next to ordinary rows: a wave's first-row
    guess (a quarter of the largest magnitude) and the guess carried from the
    previous row are far from the threshold, above and below, so the search
    gallops over many binades before it brackets the cut."""
    rng = np.random.default_rng(3000 + d)
    n = 20000
    X = rng.standard_normal((n, d)).astype(np.float32)
    kind = rng.integers(0, 3, size=n)  # 0 ordinary, 1 one coordinate 1e30, 2 scaled to 1e-30 with one 1.0
    X[kind == 2] *= np.float32(1e-30)
    rows = np.nonzero(kind > 0)[0]
    cols = rng.integers(0, d, size=rows.size)
    sign = np.where(rng.integers(0, 2, size=rows.size) == 0, 1.0, -1.0)
    X[rows, cols] = (sign * np.where(kind[rows] == 1, 1e30, 1.0)).astype(np.float32)
    assert np.isfinite(X).all()
    for x in sorted({1, 2, d // 4, oracle.default_x(d)}):
        say(f"encode outlier rows n={n} d={d} x={x}")
        assert np.array_equal(gpu_codes(tq, X, x), oracle_codes(o, X, x)), f"d={d} x={x}"


def test_encode_nonfinite_sets_flag(tq, o):
    rng = np.random.default_rng(7)
    X = rng.standard_normal((6, 64)).astype(np.float32)
    X[2, 5] = np.nan
    X[4, 63] = np.inf
    say("encode with NaN / inf rows")
    Xg = torch.from_numpy(X).cuda()
    codes = tq.tq_encode(Xg, 16)
    with pytest.raises(tq.TQError) as e:
        tq.tq_sync()
    assert e.value.status == tq.TQ_ERR_INVALID
    tq.tq_sync()  # the flag was cleared
    c = u32(codes)
    assert np.all(c[2] == 0) and np.all(c[4] == 0)
    good = [0, 1, 3, 5]
    assert np.array_equal(c[good], oracle_codes(o, X[good], 16))


# ---------------------------------------------------------------------------
# database
# ---------------------------------------------------------------------------

def test_db_create_rejects_malformed(tq, o):
    rng = np.random.default_rng(8)
    d, x = 100, 20
    C = oracle_codes(o, rng.standard_normal((10, d)).astype(np.float32), x)
    for what, mutate in (("both planes", lambda c: (c.__setitem__((3, 0), c[3, 0] | np.uint32(1)),
                                                c.__setitem__((3, 4), c[3, 4] | np.uint32(1)))),
                         ("padding bit", lambda c: c.__setitem__((5, 3), c[5, 3] | np.uint32(1 << 30))),
                         ("popcount", lambda c: c.__setitem__((7, 1), c[7, 1] ^ np.uint32(1)))):
        bad = C.copy()
        mutate(bad)
        say(f"db_create rejects: {what}")
        with pytest.raises(tq.TQError) as e:
            make_db(tq, bad, d, x)
        assert e.value.status == tq.TQ_ERR_INVALID


@pytest.mark.parametrize("n,d", [(1, 1), (63, 33), (64, 64), (65, 100), (1000, 384), (4099, 1024)])
def test_db_export_round_trip(tq, o, n, d):
    rng = np.random.default_rng(9 + n)
    x = oracle.default_x(d)
    C = oracle_codes(o, rng.standard_normal((n, d)).astype(np.float32), x)
    say(f"db export n={n} d={d}")
    db = make_db(tq, C, d, x)
    assert db.info()[:3] == (n, d, x)
    out = tq.tq_db_export(db)
    torch.cuda.synchronize()
    assert np.array_equal(u32(out), C)
    db.destroy()


# ---------------------------------------------------------------------------
# Delta and top-k
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def small(tq, o):
    w = datagen.WORKLOADS["small"]
    X = datagen.rows("small", datagen.DB, 0, w["n"]).numpy()
    Q = datagen.rows("small", datagen.QUERIES, 0, w["nq"]).numpy()
    V, VQ = o.encode(X, w["x"]), o.encode(Q, w["x"])
    CX, CQ = o.pack(V), o.pack(VQ)
    db = make_db(tq, CX, w["d"], w["x"])
    yield dict(w=w, V=V, VQ=VQ, CX=CX, CQ=CQ, db=db)
    db.destroy()


def test_delta_dump_small_workload(tq, o, small):
    say("delta dump small workload 100 x 10000")
    q = torch.from_numpy(small["CQ"].view(np.int32).copy()).cuda()
    D = tq.tq_delta_dump(small["db"], q)
    torch.cuda.synchronize()
    assert np.array_equal(D.cpu().numpy(), o.delta(small["VQ"], small["V"]))


@pytest.mark.parametrize("k", [1, 2, 10, 63, 64, 65, 100, 128, 129, 200, 256, 257, 512])
def test_search_small_workload(tq, o, small, k):
    say(f"plain search small workload k={k}")
    ids, sc = search(tq, small["db"], small["CQ"], k, path=tq.TQ_PATH_PLAIN)
    ei, es = o.knn(small["VQ"], small["V"], k)
    assert np.array_equal(sc, es)
    assert np.array_equal(ids, ei)


@pytest.mark.parametrize("grid", [1, 2, 3, 7, 40, 100])
def test_search_grid_shapes(tq, o, small, grid):
    say(f"plain search small workload grid={grid}")
    ids, sc = search(tq, small["db"], small["CQ"][:20], 10, path=tq.TQ_PATH_PLAIN, grid=grid)
    ei, es = o.knn(small["VQ"][:20], small["V"], 10)
    assert np.array_equal(ids, ei) and np.array_equal(sc, es)


@pytest.mark.parametrize("n,d,k", [(1, 16, 1), (2, 33, 2), (63, 64, 63), (64, 100, 64), (65, 100, 65),
                                   (130, 200, 100), (1007, 384, 300), (4160, 768, 512), (3000, 1024, 17)])
def test_search_ragged(tq, o, n, d, k):
    rng = np.random.default_rng(n * 7 + d)
    x = max(1, d // 3)
    V = o.encode(rng.standard_normal((n, d)).astype(np.float32), x)
    VQ = o.encode(rng.standard_normal((5, d)).astype(np.float32), x)
    say(f"plain search ragged n={n} d={d} x={x} k={k}")
    db = make_db(tq, o.pack(V), d, x)
    ids, sc = search(tq, db, o.pack(VQ), k, path=tq.TQ_PATH_PLAIN)
    ei, es = o.knn(VQ, V, k)
    assert np.array_equal(sc, es) and np.array_equal(ids, ei)
    db.destroy()


def test_search_heavy_ties(tq, o):
    """A database of few distinct codes: hundreds of vectors share each score."""
    rng = np.random.default_rng(21)
    d, x = 256, 64
    base = o.encode(rng.standard_normal((6, d)).astype(np.float32), x)
    V = base[rng.integers(0, 6, size=20000)]
    VQ = np.concatenate([base[:3], o.encode(rng.standard_normal((3, d)).astype(np.float32), x)])
    say("plain search heavy ties n=20000 d=256")
    db = make_db(tq, o.pack(V), d, x)
    for k in (1, 10, 100, 512):
        ids, sc = search(tq, db, o.pack(VQ), k, path=tq.TQ_PATH_PLAIN)
        ei, es = o.knn(VQ, V, k)
        assert np.array_equal(sc, es) and np.array_equal(ids, ei), k
    db.destroy()


def test_search_rejects_bad_args(tq, o, small):
    q = torch.from_numpy(small["CQ"][:2].view(np.int32).copy()).cuda()
    say("search argument checks")
    for k in (0, tq.TQ_MAX_K + 1):
        with pytest.raises(tq.TQError):
            tq.tq_search_knn(small["db"], q, k)
    bad = small["CQ"][:2].copy()
    W = bad.shape[1] // 2
    bad[1, 0] |= np.uint32(1)
    bad[1, W] |= np.uint32(1)  # coordinate 0 now in both planes
    qb = torch.from_numpy(bad.view(np.int32).copy()).cuda()
    with pytest.raises(tq.TQError) as e:
        tq.tq_search_knn(small["db"], qb, 5, check_queries=True)
    assert e.value.status == tq.TQ_ERR_INVALID


@pytest.mark.parametrize("grid", [0, 37])
def test_search_sample_floor_large_k(tq, o, grid):
    """k > 128 on a database of >= 2 048 tiles: the plain path first scans a
    sample (every 32nd tile) and the full scan drops keys below the sample's
    k-th key (k = 65 and 100 check the same database without a sample).  Each planted query has copies (Delta = x) only in tiles the
    sample skips plus one in sampled tile 0, and every code has many exact
    duplicates, so the sample's k-th key ties with keys of lower and higher
    ids elsewhere; the result must still be the oracle's."""
    rng = np.random.default_rng(41 + grid)
    n, d, x = 200_000, 256, 64
    base = o.encode(rng.standard_normal((3000, d)).astype(np.float32), x)
    V = base[rng.integers(0, 3000, size=n)]  # ~67 copies of every code
    planted = o.encode(rng.standard_normal((4, d)).astype(np.float32), x)
    for j in range(4):
        V[j] = planted[j]  # tile 0 is sampled
        for c in range(30):
            t = 1 + 32 * (c + 1) + j  # tiles the sample skips
            V[t * 64 + 5] = planted[j]
    VQ = np.concatenate([planted, base[:4], o.encode(rng.standard_normal((4, d)).astype(np.float32), x)])
    db = make_db(tq, o.pack(V), d, x)
    for k in (65, 100, 200, 512):
        say(f"sample floor n={n} k={k} grid={grid}")
        ids, sc = search(tq, db, o.pack(VQ), k, path=tq.TQ_PATH_PLAIN, grid=grid)
        ei, es = o.knn(VQ, V, k)
        assert np.array_equal(sc, es) and np.array_equal(ids, ei), k
    db.destroy()


def test_search_several_tiles_per_wave(tq, o):
    """d = 1024 codes of the large workload's mixture, n = 2^19 + 77 (8 194
    tiles, a ragged last one) at the default grid of 512 workgroups: every
    wave of the plain scan takes four or five tiles through its two
    alternating load buffers, the benchmarked kernel's loop; k = 10 scans
    directly and k = 100 after a sample pass.  The batched path (both engines)
    on the same database too."""
    n, d, x = (1 << 19) + 77, 1024, 256
    dev = torch.device("cuda", 0)
    say(f"several tiles per wave: generate + encode n={n} d={d} x={x}")
    X = datagen.rows("large", datagen.DB, 0, n, dev)
    Q = datagen.rows("large", datagen.QUERIES, 0, 8, dev)
    codes = tq.tq_encode(X, x)
    qcodes = tq.tq_encode(Q, x)
    tq.tq_sync()
    V, VQ = o.encode(X.cpu().numpy(), x), o.encode(Q.cpu().numpy(), x)
    del X
    assert np.array_equal(u32(codes), o.pack(V)), "codes differ"
    db = tq.tq_db_create(codes, d, x)
    del codes
    for k in (10, 100):
        ei, es = o.knn(VQ, V, k)
        for path, engine in ((tq.TQ_PATH_PLAIN, tq.TQ_ENGINE_AUTO), (tq.TQ_PATH_BATCHED, tq.TQ_ENGINE_POPCOUNT),
                             (tq.TQ_PATH_BATCHED, tq.TQ_ENGINE_MATRIX)):
            say(f"several tiles per wave k={k} path={path} engine={engine}")
            ids, sc = tq.tq_search_knn(db, qcodes, k, path=path, engine=engine)
            torch.cuda.synchronize()
            assert np.array_equal(sc.cpu().numpy(), es) and np.array_equal(ids.cpu().numpy(), ei), (k, path, engine)
    db.destroy()
