"""Batched path (persistent query-tile kernel, hipGraph per bucket, autotuner)
against the CPU oracle, bit-exact."""
import os
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


def dev_codes(c):
    return torch.from_numpy(np.ascontiguousarray(c).view(np.int32).copy()).cuda()


@pytest.fixture(scope="module")
def small(tq, o):
    w = datagen.WORKLOADS["small"]
    X = datagen.rows("small", datagen.DB, 0, w["n"]).numpy()
    Q = datagen.rows("small", datagen.QUERIES, 0, 1500).numpy()
    V, VQ = o.encode(X, w["x"]), o.encode(Q, w["x"])
    db = tq.tq_db_create(dev_codes(o.pack(V)), w["d"], w["x"])
    yield dict(V=V, VQ=VQ, CQ=o.pack(VQ), db=db)
    db.destroy()


def run(tq, db, CQ, k, **kw):
    ids, sc = tq.tq_search_knn(db, dev_codes(CQ), k, **kw)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), sc.cpu().numpy()


@pytest.mark.parametrize("k", [1, 10, 64, 100, 128, 200, 512])
@pytest.mark.parametrize("nq", [1, 3, 17, 100])
def test_batched_vs_oracle(tq, o, small, k, nq):
    say(f"batched small k={k} nq={nq}")
    ids, sc = run(tq, small["db"], small["CQ"][:nq], k, path=tq.TQ_PATH_BATCHED)
    ei, es = o.knn(small["VQ"][:nq], small["V"], k)
    assert np.array_equal(sc, es) and np.array_equal(ids, ei)


@pytest.mark.parametrize("qtile", [2, 4, 8, 16])
@pytest.mark.parametrize("grid", [1, 5, 64, 512])
@pytest.mark.parametrize("use_graph", [0, 1])
def test_batched_shapes(tq, o, small, qtile, grid, use_graph):
    k, nq = 10, 37
    say(f"batched small qtile={qtile} grid={grid} graph={use_graph}")
    ids, sc = run(tq, small["db"], small["CQ"][:nq], k, path=tq.TQ_PATH_BATCHED, qtile=qtile, grid=grid,
                  use_graph=use_graph)
    ei, es = o.knn(small["VQ"][:nq], small["V"], k)
    assert np.array_equal(sc, es) and np.array_equal(ids, ei)


def test_batched_graph_replays(tq, o, small):
    """One bucket's graph replayed with different inputs and sizes, with other
    GPU work and host synchronisation between replays; every replay checked."""
    k = 10
    rng = np.random.default_rng(3)
    junk = torch.zeros(1 << 20, device="cuda")
    for rep in range(6):
        nq = int(rng.integers(33, 65))  # bucket 64 every time
        q0 = int(rng.integers(0, 1400))
        say(f"graph replay {rep} nq={nq} q0={q0}")
        junk.add_(1.0)
        junk.sum().item()
        ids, sc = run(tq, small["db"], small["CQ"][q0:q0 + nq], k, path=tq.TQ_PATH_BATCHED, use_graph=1)
        ei, es = o.knn(small["VQ"][q0:q0 + nq], small["V"], k)
        assert np.array_equal(sc, es) and np.array_equal(ids, ei), rep


def test_batched_many_queries(tq, o, small):
    """More than one 1024-query chunk in one call."""
    k = 10
    say("batched small nq=1500")
    ids, sc = run(tq, small["db"], small["CQ"], k, path=tq.TQ_PATH_BATCHED)
    ei, es = o.knn(small["VQ"], small["V"], k)
    assert np.array_equal(sc, es) and np.array_equal(ids, ei)


@pytest.mark.parametrize("n,d,k", [(1, 16, 1), (65, 100, 65), (130, 200, 100), (1007, 384, 300),
                                   (4160, 768, 512), (3000, 1024, 17)])
def test_batched_ragged(tq, o, n, d, k):
    rng = np.random.default_rng(n * 11 + d)
    x = max(1, d // 3)
    V = o.encode(rng.standard_normal((n, d)).astype(np.float32), x)
    VQ = o.encode(rng.standard_normal((9, d)).astype(np.float32), x)
    say(f"batched ragged n={n} d={d} k={k}")
    db = tq.tq_db_create(dev_codes(o.pack(V)), d, x)
    ids, sc = run(tq, db, o.pack(VQ), k, path=tq.TQ_PATH_BATCHED)
    ei, es = o.knn(VQ, V, k)
    assert np.array_equal(sc, es) and np.array_equal(ids, ei)
    db.destroy()


def test_batched_heavy_ties(tq, o):
    rng = np.random.default_rng(22)
    d, x = 256, 64
    base = o.encode(rng.standard_normal((6, d)).astype(np.float32), x)
    V = base[rng.integers(0, 6, size=20000)]
    VQ = np.concatenate([base[:3], o.encode(rng.standard_normal((20, d)).astype(np.float32), x)])
    say("batched heavy ties")
    db = tq.tq_db_create(dev_codes(o.pack(V)), d, x)
    for k in (1, 10, 100, 512):
        ids, sc = run(tq, db, o.pack(VQ), k, path=tq.TQ_PATH_BATCHED)
        ei, es = o.knn(VQ, V, k)
        assert np.array_equal(sc, es) and np.array_equal(ids, ei), k
    db.destroy()


def test_batched_rejects_bad_qtile(tq, small):
    q = dev_codes(small["CQ"][:4])
    for qt in (3, 32):
        with pytest.raises(tq.TQError):
            tq.tq_search_knn(small["db"], q, 10, path=tq.TQ_PATH_BATCHED, qtile=qt)
    with pytest.raises(tq.TQError):  # k = 300 supports query tiles up to 8
        tq.tq_search_knn(small["db"], q, 300, path=tq.TQ_PATH_BATCHED, qtile=16)


def test_autotune_then_auto(tq, o, small, tmp_path, monkeypatch):
    say("autotune small then auto path")
    tq.tq_autotune(small["db"], 64, [10, 100])
    for nq in (1, 2, 5, 64):
        for k in (10, 100):
            ids, sc = run(tq, small["db"], small["CQ"][:nq], k, path=tq.TQ_PATH_AUTO)
            ei, es = o.knn(small["VQ"][:nq], small["V"], k)
            assert np.array_equal(sc, es) and np.array_equal(ids, ei), (nq, k)


def test_autotune_large_buckets_then_other_k(tq, o, small):
    """Tuning k = 10 up to the 512-query bucket may store 256-query matrix
    tiles, which only k <= 16 supports; later automatic searches with k in
    other classes (17..64, 65..128, > 128) at those bucket sizes must not take
    that shape, and stay exact."""
    say("autotune to the 512 bucket at k=10, then auto at other k")
    tq.tq_autotune(small["db"], 512, [10])
    for nq, k in ((300, 50), (300, 17), (500, 100), (260, 200), (300, 10)):
        ids, sc = run(tq, small["db"], small["CQ"][:nq], k, path=tq.TQ_PATH_AUTO)
        ei, es = o.knn(small["VQ"][:nq], small["V"], k)
        assert np.array_equal(sc, es) and np.array_equal(ids, ei), (nq, k)


# ---------------------------------------------------------------------------
# the matrix-core engine (fp4 MFMA): same results, bit for bit
# ---------------------------------------------------------------------------

MATRIX_CASES = [(qtile, nq, k) for qtile in (64, 128, 256) for nq in (1, 3, 17, 100, 300)
                for k in (1, 10, 16, 17, 64, 65, 100, 128)]


@pytest.mark.parametrize("qtile,nq,k", MATRIX_CASES)
def test_matrix_vs_oracle(tq, o, small, k, nq, qtile):
    say(f"matrix engine small k={k} nq={nq} qtile={qtile}")
    ids, sc = run(tq, small["db"], small["CQ"][:nq], k, path=tq.TQ_PATH_BATCHED, engine=tq.TQ_ENGINE_MATRIX,
                  qtile=qtile)
    ei, es = o.knn(small["VQ"][:nq], small["V"], k)
    assert np.array_equal(sc, es) and np.array_equal(ids, ei)


@pytest.mark.parametrize("grid", [1, 7, 256, 1024])
@pytest.mark.parametrize("use_graph", [0, 1])
def test_matrix_shapes(tq, o, small, grid, use_graph):
    say(f"matrix engine grid={grid} graph={use_graph}")
    ids, sc = run(tq, small["db"], small["CQ"][:200], 10, path=tq.TQ_PATH_BATCHED, engine=tq.TQ_ENGINE_MATRIX,
                  grid=grid, use_graph=use_graph)
    ei, es = o.knn(small["VQ"][:200], small["V"], 10)
    assert np.array_equal(sc, es) and np.array_equal(ids, ei)


def test_matrix_many_queries(tq, o, small):
    say("matrix engine nq=1500")
    ids, sc = run(tq, small["db"], small["CQ"], 100, path=tq.TQ_PATH_BATCHED, engine=tq.TQ_ENGINE_MATRIX)
    ei, es = o.knn(small["VQ"], small["V"], 100)
    assert np.array_equal(sc, es) and np.array_equal(ids, ei)


@pytest.mark.parametrize("k", [10, 20])
@pytest.mark.parametrize("d", [1, 31, 33, 100, 128, 129, 255, 384, 500, 640, 768, 1000, 1024])
def test_matrix_dims(tq, o, d, k):
    rng = np.random.default_rng(300 + d)
    n, x = 777, max(1, (2 * d) // 3)
    V = o.encode(rng.standard_normal((n, d)).astype(np.float32), x)
    VQ = o.encode(rng.standard_normal((40, d)).astype(np.float32), x)
    say(f"matrix engine d={d} n={n} x={x} k={k}")
    db = tq.tq_db_create(dev_codes(o.pack(V)), d, x)
    ids, sc = run(tq, db, o.pack(VQ), k, path=tq.TQ_PATH_BATCHED, engine=tq.TQ_ENGINE_MATRIX)
    ei, es = o.knn(VQ, V, k)
    assert np.array_equal(sc, es) and np.array_equal(ids, ei)
    db.destroy()


def test_matrix_heavy_ties(tq, o):
    rng = np.random.default_rng(23)
    d, x = 256, 64
    base = o.encode(rng.standard_normal((6, d)).astype(np.float32), x)
    V = base[rng.integers(0, 6, size=20000)]
    VQ = np.concatenate([base[:3], o.encode(rng.standard_normal((40, d)).astype(np.float32), x)])
    say("matrix engine heavy ties")
    db = tq.tq_db_create(dev_codes(o.pack(V)), d, x)
    for k, qt in ((1, 64), (10, 128), (16, 256), (100, 64), (128, 128), (100, 256)):
        ids, sc = run(tq, db, o.pack(VQ), k, path=tq.TQ_PATH_BATCHED, engine=tq.TQ_ENGINE_MATRIX, qtile=qt)
        ei, es = o.knn(VQ, V, k)
        assert np.array_equal(sc, es) and np.array_equal(ids, ei), k
    db.destroy()


def test_matrix_graph_replays(tq, o, small):
    rng = np.random.default_rng(4)
    junk = torch.zeros(1 << 20, device="cuda")
    for rep in range(5):
        nq = int(rng.integers(65, 129))
        q0 = int(rng.integers(0, 1300))
        say(f"matrix graph replay {rep} nq={nq}")
        junk.add_(1.0)
        junk.sum().item()
        ids, sc = run(tq, small["db"], small["CQ"][q0:q0 + nq], 10, path=tq.TQ_PATH_BATCHED,
                      engine=tq.TQ_ENGINE_MATRIX)
        ei, es = o.knn(small["VQ"][q0:q0 + nq], small["V"], 10)
        assert np.array_equal(sc, es) and np.array_equal(ids, ei), rep


def test_matrix_rejects(tq, small):
    q = dev_codes(small["CQ"][:4])
    with pytest.raises(tq.TQError):
        tq.tq_search_knn(small["db"], q, 200, path=tq.TQ_PATH_BATCHED, engine=tq.TQ_ENGINE_MATRIX)
    with pytest.raises(tq.TQError):
        tq.tq_search_knn(small["db"], q, 10, path=tq.TQ_PATH_BATCHED, engine=tq.TQ_ENGINE_MATRIX, qtile=16)
    with pytest.raises(tq.TQError):  # query tiles are 64, 128 or 256
        tq.tq_search_knn(small["db"], q, 17, path=tq.TQ_PATH_BATCHED, engine=tq.TQ_ENGINE_MATRIX, qtile=512)
    with pytest.raises(tq.TQError):
        tq.tq_search_knn(small["db"], q, 10, path=tq.TQ_PATH_BATCHED, engine=7)


@pytest.mark.parametrize("qtile", [64, 128])
@pytest.mark.parametrize("grid", [64, 256, 512])
def test_matrix_cross_part_bound_adversarial(tq, o, qtile, grid):
    """The parts of a query share a lower bound on its k-th key and drop keys
    below it.  Here each planted query's 52 exact copies (Delta = x) sit in
    three places -- 6 among the lowest ids, 40 in one contiguous block in the
    middle, 6 among the highest ids -- so one part holds most of the top-k,
    parts of higher ids publish bounds with the top score, and the order among
    the copies is decided by the ids alone: the lowest-id copies must win on
    every grid and tile."""
    rng = np.random.default_rng(31 + grid + qtile)
    d, x, n = 256, 64, 30000
    V = o.encode(rng.standard_normal((n, d)).astype(np.float32), x)
    planted = o.encode(rng.standard_normal((8, d)).astype(np.float32), x)
    for j in range(8):
        V[j * 6:j * 6 + 6] = planted[j]                     # 6 copies among the lowest ids
        V[12000 + j * 40:12000 + j * 40 + 40] = planted[j]  # 40 in one middle block
        V[n - 48 + j * 6:n - 48 + j * 6 + 6] = planted[j]   # 6 among the highest ids
    VQ = np.concatenate([planted, o.encode(rng.standard_normal((40, d)).astype(np.float32), x)])
    db = tq.tq_db_create(dev_codes(o.pack(V)), d, x)
    for k in (17, 50, 100, 128):
        say(f"matrix bound adversarial qtile={qtile} grid={grid} k={k}")
        ids, sc = run(tq, db, o.pack(VQ), k, path=tq.TQ_PATH_BATCHED, engine=tq.TQ_ENGINE_MATRIX, qtile=qtile,
                      grid=grid)
        ei, es = o.knn(VQ, V, k)
        assert np.array_equal(sc, es) and np.array_equal(ids, ei), k
    db.destroy()


@pytest.mark.parametrize("grid", [64, 512])
def test_popcount_cross_part_bound_adversarial(tq, o, grid):
    """The popcount engine's bound for k > 128 (each wave's share of a part is
    a sub-part): planted copies of each query at the lowest ids, in one middle
    block and at the highest ids, on many sub-parts, with k above and below
    the number of copies."""
    rng = np.random.default_rng(57 + grid)
    d, x, n = 256, 64, 30000
    V = o.encode(rng.standard_normal((n, d)).astype(np.float32), x)
    planted = o.encode(rng.standard_normal((4, d)).astype(np.float32), x)
    for j in range(4):
        V[j * 10:j * 10 + 10] = planted[j]
        V[15000 + j * 200:15000 + j * 200 + 200] = planted[j]
        V[n - 40 + j * 10:n - 40 + j * 10 + 10] = planted[j]
    VQ = np.concatenate([planted, o.encode(rng.standard_normal((5, d)).astype(np.float32), x)])
    db = tq.tq_db_create(dev_codes(o.pack(V)), d, x)
    for k in (129, 200, 512):
        say(f"popcount bound adversarial grid={grid} k={k}")
        ids, sc = run(tq, db, o.pack(VQ), k, path=tq.TQ_PATH_BATCHED, engine=tq.TQ_ENGINE_POPCOUNT, qtile=4,
                      grid=grid)
        ei, es = o.knn(VQ, V, k)
        assert np.array_equal(sc, es) and np.array_equal(ids, ei), k
    db.destroy()


def test_autotune_cache_file(tq, o, small, tmp_path, monkeypatch):
    """tq_autotune writes its choices to TQ_TUNE_CACHE, keyed by plane width,
    k class, batch-size bucket and the database's size class, and per bucket
    the best matrix shape of each query tile with its time (the key + /q<tile>);
    searches that use them, at sizes between the buckets too, are still
    exact."""
    import json
    import re
    path = tmp_path / "tune.json"
    monkeypatch.setenv("TQ_TUNE_CACHE", str(path))
    say("autotune cache file")
    tq.tq_autotune(small["db"], 16, [10])
    data = json.loads(path.read_text())
    assert data and all(re.fullmatch(r"nc\d+/kc\d+/b\d+/t\d+(/q\d+)?", key) for key in data), list(data)[:4]
    assert all({"qtile", "grid", "plain", "engine", "ms"} <= set(v) for v in data.values())
    per_tile = {key: v for key, v in data.items() if "/q" in key}
    assert per_tile and all(v["engine"] == tq.TQ_ENGINE_MATRIX and v["ms"] > 0 and key.endswith(f"/q{v['qtile']}")
                            for key, v in per_tile.items()), per_tile
    for nq in (1, 9, 12, 16):
        ids, sc = run(tq, small["db"], small["CQ"][:nq], 10, path=tq.TQ_PATH_AUTO)
        ei, es = o.knn(small["VQ"][:nq], small["V"], 10)
        assert np.array_equal(sc, es) and np.array_equal(ids, ei), nq


def test_many_distinct_k_evicts_entries(tq, o, small):
    """Every distinct (bucket, k, shape) keeps buffers and a graph; beyond 96
    the least recently used is freed after its latest use.  110 values of k in
    a row, each checked, then the first ones again."""
    say("batched: 110 distinct k values")
    CQ, VQ = small["CQ"][:3], small["VQ"][:3]
    for k in list(range(1, 111)) + [1, 2, 3]:
        ids, sc = run(tq, small["db"], CQ, k, path=tq.TQ_PATH_BATCHED, engine=tq.TQ_ENGINE_POPCOUNT)
        ei, es = o.knn(VQ, small["V"], k)
        assert np.array_equal(sc, es) and np.array_equal(ids, ei), k
