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
