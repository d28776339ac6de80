"""Masked-addition search of float queries (tq_search_masked) against the
oracle's.  Both sum in double and round once to float; the sums are taken in
different orders, so a float score may differ by one unit in the last place
where the double sum lies within ~1e-12 of a rounding boundary.  Where every
score of a query matches (the normal case) the ids must match exactly; a
query with such a boundary case is checked by properties instead (every
returned score is the rounded scalar product of its id, and a score that
differs from it lies next to a rounding boundary; the order is (score desc, id
asc); nothing left out beats the k-th), and at most MAX_FALLBACK queries of a
call may need that."""
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


# Queries of one call that may be checked by properties instead of equality
# (rounding-boundary cases are rare: a double sum lies within ~1e-12 of a
# float rounding boundary for roughly one score in 10^4 to 10^5).
MAX_FALLBACK = 2


def check(gi, gs, ei, es, Q, V, exact_required=False):
    full = None
    fallback = 0
    for q in range(ei.shape[0]):
        if np.array_equal(gs[q], es[q]):
            assert np.array_equal(gi[q], ei[q]), q
            continue
        assert not exact_required, f"query {q}: scores differ"
        fallback += 1
        say(f"masked: query {q} differs from the oracle; checked by properties")
        assert fallback <= MAX_FALLBACK, f"{fallback} of {ei.shape[0]} queries differ from the oracle"
        if full is None:
            full = Q.astype(np.float64) @ V.astype(np.float64).T
        row = full[q]
        k = gi.shape[1]
        assert len(set(gi[q].tolist())) == k
        for j in range(k):
            s = float(row[gi[q, j]])
            f = np.float32(s)
            g = float(gs[q, j])
            if g != float(f):
                # one unit in the last place, and only where the double sum
                # lies next to the boundary between the two floats
                assert abs(g - float(f)) <= float(np.spacing(np.float32(abs(f)))), (q, j)
                boundary = (g + float(f)) / 2
                assert abs(s - boundary) <= 1e-12 * abs(s), (q, j, "score differs away from a rounding boundary")
            if j:
                assert gs[q, j - 1] > gs[q, j] or (gs[q, j - 1] == gs[q, j] and gi[q, j - 1] < gi[q, j])
        rest = np.setdiff1d(np.arange(V.shape[0]), gi[q])
        lim = float(gs[q, -1]) + float(np.spacing(np.float32(abs(gs[q, -1]))))
        assert np.all(row[rest].astype(np.float32) <= lim), q


def run(tq, db, Q, k, **kw):
    ids, sc = tq.tq_search_masked(db, torch.from_numpy(np.ascontiguousarray(Q, dtype=np.float32)).cuda(), k, **kw)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), sc.cpu().numpy()


@pytest.fixture(scope="module")
def small(tq, o):
    w = datagen.WORKLOADS["small"]
    X = datagen.rows("small", datagen.DB, 0, w["n"]).numpy()
    Q = datagen.rows("small", datagen.QUERIES, 0, 40).numpy()
    V = o.encode(X, w["x"])
    db = tq.tq_db_create(dev_codes(o.pack(V)), w["d"], w["x"])
    yield dict(V=V, Q=Q, db=db)
    db.destroy()


@pytest.mark.parametrize("k", [1, 10, 64, 65, 100, 257, 512])
def test_masked_small_workload(tq, o, small, k):
    say(f"masked small workload k={k}")
    gi, gs = run(tq, small["db"], small["Q"], k)
    ei, es, _ = o.masked_knn(small["Q"], small["V"], k)
    check(gi, gs, ei, es, small["Q"], small["V"])


@pytest.mark.parametrize("grid", [1, 3, 40, 512])
def test_masked_grids(tq, o, small, grid):
    say(f"masked small workload grid={grid}")
    gi, gs = run(tq, small["db"], small["Q"][:7], 10, grid=grid)
    ei, es, _ = o.masked_knn(small["Q"][:7], small["V"], 10)
    check(gi, gs, ei, es, small["Q"][:7], small["V"])


@pytest.mark.parametrize("d", [1, 31, 33, 64, 100, 129, 384, 500, 768, 1000, 1024])
def test_masked_dims(tq, o, d):
    rng = np.random.default_rng(400 + d)
    n, x = 2500, max(1, (2 * d) // 3)
    V = o.encode(rng.standard_normal((n, d)).astype(np.float32), x)
    Q = rng.standard_normal((6, d)).astype(np.float32)
    Q[1] *= 1e-20  # tiny and huge magnitudes
    Q[2] *= 1e20
    db = tq.tq_db_create(dev_codes(o.pack(V)), d, x)
    say(f"masked d={d} n={n} x={x}")
    for k in (1, 17, 100):
        gi, gs = run(tq, db, Q, k)
        ei, es, _ = o.masked_knn(Q, V, k)
        check(gi, gs, ei, es, Q, V)
    db.destroy()


def test_masked_ternary_queries_are_exact(tq, o):
    """Ternary-valued float queries give integer scores (= Delta): exact, with
    many ties, which must go to the lower id."""
    rng = np.random.default_rng(31)
    d, x = 256, 64
    base = o.encode(rng.standard_normal((8, d)).astype(np.float32), x)
    V = base[rng.integers(0, 8, size=9000)]
    VQ = np.concatenate([base[:2], o.encode(rng.standard_normal((10, d)).astype(np.float32), x)])
    db = tq.tq_db_create(dev_codes(o.pack(V)), d, x)
    say("masked ternary queries, heavy ties")
    for k in (1, 10, 100, 512):
        gi, gs = run(tq, db, VQ.astype(np.float32), k)
        ei, es, _ = o.masked_knn(VQ.astype(np.float32), V, k)
        check(gi, gs, ei, es, VQ.astype(np.float32), V, exact_required=True)
        kid, ksc = o.knn(VQ, V, k)  # and they are the Delta search's results
        assert np.array_equal(gi, kid) and np.array_equal(gs, ksc.astype(np.float32))
    db.destroy()


def test_masked_rejects(tq, small):
    Q = torch.zeros((2, 384), dtype=torch.float32, device="cuda")
    with pytest.raises(tq.TQError):
        tq.tq_search_masked(small["db"], Q, 0)
    with pytest.raises(tq.TQError):
        tq.tq_search_masked(small["db"], Q, 513)
    with pytest.raises(ValueError):
        tq.tq_search_masked(small["db"], torch.zeros((2, 100), dtype=torch.float32, device="cuda"), 5)


@pytest.mark.parametrize("grid", [0, 8, 256])
def test_masked_sample_floor_large_k(tq, o, grid):
    """A database of >= 2 048 tiles: where a wave scans few vectors against k,
    masked addition first scans a sample (every 32nd tile) and the full scan
    drops keys below the sample's k-th key -- every k here at grids 0 and 256;
    at grid 8 (6 250 vectors per wave) k = 200 and 512 take the sample and
    k = 100 and 128 scan without one.
    Ternary-valued queries make the scores exact integers: each planted query
    has copies only in tiles the sample skips plus one in sampled tile 0, and
    every code has many exact duplicates, so the sample's k-th key ties with
    keys of lower and higher ids elsewhere; float queries of the same database
    are checked as the other masked tests are."""
    rng = np.random.default_rng(73 + grid)
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
    Qt = VQ.astype(np.float32)
    Qf = rng.standard_normal((6, d)).astype(np.float32)
    db = tq.tq_db_create(dev_codes(o.pack(V)), d, x)
    for k in (100, 128, 200, 512):
        say(f"masked sample floor n={n} k={k} grid={grid}")
        gi, gs = run(tq, db, Qt, k, grid=grid)
        ei, es, _ = o.masked_knn(Qt, V, k)
        check(gi, gs, ei, es, Qt, V, exact_required=True)
        kid, ksc = o.knn(VQ, V, k)
        assert np.array_equal(gi, kid) and np.array_equal(gs, ksc.astype(np.float32)), k
        gi, gs = run(tq, db, Qf, k, grid=grid)
        ei, es, _ = o.masked_knn(Qf, V, k)
        check(gi, gs, ei, es, Qf, V)
    db.destroy()
