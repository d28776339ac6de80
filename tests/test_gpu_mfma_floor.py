"""The matrix engine's sample floor (k > 16 on databases of >= 2 048 tiles).

Before the full scan, every 16th tile is scored with 16-key lists per
(query, part); the largest score s that at least k of those sample keys reach
is a floor (the query's k-th key overall scores >= s), and the full scan
drops keys scoring below s.  The result must be the exhaustive top-k of the
kNN problem (Sec. 1.1), bit for bit.

The database (2 049 tiles, a ragged last tile) holds 50 hub rows, each copied
about 500 times at random ids, so the queries made from hubs meet hundreds of
keys of one score -- more than k -- spread over sampled and unsampled tiles:
the floor then sits exactly at the k-th score and every tie at it must reach
the result by id.  The other queries are noisy database rows.  Results are
compared with the oracle's exhaustive top-k at k = 17, 64, 100, 128, on 64-,
128- and 256-query tiles, at the default grid and on 8 workgroups."""
import sys

import numpy as np
import pytest
import torch

import oracle
from tests.libtq import ensure_built

pytestmark = pytest.mark.gpu

N, D, X = 2048 * 64 + 37, 256, 64
NHUB, NQ = 50, 130


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stderr.flush()


@pytest.fixture(scope="module")
def tq():
    return ensure_built()


@pytest.fixture(scope="module")
def o():
    return oracle.default()


@pytest.fixture(scope="module")
def setup(tq, o):
    rng = np.random.default_rng(0x5A3F)
    centers = rng.standard_normal((16, D)).astype(np.float32)
    Xh = (centers[rng.integers(0, 16, N)] + 0.8 * rng.standard_normal((N, D))).astype(np.float32)
    hubs = Xh[rng.choice(N, NHUB, replace=False)].copy()
    dup = rng.choice(N, N // 5, replace=False)
    Xh[dup] = hubs[rng.integers(0, NHUB, dup.size)]
    Qh = np.concatenate([hubs[rng.integers(0, NHUB, NQ // 2)] + 0.05 * rng.standard_normal((NQ // 2, D)).astype(np.float32),
                         Xh[rng.choice(N, NQ - NQ // 2, replace=False)]
                         + 0.3 * rng.standard_normal((NQ - NQ // 2, D)).astype(np.float32)])
    say(f"floor: encode n={N} d={D} x={X} on both sides")
    dev = torch.device("cuda", 0)
    codes = tq.tq_encode(torch.from_numpy(Xh).to(dev), X)
    V = o.encode(Xh, X)
    assert np.array_equal(codes.cpu().numpy().view(np.uint32), o.pack(V)), "codes differ"
    qc = tq.tq_encode(torch.from_numpy(Qh).to(dev), X)
    VQ = o.encode(Qh, X)
    db = tq.tq_db_create(codes, D, X)
    yield db, qc, V, VQ
    db.destroy()


@pytest.mark.parametrize("k", [17, 64, 100, 128])
def test_floor_matches_oracle(tq, o, setup, k):
    db, qc, V, VQ = setup
    say(f"floor: oracle top-{k} of {NQ} queries")
    ei, es = o.knn(VQ, V, k)
    # the hub queries meet more than k equal top scores
    assert (es[: NQ // 2, k - 1] == es[: NQ // 2, 0]).sum() >= NQ // 4
    for qtile in (64, 128, 256):
        for grid in (0, 8):
            for nq in (16, NQ):
                say(f"floor: k={k} qtile={qtile} grid={grid} nq={nq}")
                ids, sc = tq.tq_search_knn(db, qc[:nq], k, path=tq.TQ_PATH_BATCHED, engine=tq.TQ_ENGINE_MATRIX,
                                           qtile=qtile, grid=grid)
                torch.cuda.synchronize()
                assert np.array_equal(sc.cpu().numpy(), es[:nq]), (k, qtile, grid, nq)
                assert np.array_equal(ids.cpu().numpy(), ei[:nq]), (k, qtile, grid, nq)


def test_floor_graph_replays(tq, o, setup):
    """One captured graph (bucket of 128 queries, k = 100) replayed with
    different query counts and offsets, other GPU work in between: the sample
    pass, the floor kernel and the full scan read the per-call parameters the
    prep kernel writes, so every replay must give the oracle's result."""
    db, qc, V, VQ = setup
    rng = np.random.default_rng(11)
    junk = torch.zeros(1 << 20, device="cuda")
    k = 100
    for rep in range(4):
        nq = int(rng.integers(65, 129))
        q0 = int(rng.integers(0, NQ - nq + 1))
        say(f"floor graph replay {rep}: nq={nq} q0={q0}")
        junk.add_(1.0)
        junk.sum().item()
        ids, sc = tq.tq_search_knn(db, qc[q0:q0 + nq], k, path=tq.TQ_PATH_BATCHED, engine=tq.TQ_ENGINE_MATRIX,
                                   qtile=64)
        torch.cuda.synchronize()
        ei, es = o.knn(VQ[q0:q0 + nq], V, k)
        assert np.array_equal(sc.cpu().numpy(), es) and np.array_equal(ids.cpu().numpy(), ei), rep
