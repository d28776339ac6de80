"""The matrix engine's k > 16 scan at the edge of its part-relative keys.

Where every database part spans at most 2^20 vectors the scan keys a
candidate by (score, id - first id of the part) in 32 bits; wider parts keep
64-bit keys.  A database of 131 072 tiles (8 388 608 vectors of d = 64) split
into 8 parts gives parts of exactly 2^20 vectors, so local ids reach
2^20 - 1; one tile more (131 073) gives parts of 16 385 tiles and the 64-bit
form.  Each query's own row is planted at local ids 2^20 - 1 - q and at the
last ids of every part (before either side encodes), so those vectors are
the query's only exact matches and the top of every result comes from the
highest local ids.  Both databases are compared with the oracle's exhaustive
top-k (its own codes of the same rows), at k = 50 and 100, with 64- and
256-query tiles on a grid of 8 workgroups (one query tile, 8 parts)."""
import sys

import numpy as np
import pytest
import torch

import oracle
from tests.libtq import ensure_built
from workloads import datagen

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

D, X_NZ, NQ = 64, 16, 48


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stderr.flush()


@pytest.fixture(scope="module")
def tq():
    return ensure_built()


@pytest.fixture(scope="module")
def o():
    return oracle.default()


@pytest.mark.parametrize("ntiles", [131072, 131073])
def test_part_of_two_to_the_twenty(tq, o, ntiles):
    n = ntiles * 64
    dev = torch.device("cuda", 0)
    W = tq.tq_code_words(D)
    # queries with codes of their own: sixteen seeded coordinates of magnitude
    # one with random signs over small noise (a row of the mixture would share
    # its code with many database rows, and equal scores go to lower ids)
    rng = np.random.default_rng(0x2506)
    Qh = (0.01 * rng.standard_normal((NQ, D))).astype(np.float32)
    for q in range(NQ):
        Qh[q, rng.choice(D, X_NZ, replace=False)] = rng.choice([-1.0, 1.0], X_NZ)
    Q = torch.from_numpy(Qh).to(dev)
    # planted rows: id -> query; parts of ceil(ntiles / 8) tiles, as the split makes them
    span = (ntiles + 7) // 8 * 64
    plant = {}
    for p in range(8):
        first, end = p * span, min(n, (p + 1) * span)
        for q in range(NQ):
            for lid in ((1 << 20) - 1 - q, end - first - 1 - q):
                if 0 <= lid < end - first:
                    plant[first + lid] = q
    codes = torch.empty((n, 2 * W), dtype=torch.int32, device=dev)
    V = np.empty((n, D), dtype=np.int8)
    say(f"key span: encode n={n} d={D} x={X_NZ} on both sides, {len(plant)} planted rows")
    for r0, Xc in datagen.iter_rows("narrow", datagen.DB, 0, n, dev):
        m = Xc.shape[0]
        for i, q in plant.items():
            if r0 <= i < r0 + m:
                Xc[i - r0] = Q[q]
        tq.tq_encode(Xc, X_NZ, codes[r0:r0 + m])
        V[r0:r0 + m] = o.encode(Xc.cpu().numpy(), X_NZ)
    tq.tq_sync()
    assert np.array_equal(codes.cpu().numpy().view(np.uint32), o.pack(V)), "codes differ"
    qc = tq.tq_encode(Q, X_NZ)
    VQ = o.encode(Qh, X_NZ)
    db = tq.tq_db_create(codes, D, X_NZ)
    del codes
    for k in (50, 100):
        say(f"key span: ntiles={ntiles} k={k} oracle top-k")
        ei, es = o.knn(VQ, V, k)
        for qtile in (64, 256):
            say(f"key span: ntiles={ntiles} k={k} qtile={qtile} matrix engine, 8 parts of {(ntiles + 7) // 8} tiles")
            ids, sc = tq.tq_search_knn(db, qc, k, path=tq.TQ_PATH_BATCHED, engine=tq.TQ_ENGINE_MATRIX, qtile=qtile,
                                       grid=8)
            torch.cuda.synchronize()
            assert np.array_equal(sc.cpu().numpy(), es) and np.array_equal(ids.cpu().numpy(), ei), (ntiles, k, qtile)
        # the planted rows lead every result, highest local ids included
        for q in range(NQ):
            mine = sorted(i for i, qq in plant.items() if qq == q)
            assert sorted(ei[q, :len(mine)].tolist()) == mine and (es[q, :len(mine)] == X_NZ).all(), q
    db.destroy()
