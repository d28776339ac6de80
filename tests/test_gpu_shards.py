"""Row sharding, checked on one GPU: the database split into G row shards,
each its own resident database searched on its own, the shards' ids offset
and their top-k lists merged on the total-order key (Delta desc, id asc),
gives the same bits as the unsharded search and as the oracle -- the property
a multi-GPU form would rest on (one exchange of nq x k keys, then a merge)."""
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


def merge_shards(parts, k):
    """parts: list of (ids with global offsets, scores), each nq x k_shard."""
    ids = np.concatenate([p[0] for p in parts], axis=1)
    sc = np.concatenate([p[1] for p in parts], axis=1)
    out_i = np.empty((ids.shape[0], k), dtype=np.int32)
    out_s = np.empty((ids.shape[0], k), dtype=np.int32)
    for q in range(ids.shape[0]):
        keep = ids[q] >= 0
        order = np.lexsort((ids[q][keep], -sc[q][keep]))[:k]
        out_i[q] = ids[q][keep][order]
        out_s[q] = sc[q][keep][order]
    return out_i, out_s


ENGINES = {
    "plain": dict(path=1),
    "popcount": dict(path=2, engine=1),
    "matrix": dict(path=2, engine=2),
    "index_list": dict(path=1, engine=3),
}


@pytest.mark.parametrize("engine", list(ENGINES))
@pytest.mark.parametrize("bounds", [(0, 20000, 40000), (0, 7, 13001, 29990, 40000), (0, 64, 128, 40000)])
def test_row_shards_merge_to_the_same_bits(tq, o, engine, bounds):
    rng = np.random.default_rng(len(bounds) * 7 + len(engine))
    n, d, x, nq = 40000, 512, 32, 70
    V = o.encode(rng.standard_normal((n, d)).astype(np.float32), x)
    # heavy ties across shard boundaries: copies of a few codes everywhere
    base = V[rng.integers(0, n, size=5)]
    for c in range(5):
        V[rng.integers(0, n, size=300)] = base[c]
    VQ = np.concatenate([base, o.encode(rng.standard_normal((nq - 5, d)).astype(np.float32), x)])
    CQ = dev_codes(o.pack(VQ))
    kw = ENGINES[engine]
    whole = tq.tq_db_create(dev_codes(o.pack(V)), d, x)
    for k in (1, 10, 100):
        say(f"shards {bounds} engine={engine} k={k}")
        wi, ws = tq.tq_search_knn(whole, CQ, k, **kw)
        torch.cuda.synchronize()
        wi, ws = wi.cpu().numpy(), ws.cpu().numpy()
        parts = []
        for a, b in zip(bounds[:-1], bounds[1:]):
            sh = tq.tq_db_create(dev_codes(o.pack(V[a:b])), d, x)
            ks = min(k, b - a)
            si, ss = tq.tq_search_knn(sh, CQ, ks, **kw)
            torch.cuda.synchronize()
            parts.append((si.cpu().numpy() + a, ss.cpu().numpy()))
            sh.destroy()
        mi, ms = merge_shards(parts, k)
        assert np.array_equal(mi, wi) and np.array_equal(ms, ws), k
        ei, es = o.knn(VQ, V, k)
        assert np.array_equal(wi, ei) and np.array_equal(ws, es), k
    whole.destroy()
