"""Parity at the full workload sizes, in the launch configuration bench.py
times (default grid and shapes).

mid (N = 1e6, d = 768, x in {96, 192, 384}): every code against the oracle's,
and top-100 of sampled queries (plain and batched) against the oracle's
exhaustive search over the oracle's own codes.

large (N = 1e7, d = 1024, x = 256): the oracle cannot encode all 10^7 rows in a
test's time, so codes are compared on sampled chunks, and each sampled
query's top-10 is checked by properties that hold at any size: every returned
score equals the oracle's Delta for that (query, row); results are ordered
(Delta desc, id asc); and no row of the sampled chunks that is not in the
result beats the k-th result.  Plain and batched results must be identical,
also for batches of 40 to 600 queries at k = 1, 10 and 100, and the
index-list engine on the same rows at x = d / 32 equals the bit-plane scan;
masked addition of the float queries is checked by the same kind of
properties.

serving (N = 5e6, d = 768, x = 192): a mix of requests served concurrently
gives the plain path's rows.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from tests.libtq import ensure_built
from workloads import datagen

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stderr.flush()


@pytest.fixture(scope="module")
def tq():
    return ensure_built()


@pytest.fixture(scope="module")
def o():
    return oracle.default()


def key_of(score, idx):
    return (int(score), -int(idx))


@pytest.fixture(scope="module")
def mid_data():
    w = datagen.WORKLOADS["mid"]
    dev = torch.device("cuda", 0)
    X = datagen.rows(w["spec"], datagen.DB, 0, w["n"], dev)
    Q = datagen.rows(w["spec"], datagen.QUERIES, 0, 16, dev)
    return w, X, Q, X.cpu().numpy(), Q.cpu().numpy()


@pytest.mark.parametrize("x", [96, 192, 384])
def test_mid_full_parity(tq, o, mid_data, x):
    w, X, Q, Xh, Qh = mid_data
    d, k = w["d"], w["k"]
    say(f"mid full size: encode N={w['n']} d={d} x={x}")
    codes = tq.tq_encode(X, x)
    qcodes = tq.tq_encode(Q, x)
    tq.tq_sync()
    V = o.encode(Xh, x)
    assert np.array_equal(codes.cpu().numpy().view(np.uint32), o.pack(V)), "codes differ"
    VQ = o.encode(Qh, x)
    ei, es = o.knn(VQ, V, k)
    db = tq.tq_db_create(codes, d, x)
    del codes
    for path in (tq.TQ_PATH_PLAIN, tq.TQ_PATH_BATCHED):
        say(f"mid full size: top-{k} x={x} path={path}")
        ids, sc = tq.tq_search_knn(db, qcodes, k, path=path)
        torch.cuda.synchronize()
        assert np.array_equal(sc.cpu().numpy(), es) and np.array_equal(ids.cpu().numpy(), ei), path
    db.destroy()


def test_large_sampled(tq, o):
    w = datagen.WORKLOADS["large"]
    n, d, x, k = w["n"], w["d"], w["x"], w["k"]
    dev = torch.device("cuda", 0)
    W = tq.tq_code_words(d)
    nchunks = (n + datagen.CHUNK - 1) // datagen.CHUNK
    sample_chunks = [0, 47, 101, nchunks - 1]
    say(f"large full size: generate + encode N={n} d={d} x={x}")
    codes = torch.empty((n, 2 * W), dtype=torch.int32, device=dev)
    xs = d // 32  # the same rows at a small x, for the index-list engine
    codes_s = torch.empty((n, 2 * W), dtype=torch.int32, device=dev)
    sampled = {}
    for r0, Xc in datagen.iter_rows(w["spec"], datagen.DB, 0, n, dev):
        tq.tq_encode(Xc, x, codes[r0:r0 + Xc.shape[0]])
        tq.tq_encode(Xc, xs, codes_s[r0:r0 + Xc.shape[0]])
        if r0 // datagen.CHUNK in sample_chunks:
            sampled[r0] = Xc.cpu().numpy()
    Q = datagen.rows(w["spec"], datagen.QUERIES, 0, 4, dev)
    qcodes = tq.tq_encode(Q, x)
    tq.tq_sync()
    say("large full size: sampled codes against the oracle")
    oracle_rows = {}
    for r0, Xh in sampled.items():
        V = o.encode(Xh, x)
        oracle_rows[r0] = V
        assert np.array_equal(codes[r0:r0 + Xh.shape[0]].cpu().numpy().view(np.uint32), o.pack(V)), r0
    db = tq.tq_db_create(codes, d, x)
    del codes
    say("large full size: top-10 plain and batched")
    ip, sp = tq.tq_search_knn(db, qcodes, k, path=tq.TQ_PATH_PLAIN)
    ib, sb = tq.tq_search_knn(db, qcodes, k, path=tq.TQ_PATH_BATCHED)
    torch.cuda.synchronize()
    assert torch.equal(ip, ib) and torch.equal(sp, sb), "plain and batched differ"
    ids, scores = ip.cpu().numpy(), sp.cpu().numpy()
    VQ = o.encode(Q.cpu().numpy(), x)
    # every returned score is the oracle's Delta for that row
    need = sorted(set(ids.ravel().tolist()))
    rows = torch.empty((len(need), d), dtype=torch.float32)
    for j, r in enumerate(need):
        c = r // datagen.CHUNK
        blk = datagen.chunk(datagen.SPECS[w["spec"]], datagen.DB, c, dev)
        rows[j] = blk[r - c * datagen.CHUNK].cpu()
    VR = o.encode(rows.numpy(), x)
    D = o.delta(VQ, VR)
    pos = {r: j for j, r in enumerate(need)}
    for q in range(4):
        for j in range(k):
            assert scores[q, j] == D[q, pos[ids[q, j]]], (q, j)
        keys = [key_of(scores[q, j], ids[q, j]) for j in range(k)]
        assert keys == sorted(keys, reverse=True), "not ordered"
        kth = keys[-1]
        chosen = set(ids[q].tolist())
        for r0, V in oracle_rows.items():
            Ds = o.delta(VQ[q:q + 1], V)[0]
            for i in np.nonzero(Ds >= kth[0])[0]:
                rid = r0 + int(i)
                if rid not in chosen:
                    assert key_of(Ds[i], rid) < kth, f"row {rid} beats the k-th result of query {q}"
    # the batched path at the batching workload's batch sizes and k (matrix
    # engine: 256-query tiles for k <= 16, 128- and 64-query tiles for k = 100)
    # gives the same bits as the plain path
    Q2 = datagen.rows(w["spec"], datagen.QUERIES, 100, 600, dev)
    qc2 = tq.tq_encode(Q2, x)
    for nq, kk in ((600, 1), (600, 10), (300, 100), (40, 100)):
        say(f"large full size: batched vs plain nq={nq} k={kk}")
        ib2, sb2 = tq.tq_search_knn(db, qc2[:nq], kk, path=tq.TQ_PATH_BATCHED)
        ip2, sp2 = tq.tq_search_knn(db, qc2[:nq], kk, path=tq.TQ_PATH_PLAIN)
        torch.cuda.synchronize()
        assert torch.equal(ib2, ip2) and torch.equal(sb2, sp2), (nq, kk)
    # masked addition of the float queries, checked by properties: every
    # returned score is the float rounding of the scalar product with the row's
    # ternary code (one unit in the last place: both sides sum in double, in
    # different orders), the order is (score desc, id asc), and no row of the
    # sampled chunks left out beats the k-th by more than that unit
    say("large full size: masked addition top-10")
    mi, ms = tq.tq_search_masked(db, Q, k)
    torch.cuda.synchronize()
    mi, ms = mi.cpu().numpy(), ms.cpu().numpy()
    Qh = Q.cpu().numpy().astype(np.float64)
    mneed = sorted(set(mi.ravel().tolist()))
    mrows = torch.empty((len(mneed), d), dtype=torch.float32)
    for j, r in enumerate(mneed):
        c = r // datagen.CHUNK
        blk = datagen.chunk(datagen.SPECS[w["spec"]], datagen.DB, c, dev)
        mrows[j] = blk[r - c * datagen.CHUNK].cpu()
    MV = o.encode(mrows.numpy(), x).astype(np.float64)
    mpos = {r: j for j, r in enumerate(mneed)}
    ulp = lambda f: float(np.spacing(np.float32(abs(f))))
    for q in range(4):
        for j in range(k):
            f = float(np.float32(Qh[q] @ MV[mpos[mi[q, j]]]))
            assert abs(float(ms[q, j]) - f) <= ulp(f), (q, j)
            if j:
                assert ms[q, j - 1] > ms[q, j] or (ms[q, j - 1] == ms[q, j] and mi[q, j - 1] < mi[q, j]), (q, j)
        lim = float(ms[q, -1]) + ulp(ms[q, -1])
        chosen = set(mi[q].tolist())
        for r0, V in oracle_rows.items():
            sc = (Qh[q] @ V.astype(np.float64).T).astype(np.float32)
            for i in np.nonzero(sc > lim)[0]:
                assert r0 + int(i) in chosen, f"row {r0 + int(i)} beats the masked k-th of query {q}"
    db.destroy()
    # the index-list engine on the x = d / 32 codes of the same rows gives the
    # bit-plane scan's results
    db_s = tq.tq_db_create(codes_s, d, xs)
    del codes_s
    qs = tq.tq_encode(Q2[:16], xs)
    for kk in (10, 100):
        say(f"large full size: index lists vs bit planes x={xs} k={kk}")
        i_s, s_s = tq.tq_search_knn(db_s, qs, kk, path=tq.TQ_PATH_PLAIN, engine=tq.TQ_ENGINE_SPARSE)
        i_b, s_b = tq.tq_search_knn(db_s, qs, kk, path=tq.TQ_PATH_PLAIN, engine=tq.TQ_ENGINE_POPCOUNT)
        torch.cuda.synchronize()
        assert torch.equal(i_s, i_b) and torch.equal(s_s, s_b), kk
    db_s.destroy()


def test_serving_full_size_mix_equals_plain(tq):
    """The serving workload's database (N = 5e6, d = 768, x = 192): requests of
    geometric size (mean 16, at most 256) with k in {10, 100}, submitted from
    four threads at once, each get exactly the plain path's rows."""
    import threading

    w = datagen.WORKLOADS["serving"]
    n, d, x = w["n"], w["d"], w["x"]
    dev = torch.device("cuda", 0)
    W = tq.tq_code_words(d)
    say(f"serving full size: generate + encode N={n} d={d} x={x}")
    codes = torch.empty((n, 2 * W), dtype=torch.int32, device=dev)
    for r0, Xc in datagen.iter_rows(w["spec"], datagen.DB, 0, n, dev):
        tq.tq_encode(Xc, x, codes[r0:r0 + Xc.shape[0]])
    nq_pool = 512
    qc = tq.tq_encode(datagen.rows(w["spec"], datagen.QUERIES, 0, nq_pool, dev), x)
    tq.tq_sync()
    db = tq.tq_db_create(codes, d, x)
    del codes
    say("serving full size: plain-path reference at k = 10 and 100")
    ref = {}
    for k in (10, 100):
        i, s = tq.tq_search_knn(db, qc, k, path=tq.TQ_PATH_PLAIN)
        torch.cuda.synchronize()
        ref[k] = (i.cpu().numpy(), s.cpu().numpy())
    qhost = qc.cpu().numpy().view(np.uint32)
    rng = np.random.default_rng(11)
    reqs = []
    for _ in range(48):
        while True:
            nq = int(rng.geometric(1 / 16))
            if nq <= 256:
                break
        reqs.append((int(rng.integers(0, nq_pool - nq + 1)), nq, int(rng.choice([10, 100]))))
    say(f"serving full size: {len(reqs)} requests from 4 threads")
    srv = tq.tq_server(db, max_k=100, budget_bytes=1 << 30)
    tickets = [None] * len(reqs)

    def submitter(part):
        for i in range(part, len(reqs), 4):
            q0, nq, k = reqs[i]
            tickets[i] = srv.submit(qhost[q0:q0 + nq], k)

    th = [threading.Thread(target=submitter, args=(p,)) for p in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    res = [srv.wait(t, 60000) for t in tickets]
    srv.destroy()
    for (q0, nq, k), r in zip(reqs, res):
        ei, es = ref[k]
        assert r is not None, (q0, nq, k)
        assert np.array_equal(r[0], ei[q0:q0 + nq]) and np.array_equal(r[1], es[q0:q0 + nq]), (q0, nq, k)
    db.destroy()
