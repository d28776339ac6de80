"""Parity at the full workload sizes, in the launch configuration bench.py
times (default grid and shapes).

mid (N = 1e6, d = 768, x in {96, 192, 384}): every code against the oracle's,
and top-100 of sampled queries (plain and batched) against the oracle's
exhaustive search over the oracle's own codes.

large (N = 1e7, d = 1024, x = 256): every code against the oracle's, chunk by
chunk; the exact top-100 of 18 sampled queries, from a running merge of the
oracle's search of each chunk (a top-k under the total order is the merge of
the top-k of disjoint parts, which the oracle pins check), against the plain
path (k = 10, 100) and the batched path at batch sizes 12 to 600 and
k = 1, 10, 100, with default and autotuned shapes; masked addition of float
queries against the oracle's masked top-10 built the same way; and the
index-list engine on the same rows at x = d / 32 equals the bit-plane scan.

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


def merge_running(run, add, K):
    """Merge two per-query key lists (ids, scores) into the K best by
    (score desc, id asc): the oracle's order, applied to partial results of
    disjoint row ranges (order independence is pinned on the oracle)."""
    if run is None:
        return add[0][:, :K].copy(), add[1][:, :K].copy()
    ids = np.concatenate([run[0], add[0]], 1)
    sc = np.concatenate([run[1], add[1]], 1)
    out_i = np.empty((ids.shape[0], K), dtype=ids.dtype)
    out_s = np.empty((ids.shape[0], K), dtype=sc.dtype)
    for q in range(ids.shape[0]):
        order = np.lexsort((ids[q], -sc[q].astype(np.float64)))[:K]
        out_i[q], out_s[q] = ids[q, order], sc[q, order]
    return out_i, out_s


# Queries of the 600-query pool whose exact top-100 the oracle computes over
# all 10^7 rows: the first and last rows of query tiles of 16, 64, 128 and 256
# queries and of the batch sizes below.
SAMPLED = [0, 1, 5, 11, 15, 16, 63, 64, 127, 128, 129, 255, 256, 299, 383, 511, 512, 599]
MASKED_Q = 4       # float queries whose exact masked-addition top-10 the oracle computes
MASKED_KEEP = 32   # oracle candidates kept per masked query (more than k, for the property check)


def test_large_exact(tq, o):
    """Every code of the 10^7 rows equals the oracle's; the exact oracle top-100
    of 18 sampled queries (a running merge over the oracle's search of each
    chunk) equals the plain path's top-10 / top-100 and the batched path's
    rows at batch sizes 12 ... 600 and k = 1, 10, 100, with default and with
    autotuned shapes, and on the matrix engine with parts of more than 2^20
    vectors; masked addition of 4 float queries equals the oracle's masked
    top-10."""
    w = datagen.WORKLOADS["large"]
    n, d, x, k = w["n"], w["d"], w["x"], w["k"]
    dev = torch.device("cuda", 0)
    W = tq.tq_code_words(d)
    nchunks = (n + datagen.CHUNK - 1) // datagen.CHUNK
    Q2 = datagen.rows(w["spec"], datagen.QUERIES, 0, 600, dev)
    qc2 = tq.tq_encode(Q2, x)
    VQS = o.encode(Q2[SAMPLED].cpu().numpy(), x)
    QM = Q2[:MASKED_Q].cpu().numpy()
    codes = torch.empty((n, 2 * W), dtype=torch.int32, device=dev)
    xs = d // 32  # the same rows at a small x, for the index-list engine
    codes_s = torch.empty((n, 2 * W), dtype=torch.int32, device=dev)
    top = None   # oracle top-100 of the sampled queries so far
    mtop = None  # oracle masked-addition candidates so far (ids, float scores)
    mexact = {}  # id -> exact double sum, per masked query, for kept candidates
    say(f"large full size: generate + encode N={n} d={d} x={x}; oracle encode and search of every chunk")
    for c, (r0, Xc) in enumerate(datagen.iter_rows(w["spec"], datagen.DB, 0, n, dev)):
        m = Xc.shape[0]
        tq.tq_encode(Xc, x, codes[r0:r0 + m])
        tq.tq_encode(Xc, xs, codes_s[r0:r0 + m])
        Xh = Xc.cpu().numpy()
        V = o.encode(Xh, x)
        assert np.array_equal(codes[r0:r0 + m].cpu().numpy().view(np.uint32), o.pack(V)), f"codes of chunk {c}"
        ci, cs = o.knn(VQS, V, min(100, m))
        top = merge_running(top, (ci.astype(np.int64) + r0, cs), 100)
        mi, ms, me = o.masked_knn(QM, V, min(MASKED_KEEP, m))
        for q in range(MASKED_Q):
            for j in range(mi.shape[1]):
                mexact[(q, int(mi[q, j]) + r0)] = float(me[q, j])
        mtop = merge_running(mtop, (mi.astype(np.int64) + r0, ms), MASKED_KEEP)
        if c % 16 == 0 or c == nchunks - 1:
            say(f"large full size: chunk {c + 1}/{nchunks} codes equal the oracle's")
    tq.tq_sync()
    db = tq.tq_db_create(codes, d, x)
    del codes
    ei, es = top

    def check_rows(ids, scores, rows, kk, what):
        ids, scores = ids.cpu().numpy(), scores.cpu().numpy()
        for r in rows:
            j = SAMPLED.index(r)
            assert np.array_equal(scores[r], es[j, :kk]), f"{what}: scores of query {r}"
            assert np.array_equal(ids[r], ei[j, :kk]), f"{what}: ids of query {r}"

    say("large full size: plain path top-10 and top-100 of the sampled queries")
    qs = qc2[SAMPLED]
    for kk in (10, 100):
        ip, sp = tq.tq_search_knn(db, qs, kk, path=tq.TQ_PATH_PLAIN)
        torch.cuda.synchronize()
        ip, sp = ip.cpu().numpy(), sp.cpu().numpy()
        assert np.array_equal(sp, es[:, :kk]) and np.array_equal(ip, ei[:, :kk]), f"plain k={kk}"
    # the batched path at the batching workload's sizes and k (both engines'
    # tiles: 16-query popcount tiles, 64 / 128 / 256-query matrix tiles), with
    # the default shapes and after the autotuner has picked its own
    cases = ((12, 1), (12, 10), (16, 100), (130, 10), (130, 100), (300, 1), (300, 100), (600, 10), (600, 100))
    for tuned in (False, True):
        if tuned:
            say("large full size: autotune (nq up to 1024, k = 1, 10, 100)")
            tq.tq_autotune(db, 1024, [1, 10, 100])
        for nq, kk in cases:
            say(f"large full size: {'auto (tuned)' if tuned else 'batched'} nq={nq} k={kk} against the oracle")
            path = tq.TQ_PATH_AUTO if tuned else tq.TQ_PATH_BATCHED
            ib, sb = tq.tq_search_knn(db, qc2[:nq], kk, path=path)
            torch.cuda.synchronize()
            check_rows(ib, sb, [r for r in SAMPLED if r < nq], kk, f"nq={nq} k={kk} tuned={tuned}")
            if not tuned and nq in (12, 300, 600):
                ip2, sp2 = tq.tq_search_knn(db, qc2[:nq], kk, path=tq.TQ_PATH_PLAIN)
                torch.cuda.synchronize()
                assert torch.equal(ib, ip2) and torch.equal(sb, sp2), ("batched vs plain", nq, kk)
    # the matrix engine with parts of more than 2^20 vectors (a grid of 8 or 16
    # workgroups: 8 parts of 19 532 tiles), where its k > 16 scan keeps 64-bit
    # keys instead of keys relative to the part's first id
    for nq, kk, grid in ((16, 100, 8), (130, 50, 16)):
        say(f"large full size: matrix engine, 8 parts of 1.25 M vectors, nq={nq} k={kk} grid={grid}")
        ib, sb = tq.tq_search_knn(db, qc2[:nq], kk, path=tq.TQ_PATH_BATCHED, engine=tq.TQ_ENGINE_MATRIX,
                                  qtile=64, grid=grid)
        torch.cuda.synchronize()
        check_rows(ib, sb, [r for r in SAMPLED if r < nq], kk, f"wide parts nq={nq} k={kk}")
    # masked addition of the float queries against the oracle's masked
    # top-10 (both sum in double and round once; a query whose float scores
    # differ -- a double sum within ~1e-12 of a rounding boundary -- is
    # checked by properties, at most one of the four)
    say("large full size: masked addition top-10 against the oracle")
    gi, gs = tq.tq_search_masked(db, Q2[:MASKED_Q], k)
    torch.cuda.synchronize()
    gi, gs = gi.cpu().numpy(), gs.cpu().numpy()
    oi, osc = mtop
    fallback = 0
    for q in range(MASKED_Q):
        if np.array_equal(gs[q], osc[q, :k]):
            assert np.array_equal(gi[q], oi[q, :k]), q
            continue
        fallback += 1
        assert fallback <= 1, "more than one masked query differs from the oracle"
        for j in range(k):
            assert (q, int(gi[q, j])) in mexact, (q, j, "not among the oracle's candidates")
            s = mexact[(q, int(gi[q, j]))]
            f, g = float(np.float32(s)), float(gs[q, j])
            if g != f:
                assert abs(g - f) <= float(np.spacing(np.float32(abs(f)))), (q, j)
                assert abs(s - (g + f) / 2) <= 1e-12 * abs(s), (q, j, "differs away from a rounding boundary")
            if j:
                assert gs[q, j - 1] > gs[q, j] or (gs[q, j - 1] == gs[q, j] and gi[q, j - 1] < gi[q, j])
        lim = float(gs[q, -1]) + float(np.spacing(np.float32(abs(gs[q, -1]))))
        chosen = set(gi[q].tolist())
        for j in range(MASKED_KEEP):
            if int(oi[q, j]) not in chosen:
                assert float(osc[q, j]) <= lim, (q, j, "an oracle candidate left out beats the k-th")
    db.destroy()
    # the index-list engine on the x = d / 32 codes of the same rows gives the
    # bit-plane scan's results
    db_s = tq.tq_db_create(codes_s, d, xs)
    del codes_s
    qs_s = tq.tq_encode(Q2[:16], xs)
    for kk in (10, 100):
        say(f"large full size: index lists vs bit planes x={xs} k={kk}")
        i_s, s_s = tq.tq_search_knn(db_s, qs_s, kk, path=tq.TQ_PATH_PLAIN, engine=tq.TQ_ENGINE_SPARSE)
        i_b, s_b = tq.tq_search_knn(db_s, qs_s, kk, path=tq.TQ_PATH_PLAIN, engine=tq.TQ_ENGINE_POPCOUNT)
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
