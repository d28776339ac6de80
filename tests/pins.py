"""Checks that pin the CPU oracle to what the paper and plain mathematics fix.

Each check takes an ``oracle.Oracle`` so the same checks can be run against
deliberately broken builds of the oracle (tests/test_oracle_mutants.py): a
plausible mistake anywhere in the oracle must make at least one of them fail.
Nothing here calls the GPU library.
"""
from __future__ import annotations

import itertools
import json
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------------------
# brute-force helpers written only here (independent of the oracle)
# ---------------------------------------------------------------------------

def all_vertices(d: int, x: int) -> np.ndarray:
    """Every {x,d} EVP vertex (Sec. 2.3): x non-zero places, each +-1."""
    out = []
    for places in itertools.combinations(range(d), x):
        for signs in itertools.product((-1, 1), repeat=x):
            v = [0] * d
            for p, s in zip(places, signs):
                v[p] = s
            out.append(v)
    return np.array(out, dtype=np.int8)


def bit_b2sp(cq: np.ndarray, cv: np.ndarray, W: int) -> np.ndarray:
    """b2sp of Sec. 5.1.2 written straight from the packed bit planes with
    Python integer popcounts: (bsp(+,+) + bsp(-,-)) - (bsp(+,-) + bsp(-,+))."""
    def plane(c, off):
        return [int.from_bytes(np.ascontiguousarray(r[off:off + W]).astype("<u4").tobytes(), "little")
                for r in c]
    qp, qm, vp, vm = plane(cq, 0), plane(cq, W), plane(cv, 0), plane(cv, W)
    out = np.empty((len(qp), len(vp)), dtype=np.int64)
    for a in range(len(qp)):
        for b in range(len(vp)):
            bsp = lambda s, t: bin(s & t).count("1")
            out[a, b] = (bsp(qp[a], vp[b]) + bsp(qm[a], vm[b])) - (bsp(qp[a], vm[b]) + bsp(qm[a], vp[b]))
    return out


def lexsort_topk(scores_row: np.ndarray, k: int):
    """Nearest first: larger score first, then lower id (np.lexsort brute force)."""
    ids = np.arange(scores_row.shape[0])
    order = np.lexsort((ids, -scores_row.astype(np.int64)))
    return order[:k].astype(np.int32), scores_row[order[:k]].astype(np.int32)


# ---------------------------------------------------------------------------
# encode (Sec. 2.4)
# ---------------------------------------------------------------------------

def check_table3_encode(o):
    g = golden("table3_worked_example.json")
    V = o.encode(np.array([g["u1"], g["u2"]], dtype=np.float32), g["x"])
    assert V[0].tolist() == g["v1_printed"], "Table 3: v1 must match the printed vertex"
    sel = sorted(np.nonzero(V[1])[0].tolist())
    assert sel == g["u2_highlighted"], "Table 3: u2's highlighted cells are its x largest"
    # the four signs the table prints consistently; index 8 is the erratum
    for i in (1, 2, 3, 6):
        assert V[1][i] == g["v2_printed"][i]
    assert V[1][8] == 1, "u2[8] = +0.4 is positive, so its vertex coordinate is +1"


def check_enumeration_argmax(o, seed=1):
    """Sec. 2.4: the nearest vertex maximises the scalar product. For every d<=10
    and every x, the encoding is an argmax over all C(d,x)*2^x vertices, and is
    the argmax when that is unique."""
    rng = np.random.default_rng(seed)
    for d in range(1, 11):
        for x in range(1, d + 1):
            verts = all_vertices(d, x)
            assert verts.shape[0] == math.comb(d, x) * 2 ** x
            U = rng.standard_normal((6, d)).astype(np.float32)
            V = o.encode(U, x)
            for u, v in zip(U, V):
                s = verts.astype(np.float64) @ u.astype(np.float64)
                best = s.max()
                mine = float(v.astype(np.float64) @ u.astype(np.float64))
                assert mine == best, f"d={d} x={x}: encoding is not the nearest vertex"
                winners = np.nonzero(s == best)[0]
                if winners.size == 1:
                    assert np.array_equal(verts[winners[0]], v)


def check_fig2_cuboctahedron(o, seed=2):
    g = golden("fig2_cuboctahedron.json")
    printed = sorted(tuple(v) for v in g["vertices"])
    assert sorted(tuple(v) for v in all_vertices(3, 2).tolist()) == printed
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((3000, 3)).astype(np.float32)
    seen = {tuple(r) for r in o.encode(U, 2).tolist()}
    assert sorted(seen) == printed, "random points land on exactly the 12 printed vertices"


def check_special_cases(o, seed=3):
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((50, 37)).astype(np.float32)
    # x = d: the sign vector, i.e. 1-bit quantisation (Sec. 4.2: {d,d} EVP)
    Vd = o.encode(U, 37)
    assert np.array_equal(Vd, np.where(U < 0, -1, 1).astype(np.int8))
    # x = 1: signed one-hot at the largest magnitude
    V1 = o.encode(U, 1)
    am = np.argmax(np.abs(U), axis=1)
    exp = np.zeros_like(V1)
    exp[np.arange(50), am] = np.where(U[np.arange(50), am] < 0, -1, 1)
    assert np.array_equal(V1, exp)


def check_invariants(o, seed=4):
    rng = np.random.default_rng(seed)
    for d, x in ((1, 1), (31, 7), (32, 32), (33, 11), (100, 67), (384, 96)):
        U = rng.standard_normal((40, d)).astype(np.float32)
        V = o.encode(U, x)
        assert np.all(np.count_nonzero(V, axis=1) == x), "exactly x non-zeros"
        assert set(np.unique(V).tolist()) <= {-1, 0, 1}
        # positive scaling by a power of two does not move the vertex
        assert np.array_equal(o.encode(U * np.float32(8.0), x), V)
        # reflection through the origin reflects the vertex (no zeros here)
        assert np.array_equal(o.encode(-U, x), -V)


def check_ties_and_zeros(o):
    # equal magnitudes at the cut: lower index wins
    V = o.encode(np.array([[0.5, -0.5, 0.5, 0.25]], np.float32), 2)
    assert V[0].tolist() == [1, -1, 0, 0]
    V = o.encode(np.array([[0.25, 0.5, -0.5, 0.5, 0.5]], np.float32), 3)
    assert V[0].tolist() == [0, 1, -1, 1, 0]
    # selected zeros, including -0.0, get +1 (negative iff u < 0)
    V = o.encode(np.array([[0.0, -0.0, 0.0, 1.0]], np.float32), 3)
    assert V[0].tolist() == [1, 1, 0, 1]
    # subnormals keep their order and sign
    tiny = np.float32(1e-45)
    V = o.encode(np.array([[tiny, -tiny * 3, 0.0, -tiny * 2]], np.float32), 2)
    assert V[0].tolist() == [0, -1, 0, -1]
    V = o.encode(np.array([[0.0, -tiny, 0.0, 0.0]], np.float32), 2)
    assert V[0].tolist() == [1, -1, 0, 0]


# ---------------------------------------------------------------------------
# bit planes (Sec. 5.1.2, Table 3)
# ---------------------------------------------------------------------------

def _bits_from_word_rows(C, W, d):
    plus = [(int(C[w]) >> b) & 1 for w in range(W) for b in range(32)][:d]
    minus = [(int(C[W + w]) >> b) & 1 for w in range(W) for b in range(32)][:d]
    return plus, minus


def check_table3_pack(o):
    g = golden("table3_worked_example.json")
    W = o.words_per_plane(10)
    assert W == 1
    for v, vp, vm in (("v1_printed", "v1_plus_printed", "v1_minus_printed"),
                      ("v2_printed", "v2_plus_printed", "v2_minus_printed")):
        C = o.pack(np.array([g[v]], np.int8))
        plus, minus = _bits_from_word_rows(C[0], W, 10)
        assert plus == g[vp] and minus == g[vm], f"Table 3 bit rows of {v}"


def check_pack_layout(o, seed=5):
    rng = np.random.default_rng(seed)
    for d in (1, 5, 32, 33, 64, 100, 384):
        W = o.words_per_plane(d)
        assert W == (d + 31) // 32
        V = rng.integers(-1, 2, size=(20, d)).astype(np.int8)
        C = o.pack(V)
        assert C.shape == (20, 2 * W)
        for r in range(20):
            plus, minus = _bits_from_word_rows(C[r], W, d)
            assert plus == (V[r] == 1).astype(int).tolist()
            assert minus == (V[r] == -1).astype(int).tolist()
        assert np.all((C[:, :W] & C[:, W:]) == 0)
        if d % 32:
            pad = np.uint32((0xFFFFFFFF << (d % 32)) & 0xFFFFFFFF)
            assert np.all((C[:, W - 1] & pad) == 0) and np.all((C[:, 2 * W - 1] & pad) == 0)
        assert np.array_equal(o.unpack(C, d), V), "pack/unpack round trip"


# ---------------------------------------------------------------------------
# Delta = b2sp (Sec. 5.1.2)
# ---------------------------------------------------------------------------

def check_table3_delta(o):
    g = golden("table3_worked_example.json")
    v1 = np.array([g["v1_printed"]], np.int8)
    v2p = np.array([g["v2_printed"]], np.int8)
    v2 = o.encode(np.array([g["u2"]], np.float32), g["x"])
    assert int(o.delta(v1, v2p)[0, 0]) == g["delta_v1_v2"]
    assert int(o.delta(v1, v2)[0, 0]) == g["delta_v1_v2"]


def check_delta_identities(o, seed=6):
    rng = np.random.default_rng(seed)
    d, x = 100, 67
    V = o.encode(rng.standard_normal((60, d)).astype(np.float32), x)
    D = o.delta(V, V)
    assert np.all(np.diag(D) == x), "Delta(v,v) = x"
    assert np.array_equal(D, D.T), "symmetry"
    assert np.all(np.abs(D) <= x)
    assert np.all(np.diag(o.delta(V, -V)) == -x), "Delta(v,-v) = -x"
    # squared vertex distance 2x - 2 Delta is the squared Euclidean distance
    Vf = V.astype(np.float64)
    sq = ((Vf[:, None, :] - Vf[None, :, :]) ** 2).sum(-1)
    assert np.array_equal(sq, 2 * x - 2 * D.astype(np.float64))
    # library routine: an FP64 product of ternary matrices is exact here
    assert np.array_equal((Vf @ Vf.T).astype(np.int64), D.astype(np.int64))


def check_delta_one_bit_hamming(o, seed=7):
    """x = d: Delta = d - 2 * Hamming distance of the sign bits (Sec. 4.2)."""
    rng = np.random.default_rng(seed)
    d = 77
    U = rng.standard_normal((30, d)).astype(np.float32)
    V = o.encode(U, d)
    D = o.delta(V, V)
    neg = V < 0
    ham = (neg[:, None, :] != neg[None, :, :]).sum(-1)
    assert np.array_equal(D, d - 2 * ham)


def check_delta_bitwise(o, seed=8):
    rng = np.random.default_rng(seed)
    for d in (10, 33, 96):
        W = o.words_per_plane(d)
        Q = rng.integers(-1, 2, size=(5, d)).astype(np.int8)
        V = rng.integers(-1, 2, size=(9, d)).astype(np.int8)
        assert np.array_equal(o.delta(Q, V).astype(np.int64), bit_b2sp(o.pack(Q), o.pack(V), W))


# ---------------------------------------------------------------------------
# top-k (exhaustive kNN, Sec. 1.1 / Table 1; "closest n", Sec. 5.3)
# ---------------------------------------------------------------------------

def check_knn_bruteforce(o, seed=9):
    rng = np.random.default_rng(seed)
    for n, d, x, k in ((50, 16, 5, 7), (300, 40, 10, 30), (64, 8, 2, 64)):
        V = o.encode(rng.standard_normal((n, d)).astype(np.float32), x)
        Q = o.encode(rng.standard_normal((6, d)).astype(np.float32), x)
        ids, sc = o.knn(Q, V, k)
        D = (Q.astype(np.int64) @ V.astype(np.int64).T)
        for q in range(Q.shape[0]):
            ei, es = lexsort_topk(D[q], k)
            assert np.array_equal(ids[q], ei) and np.array_equal(sc[q], es)


def check_knn_ties(o, seed=10):
    """Many exact ties: duplicated database codes; lower id must win."""
    rng = np.random.default_rng(seed)
    base = o.encode(rng.standard_normal((5, 24)).astype(np.float32), 6)
    V = base[rng.integers(0, 5, size=400)]
    Q = base[:3]
    k = 50
    ids, sc = o.knn(Q, V, k)
    D = Q.astype(np.int64) @ V.astype(np.int64).T
    for q in range(3):
        assert np.all(np.diff(sc[q]) <= 0)
        for j in range(k - 1):
            if sc[q][j] == sc[q][j + 1]:
                assert ids[q][j] < ids[q][j + 1]
        chosen = set(ids[q].tolist())
        kth = (int(sc[q][-1]), -int(ids[q][-1]))
        for i in range(400):
            if i not in chosen:
                assert (int(D[q, i]), -i) < kth, "an excluded id beats the k-th result"
        ei, es = lexsort_topk(D[q], k)
        assert np.array_equal(ids[q], ei)


def check_knn_shard_merge(o, seed=11):
    """Order independence of the total-order key: top-k of shard top-ks."""
    rng = np.random.default_rng(seed)
    n, d, x, k = 700, 48, 20, 25
    V = o.encode(rng.standard_normal((n, d)).astype(np.float32), x)
    Q = o.encode(rng.standard_normal((4, d)).astype(np.float32), x)
    full_i, full_s = o.knn(Q, V, k)
    cuts = [0, 90, 91, 400, n]
    cand_i, cand_s = [], []
    for a, b in zip(cuts[:-1], cuts[1:]):
        kk = min(k, b - a)
        i, s = o.knn(Q, V[a:b], kk)
        cand_i.append(i + a)
        cand_s.append(s)
    ci, cs = np.concatenate(cand_i, 1), np.concatenate(cand_s, 1)
    for q in range(4):
        order = np.lexsort((ci[q], -cs[q].astype(np.int64)))[:k]
        assert np.array_equal(ci[q][order], full_i[q]) and np.array_equal(cs[q][order], full_s[q])


# ---------------------------------------------------------------------------
# refinement of proxy candidates with the float vectors (Sec. 5.3 k@n)
# ---------------------------------------------------------------------------

def check_rerank_l2_order(o, seed=12):
    """With every id as a candidate and vectors of equal norm, the refined
    order is the order of l2 distance (Sec. 1.1: for normalised data the
    nearest in l2 have the largest scalar products).  Ternary {x,d} vertices
    as floats have norm^2 = x exactly and l2^2 = 2x - 2<q,v>, so the squared
    distances computed coordinate by coordinate below are exact."""
    rng = np.random.default_rng(seed)
    d, x, n = 24, 9, 300
    V = o.encode(rng.standard_normal((n, d)).astype(np.float32), x).astype(np.float32)
    Qv = o.encode(rng.standard_normal((6, d)).astype(np.float32), x).astype(np.float32)
    cand = np.tile(np.arange(n, dtype=np.int32), (6, 1))
    k = 25
    ids, sc = o.rerank(V, Qv, cand, k)
    for q in range(6):
        dist = [sum((float(Qv[q, i]) - float(V[j, i])) ** 2 for i in range(d)) for j in range(n)]
        order = sorted(range(n), key=lambda j: (dist[j], j))[:k]
        assert ids[q].tolist() == order, q
        assert np.array_equal(sc[q], np.array([x - dist[j] / 2 for j in order])), q


def check_rerank_invariants(o, seed=13):
    """Results are candidates, in (score desc, id asc) order, each score the
    scalar product of its pair; the candidate order does not matter; ids
    outside [0, n) are skipped and missing results are (-1, -inf)."""
    rng = np.random.default_rng(seed)
    n, d, nq, ncand, k = 400, 37, 5, 60, 12
    X = rng.standard_normal((n, d)).astype(np.float32)
    X[7] = X[3]  # an exact tie: equal rows give equal scores
    Q = rng.standard_normal((nq, d)).astype(np.float32)
    cand = np.stack([rng.permutation(n)[:ncand] for _ in range(nq)]).astype(np.int32)
    cand[:, 0], cand[:, 1] = 3, 7
    ids, sc = o.rerank(X, Q, cand, k)
    for q in range(nq):
        assert set(ids[q].tolist()) <= set(cand[q].tolist())
        for j in range(k):
            ref = float(np.dot(Q[q].astype(np.float64), X[ids[q, j]].astype(np.float64)))
            assert abs(sc[q, j] - ref) <= 1e-12 * max(1.0, abs(ref))
            if j:
                assert sc[q, j - 1] > sc[q, j] or (sc[q, j - 1] == sc[q, j] and ids[q, j - 1] < ids[q, j])
        # nothing left out beats the k-th
        left = [c for c in cand[q] if c not in set(ids[q].tolist())]
        for c in left:
            s = float(np.dot(Q[q].astype(np.float64), X[c].astype(np.float64)))
            assert (s, -c) < (sc[q, k - 1], -ids[q, k - 1])
        pos3, pos7 = list(ids[q]).index(3) if 3 in ids[q] else None, list(ids[q]).index(7) if 7 in ids[q] else None
        if pos3 is not None and pos7 is not None:
            assert pos3 < pos7, "equal scores: the lower id first"
    perm = np.stack([rng.permutation(ncand) for _ in range(nq)])
    ids2, sc2 = o.rerank(X, Q, np.take_along_axis(cand, perm, 1), k)
    assert np.array_equal(ids, ids2) and np.array_equal(sc, sc2)
    bad = cand.copy()
    bad[:, 2:] = -1
    bad[:, 1] = n  # outside [0, n)
    ids3, sc3 = o.rerank(X, Q, bad, 3)
    assert np.all(ids3[:, 0] == 3) and np.all(ids3[:, 1:] == -1) and np.all(np.isneginf(sc3[:, 1:]))


# ---------------------------------------------------------------------------
# masked addition: float query against ternary vectors (Sec. 5.1.2, Sec. 6)
# ---------------------------------------------------------------------------

def check_masked_ternary_query_is_delta(o, seed=14):
    """A ternary query (values -1, 0, +1 as floats) makes masked addition the
    ternary scalar product, i.e. b2sp = Delta (Sec. 5.1.2 defines both as the
    scalar product): same scores, and the same top-k order (ties: lower id)."""
    rng = np.random.default_rng(seed)
    d, x, n, k = 40, 15, 500, 30
    V = o.encode(rng.standard_normal((n, d)).astype(np.float32), x)
    VQ = o.encode(rng.standard_normal((4, d)).astype(np.float32), x)
    ids, sc, ex = o.masked_knn(VQ.astype(np.float32), V, k)
    kid, ksc = o.knn(VQ, V, k)
    assert np.array_equal(ids, kid)
    assert np.array_equal(sc, ksc.astype(np.float32)) and np.array_equal(ex, ksc.astype(np.float64))


def check_masked_float_query(o, seed=15):
    """For a float query the double sums equal the scalar product with the
    ternary vector (computed here by a library product, in another order) to
    well within double rounding; the float score is that sum rounded once;
    results are ordered by float score, ties to the lower id, and nothing
    left out beats the k-th."""
    rng = np.random.default_rng(seed)
    d, x, n, k = 100, 67, 800, 40
    V = o.encode(rng.standard_normal((n, d)).astype(np.float32), x)
    V[5] = V[9]  # equal vectors: equal scores, the lower id first
    Q = rng.standard_normal((5, d)).astype(np.float32)
    ids, sc, ex = o.masked_knn(Q, V, k)
    full = Q.astype(np.float64) @ V.astype(np.float64).T
    for q in range(5):
        bound = 1e-12 * float(np.abs(Q[q]).sum())
        assert np.all(np.abs(ex[q] - full[q, ids[q]]) <= bound)
        assert np.array_equal(sc[q], ex[q].astype(np.float32))
        for j in range(1, k):
            assert sc[q, j - 1] > sc[q, j] or (sc[q, j - 1] == sc[q, j] and ids[q, j - 1] < ids[q, j])
        rest = np.setdiff1d(np.arange(n), ids[q])
        f32 = full[q, rest].astype(np.float32)
        assert np.all((f32 < sc[q, -1]) | ((f32 == sc[q, -1]) & (rest > ids[q, -1])))
        if 5 in ids[q] and 9 in ids[q]:
            assert list(ids[q]).index(5) < list(ids[q]).index(9)


# ---------------------------------------------------------------------------
# b1.58 quantisation (Sec. 4.3), per embedding
# ---------------------------------------------------------------------------

def check_b158_worked(o):
    """Hand-worked rows: mean |u| = gamma, round(u / gamma) clipped to +-1,
    ties to even, an all-zero row stays zero."""
    X = np.array([[0.2, -0.5, 1.3, 0.0],    # gamma 0.5: 0.4, -1, 2.6, 0 -> 0, -1, 1, 0
                  [1.0, 3.0, -1.0, -3.0],   # gamma 2: 0.5, 1.5, -0.5, -1.5 -> 0, 1, 0, -1
                  [0.0, 0.0, 0.0, 0.0],
                  [2.0, -2.0, 2.0, -2.0]],  # gamma 2: the sign vector
                 dtype=np.float32)
    V = o.encode_b158(X)
    assert V.tolist() == [[0, -1, 1, 0], [0, 1, 0, -1], [0, 0, 0, 0], [1, -1, 1, -1]]


def check_b158_properties(o, seed=16):
    """Signs agree with u; scaling a row by a power of two changes nothing;
    the non-zeros are exactly the coordinates with |u| above gamma / 2."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((200, 77)).astype(np.float32)
    V = o.encode_b158(X)
    assert np.all((V == 0) | (np.sign(V) == np.sign(X)))
    assert np.array_equal(o.encode_b158(X * np.float32(8.0)), V)
    assert np.array_equal(o.encode_b158(X * np.float32(2.0 ** -20)), V)
    gamma = np.abs(X.astype(np.float64)).mean(1, keepdims=True)
    assert np.array_equal(V != 0, np.abs(X.astype(np.float64)) / gamma > 0.5)


# ---------------------------------------------------------------------------
# kNN by euclidean distance between ternary vectors (codes of varying
# non-zero counts, e.g. b1.58 of Sec. 4.3)
# ---------------------------------------------------------------------------

def check_knn_l2_worked(o):
    """Hand-worked distances: q = (1, 0, -1, 0) against five codes of 0 to 4
    non-zeros.  Squared distances 1, 2, 2, 0, 8 give the order 3, 0, 1, 2, 4
    (equal distances: lower id first) and scores nnz(q) - distance = 2, 1, 0,
    0, -6; the plain scalar product would rank codes 1 and 3 (Delta 2) first."""
    Q = np.array([[1, 0, -1, 0]], dtype=np.int8)
    V = np.array([[1, 0, 0, 0], [1, 1, -1, 1], [0, 0, 0, 0], [1, 0, -1, 0], [-1, 0, 1, 0]], dtype=np.int8)
    ids, sc = o.knn_l2(Q, V, 5)
    assert ids.tolist() == [[3, 0, 1, 2, 4]] and sc.tolist() == [[2, 1, 0, 0, -6]]


def check_knn_l2_library_distance(o, seed=17):
    """b1.58 codes (varying non-zero counts, with duplicates for ties): the
    order is that of scipy's squared euclidean distance (lexsort, lower id on
    ties), and every score is 2 Delta - nnz(v) by the oracle's Delta."""
    from scipy.spatial.distance import cdist

    rng = np.random.default_rng(seed)
    for n, d, k in ((300, 24, 40), (120, 7, 120)):
        base = o.encode_b158(rng.standard_normal((n // 3, d)).astype(np.float32))
        V = base[rng.integers(0, base.shape[0], size=n)]
        Q = np.concatenate([base[:2], o.encode_b158(rng.standard_normal((3, d)).astype(np.float32))])
        ids, sc = o.knn_l2(Q, V, k)
        dist = cdist(Q.astype(np.float64), V.astype(np.float64), "sqeuclidean")
        D = o.delta(Q, V)
        nnz_v = (V != 0).sum(1)
        for q in range(Q.shape[0]):
            order = np.lexsort((np.arange(n), dist[q]))[:k]
            assert np.array_equal(ids[q], order), q
            assert np.array_equal(sc[q], 2 * D[q, ids[q]] - nnz_v[ids[q]]), q


def check_knn_l2_equal_counts_is_delta(o, seed=18):
    """With exactly x non-zeros in every code the distance is 2x - 2 Delta, so
    the order is the Delta order and the score 2 Delta - x."""
    rng = np.random.default_rng(seed)
    n, d, x, k = 400, 40, 13, 60
    V = o.encode(rng.standard_normal((n, d)).astype(np.float32), x)
    Q = o.encode(rng.standard_normal((5, d)).astype(np.float32), x)
    ids, sc = o.knn_l2(Q, V, k)
    ei, es = o.knn(Q, V, k)
    assert np.array_equal(ids, ei) and np.array_equal(sc, 2 * es - x)


ALL_CHECKS = [
    check_table3_encode, check_enumeration_argmax, check_fig2_cuboctahedron, check_special_cases,
    check_invariants, check_ties_and_zeros, check_table3_pack, check_pack_layout, check_table3_delta,
    check_delta_identities, check_delta_one_bit_hamming, check_delta_bitwise, check_knn_bruteforce,
    check_knn_ties, check_knn_shard_merge, check_rerank_l2_order, check_rerank_invariants,
    check_masked_ternary_query_is_delta, check_masked_float_query, check_b158_worked, check_b158_properties,
    check_knn_l2_worked, check_knn_l2_library_distance, check_knn_l2_equal_counts_is_delta,
]
