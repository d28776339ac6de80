"""The CPU oracle against the paper's printed values and plain mathematics."""
import math

import numpy as np
import pytest

import oracle
from tests import pins


@pytest.fixture(scope="module")
def o():
    return oracle.default()


@pytest.mark.parametrize("check", pins.ALL_CHECKS, ids=lambda c: c.__name__)
def test_pin(o, check):
    check(o)


def test_default_x_matches_printed_pairs():
    g = pins.golden("evp_pairs.json")
    for row in g["table2"] + g["table5"]:
        assert oracle.default_x(row["d"]) == row["x"], row


def test_default_x_closed_form():
    # C(d,x+1)2^(x+1) / (C(d,x)2^x) = 2(d-x)/(x+1), which is >= 1 iff x <= (2d-1)/3;
    # so the maximum sits at floor((2d-1)/3)+1, and at floor((2d-1)/3) when the
    # two counts are equal (3 divides 2d-1), the smaller x being taken
    for d in range(1, 400):
        m = (2 * d - 1) // 3
        expect = m if (2 * d - 1) % 3 == 0 else m + 1
        assert oracle.default_x(d) == expect, d


def test_vertex_counts():
    g = pins.golden("evp_pairs.json")
    for row in g["table2"]:
        lg = math.log10(oracle.vertex_count(row["d"], row["x"]))
        assert abs(lg - row["log10_vertices_printed"]) < 1.0, row
    assert oracle.vertex_count(3, 2) == 12  # Figure 2
    for d in range(1, 12):  # sum over x of C(d,x) 2^x = 3^d - 1 (all non-zero ternary vectors)
        assert sum(oracle.vertex_count(d, x) for x in range(1, d + 1)) == 3 ** d - 1


def test_encode_rejects_bad_input(o):
    X = np.ones((2, 8), np.float32)
    with pytest.raises(oracle.OracleError):
        o.encode(X, 0)
    with pytest.raises(oracle.OracleError):
        o.encode(X, 9)
    X[1, 3] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        o.encode(X, 4)
    assert e.value.rc == oracle.ENONFINITE
    X[1, 3] = np.inf
    with pytest.raises(oracle.OracleError):
        o.encode(X, 4)


def test_unpack_rejects_malformed(o):
    C = np.zeros((1, 2), np.uint32)
    C[0, 0] = C[0, 1] = 1  # coordinate 0 in both planes
    with pytest.raises(oracle.OracleError):
        o.unpack(C, 10)
    C = np.zeros((1, 2), np.uint32)
    C[0, 0] = 1 << 12  # beyond d = 10
    with pytest.raises(oracle.OracleError):
        o.unpack(C, 10)


def test_knn_rejects_bad_k(o):
    V = np.ones((5, 4), np.int8)
    with pytest.raises(oracle.OracleError):
        o.knn(V[:1], V, 6)
    with pytest.raises(oracle.OracleError):
        o.knn(V[:1], V, 0)


@pytest.mark.parametrize("row", [0, 1])
def test_spearman_uniform_sanity(o, row):
    """Loose statistical band around Table 2's uniform rows (not a pin), and
    the comparative claim: EVP ranks distances better than b1.58, which beats
    1-bit.  Distances in the ternary spaces are l2 between the ternary vectors
    (nnz(a) + nnz(b) - 2 <a,b>; for EVP and 1-bit the norms are constant, so
    that is a function of Delta alone)."""
    from scipy.stats import spearmanr
    g = pins.golden("spearman_uniform.json")["rows"][row]
    rng = np.random.default_rng(12)
    d, x, npairs = g["d"], g["x"], 20000
    U = rng.standard_normal((2 * npairs, d))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    U = U.astype(np.float32)
    a, b = U[:npairs], U[npairs:]
    true = np.linalg.norm(a.astype(np.float64) - b.astype(np.float64), axis=1)
    rhos = {}
    for name, enc in (("evp", lambda A: o.encode(A, x)), ("one_bit", lambda A: o.encode(A, d)),
                      ("b158", o.encode_b158)):
        Va, Vb = enc(a).astype(np.int32), enc(b).astype(np.int32)
        dist2 = (Va * Va).sum(1) + (Vb * Vb).sum(1) - 2 * (Va * Vb).sum(1)
        rhos[name] = spearmanr(true, dist2).correlation
    assert abs(rhos["evp"] - g["evp"]) < 0.06, rhos
    assert abs(rhos["b158"] - g["b158"]) < 0.06, rhos
    assert rhos["evp"] > rhos["b158"] + 0.03 and rhos["b158"] > rhos["one_bit"] + 0.03, rhos
