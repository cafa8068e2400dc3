"""Pins of the CPU oracle against facts that do not come from the oracle.

* the paper's worked multiline example (Sec. 4.2, golden fixture);
* RREF uniqueness: the FL route must equal direct Gauss-Jordan on M, done by
  two independent brute-force implementations (C and pure Python), on random
  tiny matrices and exhaustively over small fields;
* planted closed forms (Schur complement and its RREF) built by the input
  generator;
* the block identity of Sec. 4.1 (A X = B, checked by a sparse product that
  is not the solve) and the equality of the two orders of operations
  (Sec. 4.1 vs Sec. 4.3);
* a rowspace certificate that uses only M and the output.
"""
import itertools
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import flgen
import oracle
from oracle.bruteforce import rref_lists
from tests.certify import certify_rref, csr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
PRIMES = [2, 3, 5, 7, 251, 65521]


def _dense_rows(csr_triple, rows, n):
    rp, ci, v = csr_triple
    out = np.zeros((rows, n), np.int64)
    for i in range(rows):
        out[i, ci[rp[i]:rp[i + 1]]] = v[rp[i]:rp[i + 1]]
    return out


def _mat_from_dense(a, p):
    a = sp.csr_matrix(np.asarray(a, np.int64) % p)
    a.eliminate_zeros()
    a.sort_indices()
    return dict(m=a.shape[0], n=a.shape[1], p=p, row_ptr=a.indptr.astype(np.uint64),
                col=a.indices.astype(np.uint32), val=a.data.astype(np.uint16))


def test_modular_inverse_exhaustive():
    for p in (2, 3, 251, 65521):
        a = np.arange(1, p, dtype=np.int64)
        inv = np.array([oracle.inv(int(x), p) for x in a], dtype=np.int64)
        assert np.all((a * inv) % p == 1)
        assert np.all((inv >= 1) & (inv < p))


def test_multiline_paper_example():
    g = json.load(open(os.path.join(GOLDEN, "multiline_example.json")))
    mat = _mat_from_dense(g["rows"], 65521)
    gptr, pos, val = oracle.multiline((mat["row_ptr"], mat["col"], mat["val"]), 2, 7, 2)
    assert list(gptr) == [0, 5]
    assert pos.tolist() == g["multiline"]["pos"]
    assert val.tolist() == g["multiline"]["val"]
    assert int((val == 0).sum()) == g["padding_zeros"]
    # 1-multilines are plain sparse rows (the example's v_i / p_i)
    gp1, pos1, val1 = oracle.multiline((mat["row_ptr"], mat["col"], mat["val"]), 2, 7, 1)
    assert pos1[:3].tolist() == g["sparse"]["p1"] and val1[:3].tolist() == g["sparse"]["v1"]
    assert pos1[3:].tolist() == g["sparse"]["p2"] and val1[3:].tolist() == g["sparse"]["v2"]


@pytest.mark.parametrize("w", [1, 2, 3, 4, 8])
def test_multiline_roundtrip(w):
    """Unpacking a w-multiline gives back the rows; pos is the union of supports."""
    mat = flgen.random_sparse(13, 40, 0.2, 251, seed=w, zero_rows=0.2)
    csr3 = (mat["row_ptr"], mat["col"], mat["val"])
    gptr, pos, val = oracle.multiline(csr3, 13, 40, w)
    dense = _dense_rows(csr3, 13, 40)
    back = np.zeros_like(dense)
    for g in range(len(gptr) - 1):
        for k in range(int(gptr[g]), int(gptr[g + 1])):
            for q in range(w):
                if g * w + q < 13:
                    back[g * w + q, pos[k]] = val[k * w + q]
        union = np.nonzero(dense[g * w:(g + 1) * w].any(axis=0))[0]
        assert pos[gptr[g]:gptr[g + 1]].tolist() == union.tolist()
    assert np.array_equal(back, dense)


def _check_against_bruteforce(mat):
    p, n = mat["p"], mat["n"]
    res = oracle.fl_rref(mat)
    bf, rk = oracle.bruteforce_rref(mat)
    pr, _ = rref_lists(flgen.csr_to_dense(mat).astype(int).tolist(), p)
    assert res["rank"] == rk == len(pr)
    a = _dense_rows(res["rref"], rk, n)
    assert np.array_equal(a, _dense_rows(bf, rk, n))
    assert np.array_equal(a, np.array(pr, np.int64).reshape(rk, n))
    # the two orders of operations reach the same Schur complement
    assert np.array_equal(oracle.reduce_neworder(res["split"]), res["Dt"])


@pytest.mark.parametrize("seed", range(60))
def test_fl_equals_bruteforce_random(seed):
    rng = np.random.default_rng(1000 + seed)
    p = int(rng.choice(PRIMES))
    m, n = int(rng.integers(1, 12)), int(rng.integers(1, 16))
    mat = flgen.random_sparse(m, n, float(rng.uniform(0.05, 0.9)), p, seed,
                              monic=bool(seed % 2), zero_rows=0.15, dup_rows=0.25)
    assert oracle.validate(mat) == oracle.OR_OK
    _check_against_bruteforce(mat)


def test_exhaustive_2x3_f3_and_3x3_f2():
    for p, m, n in ((3, 2, 3), (2, 3, 3)):
        for vals in itertools.product(range(p), repeat=m * n):
            a = np.array(vals, np.int64).reshape(m, n)
            mat = _mat_from_dense(a, p)
            res = oracle.fl_rref(mat)
            pr, _ = rref_lists(a.tolist(), p)
            assert res["rank"] == len(pr)
            assert np.array_equal(_dense_rows(res["rref"], res["rank"], n),
                                  np.array(pr, np.int64).reshape(len(pr), n))


def test_pivot_row_selection_rule():
    """Rows 0, 1, 3 share lead column 0: row 3 has fewest nonzeros -> pivot;
    rows 1 and 2 tie on lead 2 with equal nnz -> lower index (1) wins."""
    a = np.array([[1, 0, 5, 6, 7, 0],
                  [0, 0, 1, 3, 0, 0],
                  [0, 0, 1, 0, 4, 0],
                  [1, 2, 0, 0, 0, 0]], np.int64)
    s = oracle.split(_mat_from_dense(a, 7))
    assert s["npiv"] == 2
    assert s["col_perm"].tolist() == [0, 2, 1, 3, 4, 5]
    assert s["row_perm"].tolist() == [3, 1, 0, 2]


def test_split_normalizes_pivot_rows_only():
    a = np.array([[3, 1, 2], [0, 5, 1], [4, 0, 6]], np.int64)  # lead 3 and 5, p = 7
    s = oracle.split(_mat_from_dense(a, 7))
    # pivot rows: row 2 (lead col 0, nnz 2 < 3) and row 1 (lead col 1)
    assert s["row_perm"].tolist() == [2, 1, 0]
    inv4, inv5 = oracle.inv(4, 7), oracle.inv(5, 7)
    A = _dense_rows(s["A"], 2, 2)
    assert A.tolist() == [[1, 0], [0, 1]]
    assert _dense_rows(s["B"], 2, 1).tolist() == [[6 * inv4 % 7], [1 * inv5 % 7]]
    assert _dense_rows(s["C"], 1, 2).tolist() == [[3, 1]]  # untouched
    assert _dense_rows(s["D"], 1, 1).tolist() == [[2]]


def test_validation_codes():
    good = flgen.random_sparse(4, 6, 0.5, 7, seed=3)
    assert oracle.validate(good) == oracle.OR_OK
    bad = dict(good); bad["p"] = 65537
    assert oracle.validate(bad) == oracle.OR_BAD_P
    k = int(good["row_ptr"][1]) - 1
    for field, value, code in (("col", 6, oracle.OR_COL_RANGE), ("val", 0, oracle.OR_BAD_VALUE),
                               ("val", 7, oracle.OR_BAD_VALUE)):
        bad = {kk: (vv.copy() if isinstance(vv, np.ndarray) else vv) for kk, vv in good.items()}
        bad[field][k] = value
        assert oracle.validate(bad) == code
    bad = {kk: (vv.copy() if isinstance(vv, np.ndarray) else vv) for kk, vv in good.items()}
    r0 = int(bad["row_ptr"][0]), int(bad["row_ptr"][1])
    if r0[1] - r0[0] >= 2:
        bad["col"][r0[0] + 1] = bad["col"][r0[0]]
        assert oracle.validate(bad) == oracle.OR_COL_ORDER


@pytest.fixture(scope="module")
def c1_case():
    g = flgen.config_matrix("c1")
    return g, oracle.fl_rref(g)


def test_c1_planted_closed_forms(c1_case):
    g, res = c1_case
    assert g["plant_ok"]
    s = res["split"]
    assert s["npiv"] == g["npiv"]
    assert np.array_equal(s["col_perm"][:s["npiv"]], g["piv_cols"])
    assert np.array_equal(res["Dt"], g["Dt"].toarray())
    assert res["rank_d"] == g["rank_d"]
    assert np.array_equal(res["RD"], g["V"].toarray())
    assert res["rank"] == g["npiv"] + g["rank_d"]


def test_c1_block_identity(c1_case):
    """A X = B (Sec. 4.1 step 2), via a sparse product, not the solve."""
    g, res = c1_case
    s, p = res["split"], g["p"]
    A = csr(*s["A"], s["npiv"], s["npiv"])
    B = csr(*s["B"], s["npiv"], s["nB"]).toarray()
    assert np.array_equal((A @ res["X"].astype(np.int64)) % p, B)
    C = csr(*s["C"], s["mD"], s["npiv"])
    D = csr(*s["D"], s["mD"], s["nB"]).toarray()
    assert np.array_equal((D - C @ res["X"].astype(np.int64)) % p, res["Dt"])


def test_c1_two_orders_agree(c1_case):
    g, res = c1_case
    assert np.array_equal(oracle.reduce_neworder(res["split"]), res["Dt"])


def test_c1_rowspace_certificate(c1_case):
    g, res = c1_case
    M = csr(g["row_ptr"], g["col"], g["val"], g["m"], g["n"])
    R = csr(*res["rref"], res["rank"], g["n"])
    certify_rref(M, R, g["p"], g["npiv"] + g["rank_d"])


@pytest.mark.slow
def test_c1_equals_bruteforce(c1_case):
    g, res = c1_case
    bf, rk = oracle.bruteforce_rref(g)
    assert rk == res["rank"]
    for x, y in zip(bf, res["rref"]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("p", [251, 65521])
def test_small_planted_various(p):
    g = flgen.fl_matrix(m=300, n=420, npiv=200, rank_d=60, density=0.08, p=p, seed=p)
    res = oracle.fl_rref(g)
    if g["plant_ok"]:
        assert np.array_equal(res["Dt"], g["Dt"].toarray())
    assert res["rank"] == 200 + 60
    assert np.array_equal(res["RD"], g["V"].toarray())
    bf, rk = oracle.bruteforce_rref(g)
    assert rk == res["rank"]
    for x, y in zip(bf, res["rref"]):
        assert np.array_equal(x, y)


def test_degenerate_inputs():
    # empty matrix, all-zero rows, a single row, full-rank square identity
    for a, p in ((np.zeros((3, 4), np.int64), 5), (np.eye(4, dtype=np.int64), 7),
                 (np.array([[0, 3, 0, 2]], np.int64), 5), (np.zeros((1, 1), np.int64), 2)):
        mat = _mat_from_dense(a, p)
        res = oracle.fl_rref(mat)
        pr, _ = rref_lists(a.tolist(), p)
        assert res["rank"] == len(pr)
        assert np.array_equal(_dense_rows(res["rref"], res["rank"], a.shape[1]),
                              np.array(pr, np.int64).reshape(len(pr), a.shape[1]))


def test_dense_planted_rank_generator_pin():
    d = flgen.dense_planted_rank(40, 56, 29, 251, seed=5)
    R, r, pc = oracle.rref_dense(d["D"], 251)
    assert r == 29 and np.array_equal(pc, d["pivcols"])
    assert np.array_equal(R[:r], d["V"])
    assert not R[r:].any()


@pytest.mark.parametrize("threads", [2, 5, 16])
def test_striped_trsm_equals_single_call(c1_case, threads):
    """The oracle's TRSM over column stripes in several threads is the same
    back substitution on independent column sets (Sec. 4.2): it must return
    the single call's X exactly, also with stripes narrower than a row run
    and with more stripes than the workload has cores."""
    g, r = c1_case
    s = r["split"]
    assert np.array_equal(oracle.trsm(s, threads), r["X"])


def test_column_subset_and_stripe():
    """The column selections the benchmark's CPU sample uses: relabelled
    columns, row pointers of the kept entries, values carried along."""
    import scipy.sparse as sps
    g = flgen.random_sparse(40, 90, 0.2, 65521, seed=9, zero_rows=0.1)
    M = sps.csr_matrix((g["val"].astype(np.int64), g["col"].astype(np.int64), g["row_ptr"].astype(np.int64)),
                       shape=(40, 90)).toarray()
    cols = np.array([0, 3, 4, 17, 50, 89])
    rp, ci, v = oracle.column_subset((g["row_ptr"], g["col"], g["val"]), 40, cols)
    S = sps.csr_matrix((v.astype(np.int64), ci.astype(np.int64), rp.astype(np.int64)), shape=(40, len(cols)))
    assert np.array_equal(S.toarray(), M[:, cols])
    rp, ci, v = oracle.column_stripe((g["row_ptr"], g["col"], g["val"]), 40, 10, 33)
    S = sps.csr_matrix((v.astype(np.int64), ci.astype(np.int64), rp.astype(np.int64)), shape=(40, 23))
    assert np.array_equal(S.toarray(), M[:, 10:33])
