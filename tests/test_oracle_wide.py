"""Pins of the CPU oracle for 32-bit field characteristic (uint32 residues,
fl_oracle_wide.c) -- no GPU.

  * for p < 2^16 it equals the uint16 oracle (itself pinned by brute force
    and the planted forms) on every intermediate and output;
  * for 32-bit primes its RREF(M) equals pure-Python Gauss-Jordan on the
    whole matrix (arbitrary-precision integers) on small random matrices,
    empty and duplicate rows included;
  * on planted FL matrices over 32-bit primes: D - C A^{-1} B equals the
    planted Schur complement, its RREF the planted V, and the rank
    npiv + planted rank; A X = B and D - C X = Dt by products in exact
    integers.
"""
import numpy as np
import pytest

import flgen
import oracle
from oracle.bruteforce import rref_lists

BIG = [4294967291, 4294967279, 2147483647, 65537, 1000000007]


def _dense_obj(csr, rows, cols):
    rp, ci, v = csr
    out = np.zeros((rows, cols), dtype=object)
    rp = rp.astype(np.int64)
    for i in range(rows):
        for k in range(rp[i], rp[i + 1]):
            out[i, int(ci[k])] = int(v[k])
    return out


def _as_wide(g):
    h = dict(g)
    h["val"] = g["val"].astype(np.uint32)
    return h


@pytest.mark.parametrize("p", [65521, 251, 7, 2])
def test_wide_equals_narrow_below_2_16(p):
    mats = [flgen.fl_matrix(m=300, n=420, npiv=200, rank_d=60, density=0.06, p=p, seed=11),
            flgen.random_sparse(90, 130, 0.08, p, seed=12, zero_rows=0.1, dup_rows=0.1)]
    for g in mats:
        a = oracle.fl_rref(g)
        b = oracle.fl_rref_wide(_as_wide(g))
        assert a["rank"] == b["rank"]
        assert np.array_equal(a["X"].astype(np.uint32), b["X"])
        assert np.array_equal(a["Dt"].astype(np.uint32), b["Dt"])
        assert np.array_equal(a["RD"].astype(np.uint32), b["RD"])
        assert np.array_equal(a["pivcols"], b["pivcols"])
        assert np.array_equal(a["Xp"].astype(np.uint32), b["Xp"])
        for x, y in zip(a["rref"], b["rref"]):
            assert np.array_equal(x.astype(np.uint64), y.astype(np.uint64))


@pytest.mark.parametrize("p", BIG + [3])
def test_wide_equals_bruteforce_32bit(p):
    rng = np.random.default_rng(p % 1000)
    for trial in range(12):
        m, n = int(rng.integers(1, 9)), int(rng.integers(1, 11))
        g = flgen.random_sparse(m, n, float(rng.uniform(0.2, 0.8)), p, seed=1000 * trial + 7,
                                zero_rows=0.15, dup_rows=0.15)
        if g["val"].dtype != np.uint32:
            g = _as_wide(g)
        res = oracle.fl_rref_wide(g)
        rows = _dense_obj((g["row_ptr"], g["col"], g["val"]), m, n).tolist()
        R, piv = rref_lists([[int(x) for x in r] for r in rows], p)
        assert res["rank"] == len(piv)
        rp, ci, v = res["rref"]
        got = _dense_obj((rp, ci, v), res["rank"], n)
        for i in range(len(R)):
            assert [int(x) for x in got[i]] == R[i], (p, trial, i)


def test_wide_inverse_and_validation():
    lib = oracle._load()
    for p in BIG:
        for a in (1, 2, 3, p - 1, p // 2, 123456789 % p):
            if a % p:
                assert (int(lib.ow_inv(a, p)) * a) % p == 1
    g = flgen.random_sparse(10, 12, 0.3, 4294967291, seed=3)
    assert oracle.validate_wide(g) == oracle.OR_OK
    bad = dict(g)
    v = g["val"].copy()
    v[0] = 4294967291          # == p
    bad["val"] = v
    assert oracle.validate_wide(bad) == oracle.OR_BAD_VALUE


@pytest.mark.parametrize("p", [4294967291, 2147483647])
def test_wide_planted_and_block_identities(p):
    g = flgen.fl_matrix(m=500, n=700, npiv=360, rank_d=100, density=0.05, p=p, seed=21)
    assert g["plant_ok"]
    r = oracle.fl_rref_wide(g)
    s = r["split"]
    npiv, mD, nB = s["npiv"], s["mD"], s["nB"]
    assert npiv == 360 and r["rank"] == npiv + g["rank_d"]
    assert np.array_equal(r["Dt"], g["Dt"].toarray().astype(np.uint32))
    assert np.array_equal(r["RD"], g["V"].toarray().astype(np.uint32))
    # A X = B and D - C X = Dt in exact integers
    A = _dense_obj(s["A"], npiv, npiv)
    B = _dense_obj(s["B"], npiv, nB)
    C = _dense_obj(s["C"], mD, npiv)
    D = _dense_obj(s["D"], mD, nB)
    X = r["X"].astype(object)
    assert ((A.dot(X) - B) % p == 0).all()
    assert ((D - C.dot(X) - r["Dt"].astype(object)) % p == 0).all()
