"""Certificate that a CSR matrix R is the reduced row echelon form of M.

Uses only M and R (no oracle, no device code):
  1. R is in RREF: every row starts with a 1 at its pivot column, pivots
     strictly increase, and each pivot column of R is a unit vector;
  2. rowspace(M) is contained in rowspace(R): since R is in RREF, row i of M
     must equal sum_t M[i, piv_t] * R_t, checked with random vectors
     (Freivalds): M x == M[:, piv] (R x) mod p; a false pass has probability
     at most p^-k for k vectors;
  3. the number of rows of R equals the known rank of M.
Together with uniqueness of the RREF this pins R = RREF(M).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def csr(mat_rp, ci, v, rows, cols):
    return sp.csr_matrix((np.asarray(v, np.int64), np.asarray(ci, np.int64),
                          np.asarray(mat_rp, np.int64)), shape=(rows, cols))


def certify_rref(M: sp.csr_matrix, R: sp.csr_matrix, p: int, rank: int, trials: int = 4,
                 seed: int = 1) -> None:
    assert R.shape[0] == rank, f"rows {R.shape[0]} != rank {rank}"
    n = M.shape[1]
    rp = R.indptr
    assert np.all(np.diff(rp) > 0), "empty row in RREF"
    piv = R.indices[rp[:-1]]
    assert np.all(R.data[rp[:-1]] == 1), "leading entry not 1"
    assert np.all(np.diff(piv.astype(np.int64)) > 0), "pivots not increasing"
    assert np.all((R.data > 0) & (R.data < p)), "entry out of range"
    colcount = np.bincount(R.indices, minlength=n)
    assert np.all(colcount[piv] == 1), "pivot column is not a unit vector"
    rng = np.random.default_rng(seed)
    Mp = M[:, piv].tocsr() if rank else None
    for _ in range(trials):
        x = rng.integers(0, p, size=n, dtype=np.int64)
        lhs = (M @ x) % p
        if rank:
            rx = (R @ x) % p
            rhs = (Mp @ rx) % p
        else:
            rhs = np.zeros(M.shape[0], np.int64)
        assert np.array_equal(lhs, rhs), "a row of M is not in rowspace(R)"
