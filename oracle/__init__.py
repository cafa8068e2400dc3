"""CPU oracle of the FL reduction -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
import this package.  The device library never loads, links or calls it, and
the two share no code.

``fl_oracle_wide.c`` holds the same steps for uint32 residues (32-bit
primes; every product reduced at once).  ``fl_oracle.c`` holds the plain FL steps (Sec. 4.1 of the paper, plus the new
order of operations of Sec. 4.3 as an independent route to the Schur
complement); ``bruteforce.c`` is direct Gauss-Jordan on the whole matrix;
``bruteforce.py`` is pure-Python Gauss-Jordan for tiny inputs.  This module
compiles the C files with gcc (``build()``) and marshals numpy arrays.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["fl_oracle.c", "fl_oracle_wide.c", "bruteforce.c"]
_lib = None

P_U64 = ct.POINTER(ct.c_uint64)
P_U32 = ct.POINTER(ct.c_uint32)
P_U16 = ct.POINTER(ct.c_uint16)

# or_validate codes
OR_OK, OR_BAD_P, OR_BAD_ROWPTR, OR_COL_RANGE, OR_COL_ORDER, OR_BAD_VALUE = range(6)


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP)."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-o", _LIB_PATH] + srcs
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ct.CDLL(_LIB_PATH)
    lib.or_inv.restype = ct.c_uint32
    lib.or_inv.argtypes = [ct.c_uint32, ct.c_uint32]
    lib.or_validate.restype = ct.c_int
    lib.or_validate.argtypes = [ct.c_uint32, ct.c_uint32, P_U64, P_U32, P_U16, ct.c_uint32]
    lib.or_split.restype = ct.c_uint32
    lib.or_split.argtypes = [ct.c_uint32, ct.c_uint32, P_U64, P_U32, P_U16, ct.c_uint32,
                             P_U32, P_U32] + [P_U64, P_U32, P_U16] * 4
    lib.or_multiline.restype = None
    lib.or_multiline.argtypes = [ct.c_uint32, ct.c_uint32, P_U64, P_U32, P_U16, ct.c_uint32,
                                 P_U64, P_U32, P_U16]
    lib.or_trsm.restype = ct.c_int
    lib.or_trsm.argtypes = [ct.c_uint32, ct.c_uint32, P_U64, P_U32, P_U16, P_U64, P_U32, P_U16,
                            ct.c_uint32, P_U16, ct.c_uint64]
    lib.or_reduce.restype = None
    lib.or_reduce.argtypes = [ct.c_uint32, ct.c_uint32, P_U64, P_U32, P_U16, P_U64, P_U32, P_U16,
                              P_U16, ct.c_uint64, ct.c_uint32, P_U16, ct.c_uint64]
    lib.or_reduce_neworder.restype = None
    lib.or_reduce_neworder.argtypes = [ct.c_uint32] * 3 + [P_U64, P_U32, P_U16] * 4 + \
        [ct.c_uint32, P_U16, ct.c_uint64]
    lib.or_rref_dense.restype = ct.c_uint32
    lib.or_rref_dense.argtypes = [ct.c_uint32, ct.c_uint32, P_U16, ct.c_uint64, ct.c_uint32, P_U32]
    lib.or_second_pass.restype = None
    lib.or_second_pass.argtypes = [ct.c_uint32, ct.c_uint32, P_U16, ct.c_uint64, ct.c_uint32,
                                   P_U16, ct.c_uint64, P_U32, ct.c_uint32]
    lib.or_assemble.restype = ct.c_uint64
    lib.or_assemble.argtypes = [ct.c_uint32, ct.c_uint32, ct.c_uint32, P_U32, P_U16, ct.c_uint64,
                                ct.c_uint32, P_U16, ct.c_uint64, P_U32, P_U64, P_U32, P_U16]
    lib.ow_inv.restype = ct.c_uint32
    lib.ow_inv.argtypes = [ct.c_uint32, ct.c_uint32]
    lib.ow_validate.restype = ct.c_int
    lib.ow_validate.argtypes = [ct.c_uint32, ct.c_uint32, P_U64, P_U32, P_U32, ct.c_uint32]
    lib.ow_split.restype = ct.c_uint32
    lib.ow_split.argtypes = [ct.c_uint32, ct.c_uint32, P_U64, P_U32, P_U32, ct.c_uint32,
                             P_U32, P_U32] + [P_U64, P_U32, P_U32] * 4
    lib.ow_trsm.restype = ct.c_int
    lib.ow_trsm.argtypes = [ct.c_uint32, ct.c_uint32, P_U64, P_U32, P_U32, P_U64, P_U32, P_U32,
                            ct.c_uint32, P_U32, ct.c_uint64]
    lib.ow_reduce.restype = None
    lib.ow_reduce.argtypes = [ct.c_uint32, ct.c_uint32, P_U64, P_U32, P_U32, P_U64, P_U32, P_U32,
                              P_U32, ct.c_uint64, ct.c_uint32, P_U32, ct.c_uint64]
    lib.ow_rref_dense.restype = ct.c_uint32
    lib.ow_rref_dense.argtypes = [ct.c_uint32, ct.c_uint32, P_U32, ct.c_uint64, ct.c_uint32, P_U32]
    lib.ow_second_pass.restype = None
    lib.ow_second_pass.argtypes = [ct.c_uint32, ct.c_uint32, P_U32, ct.c_uint64, ct.c_uint32,
                                   P_U32, ct.c_uint64, P_U32, ct.c_uint32]
    lib.ow_assemble.restype = ct.c_uint64
    lib.ow_assemble.argtypes = [ct.c_uint32, ct.c_uint32, ct.c_uint32, P_U32, P_U32, ct.c_uint64,
                                ct.c_uint32, P_U32, ct.c_uint64, P_U32, P_U64, P_U32, P_U32]
    lib.bf_rref_csr.restype = ct.c_uint64
    lib.bf_rref_csr.argtypes = [ct.c_uint32, ct.c_uint32, P_U64, P_U32, P_U16, ct.c_uint32, P_U32,
                                P_U64, P_U32, P_U16]
    _lib = lib
    return lib


def _p(a, t):
    if a is None:
        return ct.cast(None, t)
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(t)


def _csr_args(rp, ci, v):
    return [_p(rp, P_U64), _p(ci, P_U32), _p(v, P_U16)]


def inv(a: int, p: int) -> int:
    return int(_load().or_inv(a, p))


def validate(mat: dict) -> int:
    lib = _load()
    return int(lib.or_validate(mat["m"], mat["n"], *_csr_args(mat["row_ptr"], mat["col"], mat["val"]),
                               mat["p"]))


def split(mat: dict) -> dict:
    """FL step 1.  Returns npiv, col_perm, row_perm and A, B, C, D as CSR
    triples (row_ptr, col, val) over the new column indices."""
    lib = _load()
    m, n, p = mat["m"], mat["n"], mat["p"]
    nnz = int(mat["row_ptr"][-1])
    col_perm = np.zeros(n, np.uint32)
    row_perm = np.zeros(m, np.uint32)
    bufs = []
    for _ in range(4):
        bufs.append((np.zeros(m + 1, np.uint64), np.zeros(max(nnz, 1), np.uint32),
                     np.zeros(max(nnz, 1), np.uint16)))
    args = []
    for b in bufs:
        args += _csr_args(*b)
    npiv = int(lib.or_split(m, n, *_csr_args(mat["row_ptr"], mat["col"], mat["val"]), p,
                            _p(col_perm, P_U32), _p(row_perm, P_U32), *args))
    mD, nB = m - npiv, n - npiv
    rows = [npiv, npiv, mD, mD]
    out = dict(npiv=npiv, mD=mD, nB=nB, m=m, n=n, p=p, col_perm=col_perm, row_perm=row_perm)
    for name, b, r in zip("ABCD", bufs, rows):
        rp = b[0][:r + 1].copy()
        k = int(rp[-1])
        out[name] = (rp, b[1][:k].copy(), b[2][:k].copy())
    return out


def multiline(csr, rows: int, cols: int, w: int):
    """n-multiline packing (Sec. 4.2) of a CSR triple; returns (gptr, pos, val)."""
    lib = _load()
    rp, ci, v = csr
    ngroups = (rows + w - 1) // w
    nnz = int(rp[rows]) if rows else 0
    gptr = np.zeros(ngroups + 1, np.uint64)
    pos = np.zeros(max(nnz, 1), np.uint32)
    val = np.zeros(max(nnz * w, 1), np.uint16)
    lib.or_multiline(rows, cols, *_csr_args(rp, ci, v), w, _p(gptr, P_U64), _p(pos, P_U32),
                     _p(val, P_U16))
    L = int(gptr[-1])
    return gptr, pos[:L].copy(), val[:L * w].copy()


def column_stripe(csr, rows: int, c0: int, c1: int):
    """Columns [c0, c1) of a CSR triple, relabelled to [0, c1 - c0)."""
    rp, ci, v = csr
    keep = (ci >= c0) & (ci < c1)
    cs = np.zeros(len(ci) + 1, np.int64)
    np.cumsum(keep, out=cs[1:])
    nrp = cs[rp.astype(np.int64)].astype(np.uint64)
    return nrp, (ci[keep] - c0).astype(np.uint32), v[keep].copy()


def column_subset(csr, rows: int, cols: np.ndarray):
    """The columns `cols` (ascending) of a CSR triple, column cols[k]
    relabelled to k."""
    rp, ci, v = csr
    cols = np.asarray(cols, np.int64)
    lut = np.full(int(max(cols.max() + 1 if len(cols) else 0, ci.max() + 1 if len(ci) else 0)), -1, np.int64)
    lut[cols] = np.arange(len(cols))
    new = lut[ci.astype(np.int64)] if len(ci) else np.zeros(0, np.int64)
    keep = new >= 0
    cs = np.zeros(len(ci) + 1, np.int64)
    np.cumsum(keep, out=cs[1:])
    nrp = cs[rp.astype(np.int64)].astype(np.uint64)
    return nrp, new[keep].astype(np.uint32), v[keep].copy()


def trsm(s: dict, threads: int = 1) -> np.ndarray:
    """X = A^{-1} B.  With threads > 1 the columns of B are cut into that
    many stripes, each solved by its own call of the same back substitution
    in a thread of its own (the columns of X are independent, Sec. 4.2)."""
    lib = _load()
    npiv, nB = s["npiv"], s["nB"]
    X = np.zeros((npiv, nB), np.uint16)
    if npiv == 0:
        return X
    if threads <= 1 or nB < 2 * threads:
        rc = lib.or_trsm(npiv, nB, *_csr_args(*s["A"]), *_csr_args(*s["B"]), s["p"],
                         _p(X, P_U16), max(nB, 1))
        assert rc == 0, "A is not unit upper triangular"
        return X
    import concurrent.futures as cf
    edges = np.linspace(0, nB, threads + 1).astype(np.int64)

    def solve(k):
        c0, c1 = int(edges[k]), int(edges[k + 1])
        Bs = column_stripe(s["B"], npiv, c0, c1)
        Xs = np.zeros((npiv, c1 - c0), np.uint16)
        rc = lib.or_trsm(npiv, c1 - c0, *_csr_args(*s["A"]), *_csr_args(*Bs), s["p"], _p(Xs, P_U16),
                         max(c1 - c0, 1))
        assert rc == 0, "A is not unit upper triangular"
        X[:, c0:c1] = Xs

    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(solve, range(threads)))
    return X


def reduce(s: dict, X: np.ndarray) -> np.ndarray:
    lib = _load()
    Dt = np.zeros((s["mD"], s["nB"]), np.uint16)
    if s["mD"] == 0:
        return Dt
    X = np.ascontiguousarray(X)
    lib.or_reduce(s["mD"], s["nB"], *_csr_args(*s["C"]), *_csr_args(*s["D"]), _p(X, P_U16),
                  max(X.shape[1], 1), s["p"], _p(Dt, P_U16), max(s["nB"], 1))
    return Dt


def reduce_neworder(s: dict) -> np.ndarray:
    lib = _load()
    Dt = np.zeros((s["mD"], s["nB"]), np.uint16)
    if s["mD"] == 0:
        return Dt
    args = []
    for k in "ABCD":
        args += _csr_args(*s[k])
    lib.or_reduce_neworder(s["npiv"], s["mD"], s["nB"], *args, s["p"], _p(Dt, P_U16),
                           max(s["nB"], 1))
    return Dt


def rref_dense(D: np.ndarray, p: int):
    """Returns (R, rank, pivcols): R is a copy of D with rows 0..rank-1 = RREF."""
    lib = _load()
    R = np.ascontiguousarray(D, dtype=np.uint16).copy()
    rows, cols = R.shape
    piv = np.zeros(max(min(rows, cols), 1), np.uint32)
    if rows == 0 or cols == 0:
        return R, 0, piv[:0]
    rank = int(lib.or_rref_dense(rows, cols, _p(R, P_U16), cols, p, _p(piv, P_U32)))
    return R, rank, piv[:rank].copy()


def second_pass(X: np.ndarray, R: np.ndarray, rank: int, pivcols: np.ndarray, p: int) -> np.ndarray:
    lib = _load()
    Xp = np.ascontiguousarray(X, dtype=np.uint16).copy()
    npiv, nB = Xp.shape
    if npiv == 0 or rank == 0:
        return Xp
    R = np.ascontiguousarray(R, dtype=np.uint16)
    pc = np.ascontiguousarray(pivcols, dtype=np.uint32)
    lib.or_second_pass(npiv, nB, _p(Xp, P_U16), max(nB, 1), rank, _p(R, P_U16), max(R.shape[1], 1),
                       _p(pc, P_U32), p)
    return Xp


def assemble(n: int, npiv: int, col_perm, Xp, rank: int, R, pivcols):
    """Reduced form in original column order as CSR (rows sorted by pivot)."""
    lib = _load()
    nB = n - npiv
    Xp = np.ascontiguousarray(Xp, dtype=np.uint16).reshape(npiv, nB) if npiv else np.zeros((0, nB), np.uint16)
    R = np.ascontiguousarray(R, dtype=np.uint16)
    if R.size == 0:
        R = np.zeros((1, max(nB, 1)), np.uint16)
    pc = np.ascontiguousarray(pivcols, dtype=np.uint32)
    if pc.size == 0:
        pc = np.zeros(1, np.uint32)
    cp = np.ascontiguousarray(col_perm, dtype=np.uint32)
    Xarg = Xp if Xp.size else np.zeros(1, np.uint16)
    args = [n, npiv, nB, _p(cp, P_U32), _p(Xarg, P_U16), max(nB, 1), rank, _p(R, P_U16),
            max(R.shape[1], 1), _p(pc, P_U32)]
    nnz = int(lib.or_assemble(*args, _p(None, P_U64), None, None))
    rp = np.zeros(npiv + rank + 1, np.uint64)
    ci = np.zeros(max(nnz, 1), np.uint32)
    v = np.zeros(max(nnz, 1), np.uint16)
    lib.or_assemble(*args, _p(rp, P_U64), _p(ci, P_U32), _p(v, P_U16))
    return rp, ci[:nnz].copy(), v[:nnz].copy()


def fl_rref(mat: dict, keep: bool = True, threads: int = 1) -> dict:
    """The whole oracle pipeline: split, TRSM, reduce, RREF of the Schur
    complement, second pass, read-off.  Returns every intermediate.
    threads: column stripes of the TRSM solved concurrently (see trsm)."""
    s = split(mat)
    p = mat["p"]
    X = trsm(s, threads)
    Dt = reduce(s, X)
    R, r, pc = rref_dense(Dt, p)
    Xp = second_pass(X, R, r, pc, p)
    out_csr = assemble(mat["n"], s["npiv"], s["col_perm"], Xp, r, R[:r], pc)
    res = dict(split=s, rank_d=r, pivcols=pc, rank=s["npiv"] + r, rref=out_csr)
    if keep:
        res.update(X=X, Dt=Dt, RD=R[:r].copy(), Xp=Xp)
    return res


def bruteforce_rref(mat: dict):
    """RREF(M) by Gauss-Jordan on the whole dense matrix; returns (CSR, rank)."""
    lib = _load()
    m, n, p = mat["m"], mat["n"], mat["p"]
    rank = ct.c_uint32(0)
    args = [m, n, *_csr_args(mat["row_ptr"], mat["col"], mat["val"]), p, ct.byref(rank)]
    nnz = int(lib.bf_rref_csr(*args, _p(None, P_U64), None, None))
    rp = np.zeros(rank.value + 1, np.uint64)
    ci = np.zeros(max(nnz, 1), np.uint32)
    v = np.zeros(max(nnz, 1), np.uint16)
    lib.bf_rref_csr(*args, _p(rp, P_U64), _p(ci, P_U32), _p(v, P_U16))
    return (rp, ci[:nnz].copy(), v[:nnz].copy()), rank.value


# ---- 32-bit field characteristic (uint32 residues) ---------------------------

def _csr_args32(rp, ci, v):
    return [_p(rp, P_U64), _p(ci, P_U32), _p(v, P_U32)]


def validate_wide(mat: dict) -> int:
    lib = _load()
    return int(lib.ow_validate(mat["m"], mat["n"], *_csr_args32(mat["row_ptr"], mat["col"],
                                                                 np.ascontiguousarray(mat["val"], np.uint32)),
                               mat["p"]))


def split_wide(mat: dict) -> dict:
    """FL step 1 over uint32 residues (same readings as split)."""
    lib = _load()
    m, n, p = mat["m"], mat["n"], mat["p"]
    nnz = int(mat["row_ptr"][-1])
    col_perm = np.zeros(n, np.uint32)
    row_perm = np.zeros(m, np.uint32)
    bufs = [(np.zeros(m + 1, np.uint64), np.zeros(max(nnz, 1), np.uint32), np.zeros(max(nnz, 1), np.uint32))
            for _ in range(4)]
    args = []
    for b in bufs:
        args += _csr_args32(*b)
    val = np.ascontiguousarray(mat["val"], np.uint32)
    npiv = int(lib.ow_split(m, n, *_csr_args32(mat["row_ptr"], mat["col"], val), p,
                            _p(col_perm, P_U32), _p(row_perm, P_U32), *args))
    mD, nB = m - npiv, n - npiv
    out = dict(npiv=npiv, mD=mD, nB=nB, m=m, n=n, p=p, col_perm=col_perm, row_perm=row_perm)
    for name, b, r in zip("ABCD", bufs, [npiv, npiv, mD, mD]):
        rp = b[0][:r + 1].copy()
        k = int(rp[-1])
        out[name] = (rp, b[1][:k].copy(), b[2][:k].copy())
    return out


def trsm_wide(s: dict) -> np.ndarray:
    lib = _load()
    npiv, nB = s["npiv"], s["nB"]
    X = np.zeros((npiv, nB), np.uint32)
    if npiv == 0:
        return X
    rc = lib.ow_trsm(npiv, nB, *_csr_args32(*s["A"]), *_csr_args32(*s["B"]), s["p"], _p(X, P_U32), max(nB, 1))
    assert rc == 0, "A is not unit upper triangular"
    return X


def reduce_wide(s: dict, X: np.ndarray) -> np.ndarray:
    lib = _load()
    Dt = np.zeros((s["mD"], s["nB"]), np.uint32)
    if s["mD"] == 0:
        return Dt
    X = np.ascontiguousarray(X, np.uint32)
    lib.ow_reduce(s["mD"], s["nB"], *_csr_args32(*s["C"]), *_csr_args32(*s["D"]), _p(X, P_U32),
                  max(X.shape[1], 1), s["p"], _p(Dt, P_U32), max(s["nB"], 1))
    return Dt


def rref_dense_wide(D: np.ndarray, p: int):
    """(R, rank, pivcols): R is a copy of D with rows 0..rank-1 = RREF."""
    lib = _load()
    R = np.ascontiguousarray(D, dtype=np.uint32).copy()
    rows, cols = R.shape
    piv = np.zeros(max(min(rows, cols), 1), np.uint32)
    if rows == 0 or cols == 0:
        return R, 0, piv[:0]
    rank = int(lib.ow_rref_dense(rows, cols, _p(R, P_U32), cols, p, _p(piv, P_U32)))
    return R, rank, piv[:rank].copy()


def second_pass_wide(X: np.ndarray, R: np.ndarray, rank: int, pivcols: np.ndarray, p: int) -> np.ndarray:
    lib = _load()
    Xp = np.ascontiguousarray(X, dtype=np.uint32).copy()
    npiv, nB = Xp.shape
    if npiv == 0 or rank == 0:
        return Xp
    R = np.ascontiguousarray(R, dtype=np.uint32)
    pc = np.ascontiguousarray(pivcols, dtype=np.uint32)
    lib.ow_second_pass(npiv, nB, _p(Xp, P_U32), max(nB, 1), rank, _p(R, P_U32), max(R.shape[1], 1),
                       _p(pc, P_U32), p)
    return Xp


def assemble_wide(n: int, npiv: int, col_perm, Xp, rank: int, R, pivcols):
    lib = _load()
    nB = n - npiv
    Xp = np.ascontiguousarray(Xp, dtype=np.uint32).reshape(npiv, nB) if npiv else np.zeros((0, nB), np.uint32)
    R = np.ascontiguousarray(R, dtype=np.uint32)
    if R.size == 0:
        R = np.zeros((1, max(nB, 1)), np.uint32)
    pc = np.ascontiguousarray(pivcols, dtype=np.uint32)
    if pc.size == 0:
        pc = np.zeros(1, np.uint32)
    cp = np.ascontiguousarray(col_perm, dtype=np.uint32)
    Xarg = Xp if Xp.size else np.zeros(1, np.uint32)
    args = [n, npiv, nB, _p(cp, P_U32), _p(Xarg, P_U32), max(nB, 1), rank, _p(R, P_U32),
            max(R.shape[1], 1), _p(pc, P_U32)]
    nnz = int(lib.ow_assemble(*args, _p(None, P_U64), None, None))
    rp = np.zeros(npiv + rank + 1, np.uint64)
    ci = np.zeros(max(nnz, 1), np.uint32)
    v = np.zeros(max(nnz, 1), np.uint32)
    lib.ow_assemble(*args, _p(rp, P_U64), _p(ci, P_U32), _p(v, P_U32))
    return rp, ci[:nnz].copy(), v[:nnz].copy()


def fl_rref_wide(mat: dict, keep: bool = True) -> dict:
    """The whole oracle pipeline over uint32 residues (p < 2^32)."""
    s = split_wide(mat)
    p = mat["p"]
    X = trsm_wide(s)
    Dt = reduce_wide(s, X)
    R, r, pc = rref_dense_wide(Dt, p)
    Xp = second_pass_wide(X, R, r, pc, p)
    out_csr = assemble_wide(mat["n"], s["npiv"], s["col_perm"], Xp, r, R[:r], pc)
    res = dict(split=s, rank_d=r, pivcols=pc, rank=s["npiv"] + r, rref=out_csr)
    if keep:
        res.update(X=X, Dt=Dt, RD=R[:r].copy(), Xp=Xp)
    return res
