"""Seeded synthetic inputs for the Faugere-Lachartre (FL) reduction.

This module only *builds* matrices; it never reduces, solves or eliminates.
It is shared by the CPU oracle tests, the GPU parity tests and the benchmark,
and holds none of the reduction's arithmetic.

The paper's matrices (F4/F5 matrices over F_65521, Sec. 6, Table
"tab:expe:carac") are not available, so these generators reproduce their
*structure* as Sec. 3.1 and Sec. 4.2 describe it:

* every row is monic: its first nonzero entry is 1 (Sec. 3.1);
* the leading columns form a staircase; a subset of columns are pivot columns
  (Sec. 3.1, Sec. 4.1 step 1);
* nonzeros cluster to the right of the leading column (horizontal pattern) and
  consecutive rows come in runs sharing one column support (vertical pattern,
  Sec. 4.2, Fig. "multiline-illustration");
* coefficients are uniform in [1, p-1].

``fl_matrix`` additionally *plants* the Schur complement: every non-pivot row
is built as ``pivot_row[j] + sum_s x_s * pivot_row[j_s] + [0 | P_t]`` where
``P`` has a known reduced row echelon form ``V`` (rank r).  Then the FL
reduction must reach ``D - C A^{-1} B == P`` (row order of non-pivot rows in
the input) and ``RREF(D - C A^{-1} B) == V`` -- closed forms that hold at every
size, used to pin both the oracle and the device path.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

__all__ = ["CONFIGS", "BATCH_CONFIGS", "fl_matrix", "random_sparse", "dense_planted_rank",
           "csr_to_dense", "config_matrix", "batch_matrices", "config_batch", "config_batch_member"]

# Sizes of the workloads (rows x cols, pivot rows, planted rank of D, density).
CONFIGS = {
    # 2,048 x 3,072; 1,536 pivot rows; rank 384 planted in the 512 x 1,536 D.
    "c1": dict(m=2048, n=3072, npiv=1536, rank_d=384, density=0.06),
    # 60,000 x 80,000; 45,000 pivot rows; rank 12,000 in the 15,000 x 35,000 D.
    "c2": dict(m=60000, n=80000, npiv=45000, rank_d=12000, density=0.03),
    # 120,000 x 150,000; 100,000 pivot rows; rank 15,000 in the 20,000 x 50,000 D.
    "c5": dict(m=120000, n=150000, npiv=100000, rank_d=15000, density=0.015),
}
BASE_SEED = 160206097

# Batches of F4-step matrices of uneven sizes: rows log-uniform in [m_lo,
# m_hi], cols U[1.3, 1.6] x rows, pivot rows U[0.70, 0.85] x rows, density
# U[2%, 15%], planted rank U[0.5, 0.95] x min(rows of D, cols of D).
BATCH_CONFIGS = {
    "c4": dict(count=256, m_lo=500, m_hi=20000),
}


def _segment_arange(lengths: np.ndarray) -> np.ndarray:
    """Concatenation of arange(l) for every l in ``lengths``."""
    lengths = np.asarray(lengths, dtype=np.int64)
    total = int(lengths.sum())
    if total == 0:
        return np.zeros(0, dtype=np.int64)
    starts = np.cumsum(lengths) - lengths
    return np.arange(total, dtype=np.int64) - np.repeat(starts, lengths)


def _runs(total: int, lo: int, hi: int, rng) -> np.ndarray:
    """Split ``total`` items into consecutive runs with lengths in [lo, hi]."""
    if total == 0:
        return np.zeros(0, dtype=np.int64)
    lens = rng.integers(lo, hi + 1, size=total // lo + 1)
    cs = np.cumsum(lens)
    k = int(np.searchsorted(cs, total)) + 1
    lens = lens[:k].copy()
    lens[-1] -= int(cs[k - 1] - total)
    return lens[lens > 0].astype(np.int64)


def _clustered_support(bases: np.ndarray, counts: np.ndarray, limit: int,
                       rho: float, rng) -> tuple[np.ndarray, np.ndarray]:
    """For each base b, ``count`` columns b+g1, b+g1+g2, ... (geometric gaps of
    mean 1/rho), cut at ``limit``.  Returns (flat columns, per-base lengths)."""
    counts = np.asarray(counts, dtype=np.int64)
    gaps = rng.geometric(rho, size=int(counts.sum())).astype(np.int64)
    off = np.cumsum(gaps)
    seg_start = np.cumsum(counts) - counts
    prev = np.where(seg_start > 0, off[np.maximum(seg_start - 1, 0)], 0)
    off = off - np.repeat(prev, counts)
    cols = np.repeat(np.asarray(bases, dtype=np.int64), counts) + off
    keep = cols < limit
    seg_id = np.repeat(np.arange(len(counts)), counts)
    lens = np.bincount(seg_id[keep], minlength=len(counts)).astype(np.int64)
    return cols[keep], lens


def _csr(rows: int, cols: int, indptr, indices, data, p: int) -> sp.csr_matrix:
    a = sp.csr_matrix((np.asarray(data, dtype=np.int64) % p,
                       np.asarray(indices, dtype=np.int64),
                       np.asarray(indptr, dtype=np.int64)), shape=(rows, cols))
    a.sort_indices()
    return a


def _modp(a: sp.csr_matrix, p: int) -> sp.csr_matrix:
    a = a.tocsr()
    a.sum_duplicates()
    a.data %= p
    a.eliminate_zeros()
    a.sort_indices()
    return a


def _spmm_mod(a: sp.csr_matrix, b: sp.csr_matrix, p: int) -> sp.csr_matrix:
    """a @ b mod p with int64 sums that cannot overflow: for p >= 2^16 the
    entries of b are split into 16-bit halves (each term then stays below
    2^48, and the factors here have few terms per output entry)."""
    if p < (1 << 16):
        return _modp(a @ b, p)
    b = b.tocsr()
    lo = sp.csr_matrix((b.data & 0xFFFF, b.indices, b.indptr), shape=b.shape)
    hi = sp.csr_matrix((b.data >> 16, b.indices, b.indptr), shape=b.shape)
    h = _modp(a @ hi, p)
    h.data = (h.data << 16) % p
    return _modp(h + _modp(a @ lo, p), p)


def _vtype(p: int):
    """Storage type of residues: uint16 below 2^16, else uint32."""
    return np.uint16 if p <= (1 << 16) else np.uint32


def _pack(a: sp.csr_matrix, p: int = 2) -> dict:
    a = a.tocsr()
    a.sort_indices()
    return dict(m=a.shape[0], n=a.shape[1],
                row_ptr=a.indptr.astype(np.uint64),
                col=a.indices.astype(np.uint32),
                val=a.data.astype(_vtype(p)))


def _axpy_mod(d: np.ndarray, x: int, v: np.ndarray, p: int) -> np.ndarray:
    """(d + x v) mod p elementwise for residues (uint64: no overflow for p < 2^32)."""
    return (d.astype(np.uint64) + (np.uint64(x) * v.astype(np.uint64)) % np.uint64(p)) % np.uint64(p)


def fl_matrix(m: int, n: int, npiv: int, rank_d: int, density: float, p: int,
              seed: int, rho_loc: float = 0.3, v_density: float | None = None,
              run_lo: int = 2, run_hi: int = 8, shuffle_runs: bool = True) -> dict:
    """An FL matrix with a planted Schur complement (see module docstring).

    ``density`` is the target density of the whole matrix.  Returns a dict with
    the CSR input (``row_ptr`` u64, ``col`` u32, ``val`` u16, ``m``, ``n``,
    ``p``) and the plant: ``piv_cols`` (pivot columns, ascending),
    ``nonpiv_cols``, ``Dt`` (planted D - C A^{-1} B as scipy CSR in non-pivot
    column index space, rows in input order of the non-pivot rows), ``V`` (its
    RREF, scipy CSR), ``rank_d`` and ``plant_ok`` (the pivot-row selection rule
    picks the planted pivot rows; when False only rank/RREF(M) pins apply).
    """
    rng = np.random.default_rng(seed)
    assert 1 <= npiv <= min(m, n) and 0 <= rank_d <= min(m - npiv, n - npiv)
    nB, mD = n - npiv, m - npiv

    # Pivot columns: column 0 plus a uniform subset (the staircase of leads).
    piv = np.sort(np.concatenate([[0], 1 + rng.choice(n - 1, npiv - 1, replace=False)]))
    is_piv = np.zeros(n, dtype=bool)
    is_piv[piv] = True
    nonpiv = np.nonzero(~is_piv)[0]

    # Planted V (rank_d x nB) in RREF: pivots q, 1 at q_k, zero at other q,
    # clustered entries right of q_k.
    r = rank_d
    q = np.sort(rng.choice(nB, r, replace=False)) if r > 0 else np.zeros(0, np.int64)
    if v_density is None:
        v_density = min(0.5, density)
    kv = max(1, int(round(v_density * nB)))
    vc, vlen = _clustered_support(q, np.full(r, kv), nB, rho_loc, rng)
    is_q = np.zeros(nB, dtype=bool)
    is_q[q] = True
    keep = ~is_q[vc]
    seg = np.repeat(np.arange(r), vlen)
    vc = vc[keep]
    vlen = np.bincount(seg[keep], minlength=r).astype(np.int64)
    v_ptr = np.zeros(r + 1, dtype=np.int64)
    np.cumsum(vlen + 1, out=v_ptr[1:])
    v_col = np.empty(int(v_ptr[-1]), dtype=np.int64)
    v_val = rng.integers(1, p, size=len(v_col), dtype=np.int64)
    v_col[v_ptr[:-1]] = q
    v_val[v_ptr[:-1]] = 1
    vi = _segment_arange(vlen)
    v_col[np.repeat(v_ptr[:-1] + 1, vlen) + vi] = vc
    V = _csr(r, nB, v_ptr, v_col, v_val, p)
    del vc, v_col, v_val, vi, seg, keep

    # P = [(I + N) V ; W V], rows shuffled: rank r, RREF(P) = V.
    rows_t, cols_t, vals_t = [np.arange(r)], [np.arange(r)], [np.ones(r, np.int64)]
    if r > 1:  # N: strictly upper, up to 3 nearby terms per row
        nn = rng.integers(0, 4, size=r)
        ri = np.repeat(np.arange(r), nn)
        ci = ri + rng.integers(1, 64, size=len(ri))
        ok = ci < r
        rows_t.append(ri[ok]); cols_t.append(ci[ok])
        vals_t.append(rng.integers(1, p, size=int(ok.sum())))
    extra = mD - r
    if extra > 0 and r > 0:  # W: 2..8 terms per dependent row
        nw = rng.integers(2, 9, size=extra)
        ri = r + np.repeat(np.arange(extra), nw)
        rows_t.append(ri); cols_t.append(rng.integers(0, r, size=len(ri)))
        vals_t.append(rng.integers(1, p, size=len(ri)))
    T = sp.csr_matrix((np.concatenate(vals_t), (np.concatenate(rows_t), np.concatenate(cols_t))),
                      shape=(mD, r))
    P = _spmm_mod(T, V, p) if r > 0 else sp.csr_matrix((mD, nB), dtype=np.int64)
    P = _modp(P[rng.permutation(mD)], p)

    # Pivot rows, in runs sharing one clustered support right of the run's
    # last lead: row t of a run = {lead_t, ..., lead_last} U support.  The
    # support length is chosen so that the whole matrix lands near `density`
    # (a non-pivot row holds about two pivot rows' worth of entries plus P_t).
    k_row = (density * m * n - P.nnz) / (npiv + 2.0 * mD)
    k_row = max(1, int(round(k_row)))
    run_len = _runs(npiv, run_lo, run_hi, rng)
    run_start = np.cumsum(run_len) - run_len
    run_last_lead = piv[run_start + run_len - 1]
    s_cols, s_len = _clustered_support(run_last_lead, np.full(len(run_len), k_row),
                                       n, rho_loc, rng)
    s_off = np.cumsum(s_len) - s_len
    run_of = np.repeat(np.arange(len(run_len)), run_len)
    lead_cnt = (run_start + run_len)[run_of] - np.arange(npiv)
    row_len = lead_cnt + s_len[run_of]
    piv_ptr = np.zeros(npiv + 1, dtype=np.int64)
    np.cumsum(row_len, out=piv_ptr[1:])
    piv_col = np.empty(int(piv_ptr[-1]), dtype=np.int32)
    li = _segment_arange(lead_cnt)
    piv_col[np.repeat(piv_ptr[:-1], lead_cnt) + li] = piv[np.repeat(np.arange(npiv), lead_cnt) + li]
    del li
    sl = s_len[run_of]
    si = _segment_arange(sl)
    piv_col[np.repeat(piv_ptr[:-1] + lead_cnt, sl) + si] = s_cols[np.repeat(s_off[run_of], sl) + si]
    del si, s_cols
    piv_val = rng.integers(1, p, size=len(piv_col), dtype=np.int32 if p < (1 << 31) else np.int64)
    piv_val[piv_ptr[:-1]] = 1  # monic
    PIV = sp.csr_matrix((piv_val, piv_col, piv_ptr), shape=(npiv, n))
    del piv_col, piv_val

    # Non-pivot rows: pivot_row[j] + x1 pivot_row[j1] (+ x2 pivot_row[j2]) + [0|P_t],
    # in runs of consecutive rows sharing (j, j1, j2).  The lead stays piv[j]
    # with coefficient 1 because every other term starts right of piv[j].
    p_first = np.full(mD, nB, dtype=np.int64)
    nz_rows = np.diff(P.indptr) > 0
    p_first[nz_rows] = P.indices[P.indptr[:-1][nz_rows]]
    p_first_orig = np.full(mD, n, dtype=np.int64)
    if nB:
        p_first_orig[nz_rows] = nonpiv[p_first[nz_rows]]
    jmax = np.searchsorted(piv, p_first_orig, side="left") - 1  # piv[jmax] < first col
    crun = _runs(mD, run_lo, run_hi, rng)
    crun_of = np.repeat(np.arange(len(crun)), crun)
    crun_jmax = np.full(len(crun), npiv - 1, dtype=np.int64)
    np.minimum.at(crun_jmax, crun_of, jmax)
    win = 48
    base = np.maximum(crun_jmax - rng.integers(0, win, size=len(crun)), 0)
    j0 = base[crun_of]
    n_extra = rng.integers(1, 3, size=len(crun))  # 1..2 further pivot rows per run
    j1 = np.minimum(base + rng.integers(1, win, size=len(crun)), npiv - 1)[crun_of]
    j2 = np.minimum(base + rng.integers(1, win, size=len(crun)), npiv - 1)[crun_of]
    use2 = (n_extra == 2)[crun_of]
    x1 = rng.integers(1, p, size=mD)
    x2 = rng.integers(1, p, size=mD)
    srow = np.concatenate([np.arange(mD), np.arange(mD), np.nonzero(use2)[0]])
    scol = np.concatenate([j0, j1, j2[use2]])
    sval = np.concatenate([np.ones(mD, np.int64), x1, x2[use2]])
    keep = (scol > j0[srow]) | (np.arange(len(srow)) < mD)  # extra terms strictly after j0
    S = sp.csr_matrix((sval[keep], (srow[keep], scol[keep])), shape=(mD, npiv))
    Pexp = sp.csr_matrix((P.data, nonpiv[P.indices] if nB else P.indices, P.indptr), shape=(mD, n))
    PIV64 = sp.csr_matrix((PIV.data.astype(np.int64), PIV.indices, PIV.indptr), shape=PIV.shape)
    CD = _modp(_spmm_mod(S, PIV64, p) + Pexp, p)
    del PIV64, Pexp

    # Selection rule check: min (nnz, index) among rows sharing a lead must be
    # the planted pivot row, which is guaranteed when nnz is strictly larger.
    cd_nnz = np.diff(CD.indptr)
    piv_nnz = np.diff(PIV.indptr)
    plant_ok = bool(np.all(cd_nnz > piv_nnz[j0]))

    # Row order: shuffled blocks (pivot runs and non-pivot runs stay
    # consecutive).  Each block is one contiguous slice of its source CSR.
    cstart = np.cumsum(crun) - crun
    kinds = np.concatenate([np.zeros(len(run_len), np.int8), np.ones(len(crun), np.int8)])
    starts = np.concatenate([run_start, cstart]).astype(np.int64)
    lens = np.concatenate([run_len, crun]).astype(np.int64)
    order = rng.permutation(len(kinds)) if shuffle_runs else np.arange(len(kinds))
    srcs = (PIV, CD)
    row_len_out = np.empty(m, dtype=np.int64)
    pos = 0
    for b in order:
        s, l, a = starts[b], lens[b], srcs[kinds[b]]
        row_len_out[pos:pos + l] = np.diff(a.indptr[s:s + l + 1])
        pos += l
    row_ptr = np.zeros(m + 1, dtype=np.uint64)
    np.cumsum(row_len_out, out=row_ptr[1:])
    col = np.empty(int(row_ptr[-1]), dtype=np.uint32)
    val = np.empty(int(row_ptr[-1]), dtype=_vtype(p))
    dst = 0
    cd_order = []
    for b in order:
        s, l, a = starts[b], lens[b], srcs[kinds[b]]
        lo, hi = int(a.indptr[s]), int(a.indptr[s + l])
        col[dst:dst + hi - lo] = a.indices[lo:hi]
        val[dst:dst + hi - lo] = a.data[lo:hi]
        dst += hi - lo
        if kinds[b] == 1:
            cd_order.append(np.arange(s, s + l))
    cd_order = np.concatenate(cd_order) if cd_order else np.zeros(0, np.int64)
    Dt = P[cd_order] if mD else P
    return dict(m=m, n=n, row_ptr=row_ptr, col=col, val=val, p=p,
                piv_cols=piv.astype(np.uint32), nonpiv_cols=nonpiv.astype(np.uint32),
                Dt=Dt.tocsr(), V=V, rank_d=r, plant_ok=plant_ok, npiv=npiv, seed=seed)


def config_matrix(name: str, p: int = 65521, seed: int | None = None) -> dict:
    """The named workload (``c1``, ``c2``, ``c5``) with its default seed."""
    cfg = CONFIGS[name]
    if seed is None:
        seed = BASE_SEED + int(name[1:])
    return fl_matrix(p=p, seed=seed, **cfg)


def random_sparse(m: int, n: int, density: float, p: int, seed: int,
                  monic: bool = False, zero_rows: float = 0.0,
                  dup_rows: float = 0.0) -> dict:
    """Unstructured random sparse matrix (no plant): entries uniform in
    [1, p-1], optional monic rows, empty rows and duplicated rows (which create
    ties in the pivot-row selection)."""
    rng = np.random.default_rng(seed)
    mask = rng.random((m, n)) < density
    vals = rng.integers(1, p, size=(m, n)) * mask
    if zero_rows > 0:
        vals[rng.random(m) < zero_rows] = 0
    if dup_rows > 0 and m > 1:
        for i in np.nonzero(rng.random(m) < dup_rows)[0]:
            vals[i] = vals[rng.integers(0, m)]
    if monic:
        for i in range(m):
            nz = np.nonzero(vals[i])[0]
            if len(nz):
                vals[i, nz[0]] = 1
    a = sp.csr_matrix(vals.astype(np.int64))
    out = _pack(_modp(a, p), p)
    out.update(p=p)
    return out


def dense_planted_rank(rows: int, cols: int, rank: int, p: int, seed: int) -> dict:
    """Dense rows x cols matrix over F_p with rank ``rank`` and known RREF:
    D = T [V ; 0] with V a random RREF (rank x cols) and T a random invertible
    row mix (unit lower triangular times a permutation)."""
    rng = np.random.default_rng(seed)
    q = np.sort(rng.choice(cols, rank, replace=False))
    V = rng.integers(0, p, size=(rank, cols), dtype=np.int64)
    for k in range(rank):
        V[k, :q[k]] = 0
    V[:, q] = 0
    V[np.arange(rank), q] = 1
    # rows: the first `rank` rows are V mixed by a unit lower triangular
    # matrix with a few terms; the rest are random combinations of V rows.
    D = np.zeros((rows, cols), dtype=np.int64)
    D[:rank] = V
    for k in range(1, rank):
        js = rng.integers(0, k, size=min(k, 3))
        for j in js:
            D[k] = _axpy_mod(D[k], int(rng.integers(1, p)), D[j], p)
    for i in range(rank, rows):
        js = rng.integers(0, max(rank, 1), size=4) if rank else []
        for j in js:
            D[i] = _axpy_mod(D[i], int(rng.integers(1, p)), V[j], p)
    D = D[rng.permutation(rows)]
    return dict(D=D.astype(_vtype(p)), V=V.astype(_vtype(p)), pivcols=q.astype(np.uint32),
                rank=rank, p=p)


def csr_to_dense(mat: dict) -> np.ndarray:
    """Dense copy (the value type of the CSR dict) of a CSR dict (tiny inputs only)."""
    m, n = mat["m"], mat["n"]
    out = np.zeros((m, n), dtype=mat["val"].dtype)
    rp = mat["row_ptr"].astype(np.int64)
    for i in range(m):
        out[i, mat["col"][rp[i]:rp[i + 1]]] = mat["val"][rp[i]:rp[i + 1]]
    return out


def _batch_member(args) -> dict:
    i, m_lo, m_hi, p, seed = args
    s = seed ^ (i << 32)
    rng = np.random.default_rng(s)
    m = int(round(np.exp(rng.uniform(np.log(m_lo), np.log(m_hi)))))
    n = int(round(rng.uniform(1.3, 1.6) * m))
    npiv = int(round(rng.uniform(0.70, 0.85) * m))
    density = float(rng.uniform(0.02, 0.15))
    mD, nB = m - npiv, n - npiv
    r = int(np.floor(rng.uniform(0.5, 0.95) * min(mD, nB)))
    return fl_matrix(m=m, n=n, npiv=npiv, rank_d=r, density=density, p=p, seed=s + 1)


def batch_matrices(count: int, m_lo: int, m_hi: int, p: int, seed: int, workers: int = 1) -> list:
    """``count`` planted FL matrices with the batch size distribution (see
    ``BATCH_CONFIGS``); matrix i is drawn from seed ``seed ^ (i << 32)``, so
    the list does not depend on ``workers`` (processes building matrices
    concurrently)."""
    jobs = [(i, m_lo, m_hi, p, seed) for i in range(count)]
    if workers <= 1:
        return [_batch_member(j) for j in jobs]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_batch_member, jobs, chunksize=1)


def config_batch(name: str, p: int = 65521, seed: int | None = None, workers: int = 1) -> list:
    """The named batch workload (``c4``) with its default seed."""
    cfg = BATCH_CONFIGS[name]
    if seed is None:
        seed = BASE_SEED + int(name[1:])
    return batch_matrices(p=p, seed=seed, workers=workers, **cfg)


def config_batch_member(name: str, i: int, p: int = 65521, seed: int | None = None) -> dict:
    """Matrix ``i`` of the named batch workload alone (equal to
    ``config_batch(name)[i]``)."""
    cfg = BATCH_CONFIGS[name]
    if seed is None:
        seed = BASE_SEED + int(name[1:])
    return _batch_member((i, cfg["m_lo"], cfg["m_hi"], p, seed))
