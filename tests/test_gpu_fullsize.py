"""Parity at the full workload sizes, in the launch configuration the bench
times (multiline width 2, int8-limb MFMA form), plus the plain form.

At these sizes the oracle cannot run the whole reduction in a test, so the
device results are checked by what fixes them independently of the device
path:
  * split: the oracle's split of the same matrix, compared in full;
  * X = A^-1 B: the defining identity A X = B, exactly on sampled rows (first
    and last rows, TRSM block boundaries, a seeded sample) and on every row
    through random projections (Freivalds, false pass <= p^-2);
  * D - C X: equal to the Schur complement the generator planted;
  * RREF(D - C X): equal to the planted RREF V, with the planted rank;
  * second pass: X' = X - X[:, P_D] V on sampled rows;
  * CSR of RREF(M): RREF structure, rank rows, and rowspace(M) inside
    rowspace(R) by random projections; with uniqueness of the RREF this
    pins R = RREF(M);
  * the plain form's outputs equal the MFMA form's, bit for bit.
"""
import numpy as np
import pytest
import scipy.sparse as sps
import torch

import flgen
import oracle
import paper_1602_06097_amd as fl

pytestmark = pytest.mark.gpu

CONFIGS = ["c2", "c5"]
TRSM_BLOCK = 128


def _u16(t):
    return t.cpu().numpy().view(np.uint16)


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


def _strict_upper(A, npiv):
    rp, ci, v = A
    first = rp[:-1].astype(np.int64)
    keep = np.ones(len(ci), bool)
    keep[first] = False
    nrp = np.zeros(npiv + 1, np.uint64)
    nrp[1:] = np.cumsum(np.diff(rp.astype(np.int64)) - 1)
    return nrp, ci[keep], v[keep]


def _sp(csr3, rows, cols):
    rp, ci, v = csr3
    return sps.csr_matrix((v.astype(np.int64), ci.astype(np.int64), rp.astype(np.int64)),
                          shape=(rows, cols))


def _run(g, mode):
    d = torch.device("cuda")
    rp = torch.from_numpy(g["row_ptr"].view(np.int64)).to(d)
    ci = torch.from_numpy(g["col"].view(np.int32)).to(d)
    vv = torch.from_numpy(g["val"].view(np.int16)).to(d)
    res = fl.fl_reduce(rp, ci, vv, g["m"], g["n"], g["p"], mode=mode, ml_width=2, keep=True)
    torch.cuda.synchronize()
    return res


@pytest.fixture(scope="module", params=CONFIGS)
def full(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fl.load()
    name = request.param
    g = flgen.config_matrix(name)
    assert g["plant_ok"], "generator could not plant the pivot rows"
    s = oracle.split(g)
    res = _run(g, fl.FL_MFMA_I8)
    print(f"\n[fullsize] {name}: {g['m']}x{g['n']} nnz={len(g['col'])} rank={res['rref'][3]}", flush=True)
    yield dict(name=name, g=g, s=s, res=res)
    del res
    torch.cuda.empty_cache()


def test_fullsize_split_equals_oracle(full):
    g, s, sp = full["g"], full["s"], full["res"]["split"]
    assert (sp.npiv, sp.mD, sp.nB) == (s["npiv"], s["mD"], s["nB"])
    b = sp.bufs
    assert np.array_equal(_u32(b["row_perm"])[:g["m"]], s["row_perm"])
    assert np.array_equal(_u32(b["col_perm"])[:g["n"]], s["col_perm"])
    npiv, mD = s["npiv"], s["mD"]
    for key, rows in (("b", npiv), ("d", mD)):
        orp, oci, ov = s[key.upper()]
        k = int(orp[-1])
        assert np.array_equal(_u64(b[f"{key}_ptr"][:rows + 1]), orp)
        assert np.array_equal(_u32(b[f"{key}_col"][:k]), oci)
        assert np.array_equal(_u16(b[f"{key}_val"][:k]), ov)
    for key, csr3, rows, length in (("a", _strict_upper(s["A"], npiv), npiv, sp.info.lenA),
                                    ("c", s["C"], mD, sp.info.lenC)):
        gptr, pos, val = oracle.multiline(csr3, rows, npiv, 2)
        ng = (rows + 1) // 2
        assert length == len(pos)
        assert np.array_equal(_u64(b[f"{key}_gptr"][:ng + 1]), gptr)
        assert np.array_equal(_u32(b[f"{key}_pos"][:len(pos)]), pos)
        assert np.array_equal(_u16(b[f"{key}_val"][:len(val)]), val)


def _sample_rows(n, k, seed):
    rng = np.random.default_rng(seed)
    edges = [0, 1, n - 2, n - 1]
    for b in range(TRSM_BLOCK, n, TRSM_BLOCK * 37):
        edges += [b - 1, b]
    rows = np.concatenate([np.array([e for e in edges if 0 <= e < n], np.int64),
                           rng.integers(0, n, size=k)])
    return np.unique(rows)


def _project(Xdev, rows, cols, v, p):
    """(X v) mod p on the device, in row chunks, as int64 host array."""
    vt = torch.from_numpy(v).to(Xdev.device)
    out = torch.empty(rows, dtype=torch.int64, device=Xdev.device)
    step = max(1, (1 << 27) // max(cols, 1))
    for r0 in range(0, rows, step):
        r1 = min(rows, r0 + step)
        xc = Xdev[r0:r1, :cols].to(torch.int64) & 0xFFFF
        out[r0:r1] = (xc * vt).sum(dim=1) % p
    return out.cpu().numpy()


def test_fullsize_trsm_satisfies_AX_equals_B(full):
    s, res = full["s"], full["res"]
    npiv, nB, p = s["npiv"], s["nB"], s["p"]
    X = res["X"]
    A = _sp(s["A"], npiv, npiv)
    B = _sp(s["B"], npiv, nB)
    # exact on sampled rows: row i of A X, summed on the device from the X rows A_i touches
    rows = _sample_rows(npiv, 64, seed=5)
    for i in rows:
        lo, hi = A.indptr[i], A.indptr[i + 1]
        idx = torch.from_numpy(A.indices[lo:hi].astype(np.int64)).to(X.device)
        coef = torch.from_numpy(A.data[lo:hi].astype(np.int64)).to(X.device)
        acc = ((X[idx, :nB].to(torch.int64) & 0xFFFF) * coef[:, None]).sum(dim=0) % p
        assert np.array_equal(acc.cpu().numpy(), B[i].toarray()[0] % p), f"row {i}"
    # every row, through random projections
    rng = np.random.default_rng(7)
    for _ in range(2):
        v = rng.integers(0, p, size=nB, dtype=np.int64)
        y = _project(X, npiv, nB, v, p)
        assert np.array_equal((A @ y) % p, (B @ v) % p)


def test_fullsize_reduce_equals_planted_schur_complement(full):
    g, s, res = full["g"], full["s"], full["res"]
    mD, nB = s["mD"], s["nB"]
    Dt = res["Dt"]
    step = 2048
    for r0 in range(0, mD, step):
        r1 = min(mD, r0 + step)
        got = _u16(Dt[r0:r1, :nB])
        assert np.array_equal(got, g["Dt"][r0:r1].toarray().astype(np.uint16)), f"rows {r0}..{r1}"


def test_fullsize_neworder_equals_planted_schur_complement(full):
    """Sec. 4.3 at full size: D - C A^{-1} B without X, in the MFMA form."""
    g, s, res = full["g"], full["s"], full["res"]
    mD, nB = s["mD"], s["nB"]
    Dt = fl.reduce_neworder(res["split"], fl.FL_MFMA_I8)
    torch.cuda.synchronize()
    step = 2048
    for r0 in range(0, mD, step):
        r1 = min(mD, r0 + step)
        assert np.array_equal(_u16(Dt[r0:r1, :nB]), g["Dt"][r0:r1].toarray().astype(np.uint16)), f"rows {r0}..{r1}"
    del Dt
    torch.cuda.empty_cache()


def test_fullsize_rref_d_equals_planted_V(full):
    g, s, res = full["g"], full["s"], full["res"]
    mD, nB = s["mD"], s["nB"]
    ech, RD = res["echelon"], res["RD"]
    r = int(_u32(ech.rank)[0])
    assert r == g["rank_d"]
    V = g["V"].tocsr()
    V.sort_indices()
    vpiv = V.indices[V.indptr[:-1]]
    assert np.array_equal(_u32(ech.pivcol)[:r], vpiv.astype(np.uint32))
    step = 2048
    for r0 in range(0, mD, step):
        r1 = min(mD, r0 + step)
        got = _u16(RD[r0:r1, :nB])
        if r0 < r:
            exp = np.zeros((r1 - r0, nB), np.uint16)
            k1 = min(r1, r)
            exp[:k1 - r0] = V[r0:k1].toarray().astype(np.uint16)
        else:
            exp = np.zeros((r1 - r0, nB), np.uint16)
        assert np.array_equal(got, exp), f"rows {r0}..{r1}"


def test_fullsize_second_pass_rows(full):
    g, s, res = full["g"], full["s"], full["res"]
    npiv, nB, p = s["npiv"], s["nB"], s["p"]
    V = g["V"].tocsr().astype(np.int64)
    V.sort_indices()
    r = V.shape[0]
    vpiv = V.indices[V.indptr[:-1]].astype(np.int64)
    rows = _sample_rows(npiv, 96, seed=9)
    idx = torch.from_numpy(rows).to(res["X"].device)
    X = _u16(res["X"][idx][:, :nB]).astype(np.int64)
    Xp = _u16(res["Xp"][idx][:, :nB]).astype(np.int64)
    exp = (X - (X[:, vpiv] @ V).astype(np.int64) % p) % p if r else X
    assert np.array_equal(Xp, exp)


def test_fullsize_csr_is_rref_of_M(full):
    g, s, res = full["g"], full["s"], full["res"]
    m, n, p = g["m"], g["n"], g["p"]
    rp, ci, vv, rank = res["rref"]
    assert rank == s["npiv"] + g["rank_d"]
    dev = rp.device
    rp64 = rp.to(torch.int64)
    nnz = int(rp64[-1])
    starts = rp64[:-1]
    assert bool((rp64[1:] > starts).all()), "empty row"
    piv = ci[starts].to(torch.int64)
    assert bool((vv[starts] == 1).all()), "leading entry is not 1"
    assert bool((piv[1:] > piv[:-1]).all()), "pivot columns not increasing"
    is_piv = torch.zeros(n, dtype=torch.bool, device=dev)
    is_piv[piv] = True
    rng = np.random.default_rng(11)
    xs = [torch.from_numpy(rng.integers(0, p, size=n, dtype=np.int64)).to(dev) for _ in range(2)]
    rx = [torch.zeros(rank, dtype=torch.int64, device=dev) for _ in xs]
    on_piv = 0
    chunk = 1 << 27
    for e0 in range(0, nnz, chunk):
        e1 = min(nnz, e0 + chunk)
        c = ci[e0:e1].to(torch.int64)
        v = vv[e0:e1].to(torch.int64) & 0xFFFF
        assert bool(((v > 0) & (v < p)).all()), "entry out of range"
        row_of = torch.searchsorted(rp64, torch.arange(e0, e1, device=dev), right=True) - 1
        assert bool(((c[1:] > c[:-1]) | (row_of[1:] != row_of[:-1])).all()), "columns not increasing"
        on_piv += int(is_piv[c].sum())
        for x, acc in zip(xs, rx):
            acc.index_add_(0, row_of, (v * x[c]) % p)
    assert on_piv == rank, "a pivot column is not a unit vector"
    M = sps.csr_matrix((g["val"].astype(np.int64), g["col"].astype(np.int64),
                        g["row_ptr"].astype(np.int64)), shape=(m, n))
    pv = piv.cpu().numpy()
    for x, acc in zip(xs, rx):
        z = x.cpu().numpy().copy()
        z[pv] = (z[pv] - acc.cpu().numpy() % p) % p
        assert not np.any((M @ z) % p), "a row of M is not in rowspace(R)"


def _same(a, b, rows, cols, what):
    a, b = a[:rows, :cols], b[:rows, :cols]
    if torch.equal(a, b):
        return
    bad = (a != b).nonzero()
    r, c = (int(x) for x in bad[0])
    raise AssertionError(f"{what}: {bad.shape[0]} mismatches, first at ({r}, {c}): "
                         f"{int(a[r, c]) & 0xFFFF} vs {int(b[r, c]) & 0xFFFF}")


def test_fullsize_plain_form_equals_mfma_form(full):
    g, s, res = full["g"], full["s"], full["res"]
    npiv, mD, nB = s["npiv"], s["mD"], s["nB"]
    plain = _run(g, fl.FL_PLAIN)
    _same(plain["X"], res["X"], npiv, nB, "X")
    _same(plain["Dt"], res["Dt"], mD, nB, "Dt")
    _same(plain["RD"], res["RD"], mD, nB, "R_D")
    _same(plain["Xp"], res["Xp"], npiv, nB, "X'")
    assert torch.equal(plain["echelon"].rank, res["echelon"].rank)
    r = int(_u32(res["echelon"].rank)[0])
    assert torch.equal(plain["echelon"].pivcol[:r], res["echelon"].pivcol[:r])
    for a, b in zip(plain["rref"][:3], res["rref"][:3]):
        assert torch.equal(a, b)
    assert plain["rref"][3] == res["rref"][3]
