"""Contractions whose K range is longer than one int32 chunk of the int8-limb
MFMA form (65,472 terms), with every operand at the extreme of the limb
window, through the three entry points that run such contractions in one
launch: the reduce (C rows spanning all pivot columns), the TRSM band update
(pivot rows spanning the whole band) and the second pass (R_D of rank 80,000).

The residue 32880 centres to r = -32641 = 256 (-128) + 127, the pair whose
cross terms h l' + l h' = -32512 are the largest the window allows; over
80,000 terms the middle limb sum reaches -2.6e9, past the int32 range, so the
tiles must fold their accumulators every chunk.  X, D - C X, RREF and the
second pass are compared element by element with the oracle (reduce, TRSM)
or with the defining product (second pass, whose dense 128 x 80,000 x 80,192
product is out of the oracle's reach in a test)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1602_06097_amd as fl

pytestmark = pytest.mark.gpu

P = 65521
X_EXT = 32880
NB = 192


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fl.load()


def _mostly_extreme(rng, shape):
    """X_EXT with a tenth of the entries uniform in [1, p - 1]."""
    v = np.full(shape, X_EXT, np.int64)
    mask = rng.random(shape) < 0.1
    v[mask] = rng.integers(1, P, size=int(mask.sum()))
    return v.astype(np.uint16)


def _csr(m, n, lengths, cols, vals):
    rp = np.zeros(m + 1, np.uint64)
    rp[1:] = np.cumsum(lengths)
    return dict(m=m, n=n, p=P, row_ptr=rp, col=cols.astype(np.uint32), val=vals.astype(np.uint16))


def _up(g):
    d = torch.device("cuda")
    return (torch.from_numpy(g["row_ptr"].view(np.int64).copy()).to(d),
            torch.from_numpy(g["col"].view(np.int32).copy()).to(d),
            torch.from_numpy(g["val"].view(np.int16).copy()).to(d))


def _u16(t):
    return t.cpu().numpy().view(np.uint16)


def reduce_matrix(npiv=80000, mD=130, seed=1):
    """Pivot rows e_i + B_i (A = I, so X = B); non-pivot rows with entries in
    every pivot column (their lead is column 0) and 64 random columns of D."""
    rng = np.random.default_rng(seed)
    n = npiv + NB
    B = _mostly_extreme(rng, (npiv, NB))
    piv_cols = np.concatenate([np.arange(npiv)[:, None], npiv + np.tile(np.arange(NB), (npiv, 1))], axis=1)
    piv_vals = np.concatenate([np.ones((npiv, 1), np.uint16), B], axis=1)
    dcols = np.sort(rng.choice(NB, size=(mD, 64), replace=True), axis=1)
    crow_cols, crow_vals = [], []
    for t in range(mD):
        dc = np.unique(dcols[t])
        crow_cols.append(np.concatenate([np.arange(npiv), npiv + dc]))
        crow_vals.append(np.concatenate([_mostly_extreme(rng, npiv), rng.integers(1, P, size=len(dc))]))
    lengths = [NB + 1] * npiv + [len(c) for c in crow_cols]
    cols = np.concatenate([piv_cols.ravel()] + crow_cols)
    vals = np.concatenate([piv_vals.ravel()] + [v.astype(np.uint16) for v in crow_vals])
    return _csr(npiv + mD, n, lengths, cols, vals)


def trsm_matrix(npiv=80384, band_rows=128, band_start=512, seed=2):
    """Pivot rows 0..band_rows-1 hold A entries in every column from
    band_start on (past their 512-row superblock); the other pivot rows are
    e_i + B_i."""
    rng = np.random.default_rng(seed)
    n = npiv + NB
    B = _mostly_extreme(rng, (npiv, NB))
    rows_c, rows_v, lengths = [], [], []
    band = np.arange(band_start, npiv)
    for i in range(npiv):
        if i < band_rows:
            c = np.concatenate([[i], band, npiv + np.arange(NB)])
            v = np.concatenate([[1], _mostly_extreme(rng, len(band)), B[i]])
        else:
            c = np.concatenate([[i], npiv + np.arange(NB)])
            v = np.concatenate([[1], B[i]])
        rows_c.append(c)
        rows_v.append(np.asarray(v, np.int64).astype(np.uint16))
        lengths.append(len(c))
    return _csr(npiv, n, lengths, np.concatenate(rows_c), np.concatenate(rows_v))


@pytest.fixture(scope="module")
def reduce_case():
    g = reduce_matrix()
    return g, oracle.fl_rref(g)


@pytest.mark.parametrize("mode", [fl.FL_PLAIN, fl.FL_MFMA_I8])
def test_reduce_k_beyond_chunk(reduce_case, mode):
    g, r = reduce_case
    s = r["split"]
    assert s["npiv"] == 80000 and s["mD"] == 130 and s["nB"] == NB
    res = fl.fl_reduce(*_up(g), g["m"], g["n"], P, mode=mode, ml_width=2, keep=True)
    torch.cuda.synchronize()
    npiv, mD, nB = s["npiv"], s["mD"], s["nB"]
    assert np.array_equal(_u16(res["X"])[:npiv, :nB], r["X"])
    assert np.array_equal(_u16(res["Dt"])[:mD, :nB], r["Dt"])
    rank = int(res["echelon"].rank.cpu().numpy().view(np.uint32)[0])
    assert rank == r["rank_d"]
    assert np.array_equal(_u16(res["RD"])[:rank, :nB], r["RD"])
    assert np.array_equal(_u16(res["Xp"])[:npiv, :nB], r["Xp"])
    orp, oci, ov, rk = res["rref"]
    erp, eci, ev = r["rref"]
    assert rk == r["rank"]
    assert np.array_equal(orp.cpu().numpy().view(np.uint64), erp)
    assert np.array_equal(oci.cpu().numpy().view(np.uint32)[:len(eci)], eci)
    assert np.array_equal(ov.cpu().numpy().view(np.uint16)[:len(ev)], ev)


@pytest.mark.parametrize("mode", [fl.FL_PLAIN, fl.FL_MFMA_I8])
@pytest.mark.parametrize("w", [1, 2])
def test_trsm_band_k_beyond_chunk(mode, w):
    g = trsm_matrix()
    s = oracle.split(g)
    assert s["npiv"] == 80384 and s["mD"] == 0
    Xr = oracle.trsm(s)
    sp = fl.split(*_up(g), g["m"], g["n"], P, ml_width=w)
    X = fl.trsm(sp, mode)
    torch.cuda.synchronize()
    assert np.array_equal(_u16(X)[:sp.npiv, :sp.nB], Xr)


def _second_pass_reference(X, Rn, r):
    """X' = X - X[:, :r] [I | Rn] mod p, exactly: the products are summed in
    float64 in chunks of 2048 terms (each partial sum an integer below 2^43)."""
    Xl = X[:, :r].astype(np.float64)
    acc = np.zeros((X.shape[0], Rn.shape[1]), np.int64)
    for k0 in range(0, r, 2048):
        part = Xl[:, k0:k0 + 2048] @ Rn[k0:k0 + 2048].astype(np.float64)
        acc = (acc + part.astype(np.int64)) % P
    out = np.zeros_like(X, dtype=np.int64)
    out[:, r:] = (X[:, r:].astype(np.int64) - acc) % P
    return out.astype(np.uint16)


@pytest.mark.parametrize("mode", [fl.FL_PLAIN, fl.FL_MFMA_I8])
def test_second_pass_k_beyond_chunk(mode):
    """128 pivot rows against an R_D = [I | Rn] of rank 80,000 (the matrix
    has 80,000 empty non-pivot rows, so mD = 80,000 and nB = 80,192)."""
    rng = np.random.default_rng(3)
    npiv, r = 128, 80000
    nB = r + NB
    B = _mostly_extreme(rng, (npiv, nB))
    cols = np.concatenate([np.arange(npiv)[:, None], npiv + np.tile(np.arange(nB), (npiv, 1))], axis=1)
    vals = np.concatenate([np.ones((npiv, 1), np.uint16), B], axis=1)
    lengths = [nB + 1] * npiv + [0] * r
    g = _csr(npiv + r, npiv + nB, lengths, cols.ravel(), vals.ravel())
    sp = fl.split(*_up(g), g["m"], g["n"], P, ml_width=2)
    assert (sp.npiv, sp.mD, sp.nB) == (npiv, r, nB)
    X = fl.trsm(sp, mode)
    Rn = _mostly_extreme(rng, (r, NB))
    ld = X.shape[1]
    Dt = torch.zeros((r, ld), dtype=torch.int16, device="cuda")
    diag = torch.arange(r, device="cuda", dtype=torch.int64)
    Dt.view(-1)[diag * ld + diag] = 1
    Dt[:, r:nB] = torch.from_numpy(Rn.view(np.int16)).cuda()
    ech = fl.Echelon(rank=torch.tensor([r], dtype=torch.int32, device="cuda"),
                     pivcol=torch.arange(r, dtype=torch.int32, device="cuda"), rows=r, cols=nB)
    fl.rref(sp, X, Dt, ech, mode)
    torch.cuda.synchronize()
    want = _second_pass_reference(B, Rn, r)
    assert np.array_equal(_u16(X)[:npiv, :nB], want)
