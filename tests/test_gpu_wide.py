"""The FL path over 32-bit field characteristic (uint32 residues) on the GPU,
element by element against the uint32 CPU oracle: split (permutations),
X = A^-1 B, Dt = D - C X, RREF(Dt) with its pivots, the second pass X' and
the CSR of RREF(M); both arithmetic forms, multiline widths 1, 2 and 4,
32-bit primes and small ones, sizes spanning several 64-row TRSM blocks and
64-column echelon panels with ragged tails, degenerate shapes.  Also: the
uint32 path at p = 65521 equals the uint16 path bit for bit, and a reduce
whose K (40,000 pivots) spans two 32,704-term chunks of the four-limb
product with every limb at the centring window's extreme."""
import numpy as np
import pytest
import torch

import flgen
import oracle
import paper_1602_06097_amd as fl

pytestmark = pytest.mark.gpu

MODES = [fl.FL_PLAIN, fl.FL_MFMA_I8]
MODE_IDS = ["plain", "mfma"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fl.load()


def _wide(g):
    h = dict(g)
    h["val"] = g["val"].astype(np.uint32)
    return h


def _up(g):
    d = torch.device("cuda")
    return (torch.from_numpy(g["row_ptr"].view(np.int64).copy()).to(d),
            torch.from_numpy(g["col"].view(np.int32).copy()).to(d),
            torch.from_numpy(g["val"].astype(np.uint32).view(np.int32).copy()).to(d))


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


CASES = {
    "p32_planted": lambda: flgen.fl_matrix(m=900, n=1300, npiv=650, rank_d=180, density=0.05, p=4294967291,
                                           seed=31),
    "mersenne31": lambda: flgen.fl_matrix(m=700, n=1000, npiv=500, rank_d=150, density=0.06, p=2147483647,
                                          seed=32),
    "p65537": lambda: flgen.fl_matrix(m=520, n=777, npiv=333, rank_d=101, density=0.07, p=65537, seed=33),
    "p251_ragged": lambda: _wide(flgen.fl_matrix(m=333, n=517, npiv=201, rank_d=77, density=0.08, p=251,
                                                 seed=34)),
    "p3_random": lambda: _wide(flgen.random_sparse(150, 190, 0.1, 3, seed=35, zero_rows=0.1, dup_rows=0.1)),
    "p32_random": lambda: flgen.random_sparse(170, 230, 0.07, 4294967279, seed=36, zero_rows=0.05,
                                              dup_rows=0.1),
    "full_rank_d": lambda: flgen.fl_matrix(m=300, n=460, npiv=200, rank_d=100, density=0.06, p=4294967291,
                                           seed=37),
    "zero_d": lambda: flgen.fl_matrix(m=260, n=400, npiv=200, rank_d=0, density=0.06, p=4294967291, seed=38),
    "no_nonpivot_rows": lambda: flgen.fl_matrix(m=200, n=330, npiv=200, rank_d=0, density=0.06, p=4294967291,
                                                seed=39),
}
_REF = {}


def case(name):
    if name not in _REF:
        g = CASES[name]()
        _REF[name] = (g, oracle.fl_rref_wide(g))
    return _REF[name]


@pytest.mark.parametrize("w", [1, 2, 4])
@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
@pytest.mark.parametrize("name", list(CASES))
def test_wide_whole_path(name, mode, w):
    g, r = case(name)
    s = r["split"]
    rp, ci, vv = _up(g)
    sp = fl.split32(rp, ci, vv, g["m"], g["n"], g["p"], ml_width=w)
    assert (sp.npiv, sp.mD, sp.nB) == (s["npiv"], s["mD"], s["nB"])
    assert np.array_equal(_u32(sp.bufs["col_perm"])[:g["n"]], s["col_perm"])
    assert np.array_equal(_u32(sp.bufs["row_perm"])[:g["m"]], s["row_perm"])
    X = fl.trsm32(sp, mode)
    if sp.npiv and sp.nB:
        assert np.array_equal(_u32(X)[:sp.npiv, :sp.nB], r["X"])
    Dt = fl.reduce_cd32(sp, X, mode)
    if sp.mD and sp.nB:
        assert np.array_equal(_u32(Dt)[:sp.mD, :sp.nB], r["Dt"])
    ech = fl.echelon_d32(Dt, g["p"], sp.mD, sp.nB, mode)
    rank_d = int(_u32(ech.rank)[0])
    assert rank_d == r["rank_d"]
    if rank_d:
        assert np.array_equal(_u32(ech.pivcol)[:rank_d], r["pivcols"])
        assert np.array_equal(_u32(Dt)[:rank_d, :sp.nB], r["RD"])
        assert not _u32(Dt)[rank_d:sp.mD, :sp.nB].any()
    fl.rref32(sp, X, Dt, ech, mode)
    if sp.npiv and sp.nB:
        assert np.array_equal(_u32(X)[:sp.npiv, :sp.nB], r["Xp"])
    orp, oci, ov, rank = fl.rref32_to_csr(sp, X, Dt, ech)
    assert rank == r["rank"]
    erp, eci, ev = r["rref"]
    assert np.array_equal(orp.cpu().numpy().view(np.uint64), erp)
    assert np.array_equal(_u32(oci)[:len(eci)], eci)
    assert np.array_equal(_u32(ov)[:len(ev)], ev)


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_wide_equals_narrow_at_65521(mode):
    g = flgen.fl_matrix(m=640, n=900, npiv=450, rank_d=130, density=0.06, p=65521, seed=41)
    d = torch.device("cuda")
    rp = torch.from_numpy(g["row_ptr"].view(np.int64).copy()).to(d)
    ci = torch.from_numpy(g["col"].view(np.int32).copy()).to(d)
    v16 = torch.from_numpy(g["val"].view(np.int16).copy()).to(d)
    v32 = torch.from_numpy(g["val"].astype(np.uint32).view(np.int32).copy()).to(d)
    a = fl.fl_reduce(rp, ci, v16, g["m"], g["n"], g["p"], mode=mode, keep=True)
    b = fl.fl_reduce32(rp, ci, v32, g["m"], g["n"], g["p"], mode=mode, keep=True)
    npiv, nB = a["split"].npiv, a["split"].nB
    assert np.array_equal(a["X"].cpu().numpy().view(np.uint16)[:npiv, :nB].astype(np.uint32),
                          _u32(b["X"])[:npiv, :nB])
    ra, rb = a["rref"], b["rref"]
    assert ra[3] == rb[3]
    assert torch.equal(ra[0], rb[0]) and torch.equal(ra[1], rb[1])
    assert np.array_equal(ra[2].cpu().numpy().view(np.uint16).astype(np.uint32), _u32(rb[2]))


def test_wide_degenerate_shapes():
    p = 4294967291
    empty = dict(m=0, n=9, p=p, row_ptr=np.zeros(1, np.uint64), col=np.zeros(0, np.uint32),
                 val=np.zeros(0, np.uint32))
    zero = _wide(flgen.random_sparse(30, 20, 0.0, 3, seed=5))
    zero["p"] = p
    for g in (empty, zero):
        rp, ci, vv = _up(g)
        for mode in MODES:
            res = fl.fl_reduce32(rp, ci, vv, g["m"], g["n"], p, mode=mode)
            assert res["rref"][3] == 0


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_wide_reduce_k_beyond_chunk_extreme_limbs(mode):
    """A = I (pivot row i = e_i + B_i), every B and C entry x = 2139062144,
    whose centred residue x - p is the bottom of the window (limbs near
    -128): Dt = D - npiv x^2 exactly, with K = npiv = 40,000 > 32,704."""
    p, npiv, nB, mD = 4294967291, 40000, 64, 8
    x = 2139062144
    rows, cols, vals = [], [], []
    for i in range(npiv):
        rows.append(np.full(1 + nB, i))
        cols.append(np.concatenate([[i], npiv + np.arange(nB)]))
        vals.append(np.concatenate([[1], np.full(nB, x)]))
    rng = np.random.default_rng(5)
    D = rng.integers(1, p, size=(mD, nB), dtype=np.int64)
    for t in range(mD):
        rows.append(np.full(npiv + nB, npiv + t))
        cols.append(np.arange(npiv + nB))
        vals.append(np.concatenate([np.full(npiv, x), D[t]]))
    import scipy.sparse as sps
    M = sps.csr_matrix((np.concatenate(vals).astype(np.int64),
                        (np.concatenate(rows), np.concatenate(cols))), shape=(npiv + mD, npiv + nB))
    M.sort_indices()
    g = dict(m=npiv + mD, n=npiv + nB, p=p, row_ptr=M.indptr.astype(np.uint64), col=M.indices.astype(np.uint32),
             val=M.data.astype(np.uint32))
    rp, ci, vv = _up(g)
    sp = fl.split32(rp, ci, vv, g["m"], g["n"], p, ml_width=2)
    assert (sp.npiv, sp.mD, sp.nB) == (npiv, mD, nB)
    X = fl.trsm32(sp, mode)
    assert (_u32(X)[:npiv, :nB] == x).all()
    Dt = fl.reduce_cd32(sp, X, mode)
    want = (D - (npiv * x * x) % p) % p
    assert np.array_equal(_u32(Dt)[:mD, :nB].astype(np.int64), want)
