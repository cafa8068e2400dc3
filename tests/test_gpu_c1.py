"""The whole path on the 2,048 x 3,072 workload over F_65521 (1,536 pivot
rows, planted rank 384 in the Schur complement, 6% density), both arithmetic
forms and every multiline width, against the oracle element by element:
the split (permutations, B, D and the multilines of A and C), X = A^-1 B,
D - C X, RREF(D - C X) with its pivot columns, the second pass X' and the
CSR of RREF(M).  The oracle's result on this matrix is itself pinned by
brute-force Gauss-Jordan on M and by the planted closed forms (CPU tests)."""
import numpy as np
import pytest
import torch

import flgen
import oracle
import paper_1602_06097_amd as fl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c1():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fl.load()
    g = flgen.config_matrix("c1")
    return g, oracle.fl_rref(g)


def _up(g):
    d = torch.device("cuda")
    return (torch.from_numpy(g["row_ptr"].view(np.int64).copy()).to(d),
            torch.from_numpy(g["col"].view(np.int32).copy()).to(d),
            torch.from_numpy(g["val"].view(np.int16).copy()).to(d))


def _u16(t):
    return t.cpu().numpy().view(np.uint16)


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


def _strict_upper(A, npiv):
    rp, ci, v = A
    keep = np.ones(len(ci), bool)
    keep[rp[:-1].astype(np.int64)] = False
    nrp = np.zeros(npiv + 1, np.uint64)
    nrp[1:] = np.cumsum(np.diff(rp.astype(np.int64)) - 1)
    return nrp, ci[keep], v[keep]


@pytest.mark.parametrize("w", [1, 2, 4, 8])
@pytest.mark.parametrize("mode", [fl.FL_PLAIN, fl.FL_MFMA_I8], ids=["plain", "mfma"])
def test_c1_whole_path(c1, mode, w):
    g, r = c1
    s = r["split"]
    npiv, mD, nB = s["npiv"], s["mD"], s["nB"]
    assert (npiv, mD, nB) == (1536, 512, 1536) and r["rank_d"] == 384
    res = fl.fl_reduce(*_up(g), g["m"], g["n"], g["p"], mode=mode, ml_width=w, keep=True)
    torch.cuda.synchronize()
    sp = res["split"]
    b = sp.bufs
    # split
    assert (sp.npiv, sp.mD, sp.nB) == (npiv, mD, nB)
    assert np.array_equal(_u32(b["row_perm"])[:g["m"]], s["row_perm"])
    assert np.array_equal(_u32(b["col_perm"])[:g["n"]], s["col_perm"])
    for key, rows in (("b", npiv), ("d", mD)):
        orp, oci, ov = s[key.upper()]
        assert np.array_equal(_u64(b[f"{key}_ptr"])[:rows + 1], orp)
        k = int(orp[-1])
        assert np.array_equal(_u32(b[f"{key}_col"])[:k], oci)
        assert np.array_equal(_u16(b[f"{key}_val"])[:k], ov)
    for key, csr3, rows in (("a", _strict_upper(s["A"], npiv), npiv), ("c", s["C"], mD)):
        gptr, pos, val = oracle.multiline(csr3, rows, npiv, w)
        ng = (rows + w - 1) // w
        assert np.array_equal(_u64(b[f"{key}_gptr"])[:ng + 1], gptr)
        assert np.array_equal(_u32(b[f"{key}_pos"])[:len(pos)], pos)
        assert np.array_equal(_u16(b[f"{key}_val"])[:len(val)], val)
    # TRSM, reduce, RREF of the Schur complement, second pass
    assert np.array_equal(_u16(res["X"])[:npiv, :nB], r["X"])
    assert np.array_equal(_u16(res["Dt"])[:mD, :nB], r["Dt"])
    rank = int(_u32(res["echelon"].rank)[0])
    assert rank == r["rank_d"]
    assert np.array_equal(_u32(res["echelon"].pivcol)[:rank], r["pivcols"])
    RD = _u16(res["RD"])[:mD, :nB]
    assert np.array_equal(RD[:rank], r["RD"])
    assert not RD[rank:].any()
    assert np.array_equal(_u16(res["Xp"])[:npiv, :nB], r["Xp"])
    # read-off
    orp, oci, ov, rk = res["rref"]
    erp, eci, ev = r["rref"]
    assert rk == r["rank"] == 1920
    assert np.array_equal(_u64(orp), erp)
    assert np.array_equal(_u32(oci)[:len(eci)], eci)
    assert np.array_equal(_u16(ov)[:len(ev)], ev)


def test_c1_new_order(c1):
    """Sec. 4.3's reduction without X on the same matrix, both forms."""
    g, r = c1
    s = r["split"]
    for mode in (fl.FL_PLAIN, fl.FL_MFMA_I8):
        sp = fl.split(*_up(g), g["m"], g["n"], g["p"], ml_width=2)
        Dt = fl.reduce_neworder(sp, mode)
        torch.cuda.synchronize()
        assert np.array_equal(_u16(Dt)[:s["mD"], :s["nB"]], r["Dt"]), mode
