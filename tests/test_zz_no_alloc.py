"""The read-off's size query without allocation (fl_rref_csr_size_noalloc,
static device scratch) against fl_rref_csr_size with a caller workspace:
row_ptr, rank and nonzero count equal, and the CSR written from it equal,
on two calls in a row (the second on a smaller matrix, so the static
scratch holds the first call's counts when it starts); plus the size
limit and argument errors, which are reported before anything runs."""
import ctypes as ct

import numpy as np
import pytest
import torch

import flgen
import oracle
import paper_1602_06097_amd as fl

pytestmark = pytest.mark.gpu

P = 65521


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fl.load()


def _up(g):
    d = torch.device("cuda")
    return (torch.from_numpy(g["row_ptr"].view(np.int64).copy()).to(d),
            torch.from_numpy(g["col"].view(np.int32).copy()).to(d),
            torch.from_numpy(g["val"].view(np.int16).copy()).to(d))


def _pipeline(g, mode):
    rp, ci, vv = _up(g)
    sp = fl.split(rp, ci, vv, g["m"], g["n"], g["p"])
    X = fl.trsm(sp, mode)
    Dt = fl.reduce_cd(sp, X, mode)
    ech = fl.echelon_d(Dt, g["p"], sp.mD, sp.nB, mode)
    fl.rref(sp, X, Dt, ech, mode)
    return sp, X, Dt, ech


def _noalloc_csr(sp, X, Dt, ech, nnz_cap):
    rows = sp.npiv + min(sp.mD, sp.nB) + 1
    d = torch.device("cuda")
    # sentinels: the entry point must overwrite every entry it reports
    row_ptr = torch.full((rows,), -7, dtype=torch.int64, device=d)
    col = torch.full((max(nnz_cap, 1),), -7, dtype=torch.int32, device=d)
    val = torch.full((max(nnz_cap, 1),), -7, dtype=torch.int16, device=d)
    nnz, rank = fl.rref_to_csr_noalloc(sp, X, Dt, ech, row_ptr, col, val)
    torch.cuda.synchronize()
    return row_ptr[:rank + 1], col[:nnz], val[:nnz], rank


@pytest.mark.parametrize("mode", [fl.FL_PLAIN, fl.FL_MFMA_I8], ids=["plain", "mfma"])
def test_noalloc_size_equals_workspace_form_twice(mode):
    big = flgen.fl_matrix(m=1500, n=2100, npiv=1100, rank_d=260, density=0.05, p=P, seed=71)
    small = flgen.fl_matrix(m=420, n=610, npiv=300, rank_d=70, density=0.06, p=P, seed=72)
    for g in (big, small):
        sp, X, Dt, ech = _pipeline(g, mode)
        ref_rp, ref_ci, ref_v, ref_rank = fl.rref_to_csr(sp, X, Dt, ech)
        torch.cuda.synchronize()
        rp, ci, v, rank = _noalloc_csr(sp, X, Dt, ech, int(ref_rp[-1].item()) + 64)
        assert rank == ref_rank
        assert torch.equal(rp, ref_rp)
        assert torch.equal(ci, ref_ci)
        assert torch.equal(v, ref_v)
        # and the oracle agrees
        o = oracle.fl_rref(g, keep=False)
        assert rank == o["rank"]
        assert np.array_equal(rp.cpu().numpy().view(np.uint64), o["rref"][0])
        assert np.array_equal(ci.cpu().numpy().view(np.uint32), o["rref"][1])
        assert np.array_equal(v.cpu().numpy().view(np.uint16), o["rref"][2])


def test_noalloc_rejects_too_many_rows_before_running():
    lib = fl.load()
    cap = lib.fl_rref_csr_noalloc_scratch_bytes()
    assert cap == 16 << 20
    info = fl.FlSplitInfo()
    info.p, info.m, info.n, info.ml_width, info.status = P, 3_000_000, 3_000_000, 2, 0
    info.npiv, info.mD, info.nB = 2_500_000, 500_000, 500_000
    assert lib.fl_rref_csr_workspace(ct.byref(info)) > cap
    out = fl.FlSplitOut()
    h_rank, h_nnz = ct.c_uint32(0), ct.c_uint64(0)
    st = lib.fl_rref_csr_size_noalloc(ct.byref(info), ct.byref(out), None, 0, None, 0, None, None, None,
                                      ct.byref(h_rank), ct.byref(h_nnz), None)
    assert st != 0
    assert b"16 MiB" in lib.fl_last_error()


def test_noalloc_empty_reduction():
    g = flgen.random_sparse(40, 30, 0.0, P, seed=5)   # no nonzero: rank 0
    sp, X, Dt, ech = _pipeline(g, fl.FL_PLAIN)
    rp, ci, v, rank = _noalloc_csr(sp, X, Dt, ech, 0)
    assert rank == 0 and int(rp[0].item()) == 0 and ci.numel() == 0
