"""Dense-phase precision stress at full size over F_65521 and F_251:
D - C B for C 16,384 x 32,768 and B 32,768 x 16,384 (uniform residues), and
the RREF of a dense 16,384 x 16,384 matrix of planted rank 12,288.

The two run as separate sub-runs: a D whose Schur complement D - C B has a
planted rank would need the full product on the host first.  The product is
checked exactly on sampled entries (each an oracle dot product), on whole
sampled rows and columns at tile edges, and on every entry through random
projections; the RREF must equal the planted one exactly.  Both arithmetic
forms must agree bit for bit.
"""
import numpy as np
import pytest
import torch

import flgen
import paper_1602_06097_amd as fl

pytestmark = pytest.mark.gpu

M, K, N = 16384, 32768, 16384
PRIMES = [65521, 251]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fl.load()


def _u16(t):
    return t.cpu().numpy().view(np.uint16)


def _dev16(a):
    return torch.from_numpy(a.astype(np.uint16).view(np.int16)).cuda()


@pytest.mark.parametrize("p", PRIMES)
def test_c3_dense_product(p):
    rng = np.random.default_rng(3 + p)
    C = rng.integers(0, p, size=(M, K), dtype=np.uint16)
    B = rng.integers(0, p, size=(K, N), dtype=np.uint16)
    D0 = rng.integers(0, p, size=(M, N), dtype=np.uint16)
    tC, tB = _dev16(C), _dev16(B)
    outs = {}
    for mode in (fl.FL_MFMA_I8, fl.FL_PLAIN):
        tD = _dev16(D0)
        fl.matmul_sub(p, tC, tB, tD, M, N, K, mode)
        torch.cuda.synchronize()
        outs[mode] = tD
    assert torch.equal(outs[fl.FL_MFMA_I8], outs[fl.FL_PLAIN])
    R = _u16(outs[fl.FL_MFMA_I8]).astype(np.int64)
    del outs, tC, tB
    Ci, Bi = C.astype(np.int64), B.astype(np.int64)
    # sampled entries, incl. every 128-tile edge on both axes
    er = np.unique(np.concatenate([np.arange(0, M, 128), np.arange(127, M, 128), [M - 1]]))
    ec = np.unique(np.concatenate([np.arange(0, N, 128), np.arange(127, N, 128), [N - 1]]))
    ri = np.concatenate([er, rng.integers(0, M, len(ec)), rng.integers(0, M, 1024)])
    cj = np.concatenate([rng.integers(0, N, len(er)), ec, rng.integers(0, N, 1024)])
    want = (D0[ri, cj].astype(np.int64) - (Ci[ri] * Bi[:, cj].T).sum(1) % p) % p
    assert np.array_equal(R[ri, cj], want)
    # whole rows and columns at tile edges
    for i in (0, 127, 128, M - 1):
        cb = np.zeros(N, np.int64)
        for k0 in range(0, K, 2048):
            cb += (Ci[i, k0:k0 + 2048, None] * Bi[k0:k0 + 2048]).sum(0)
        row = (D0[i].astype(np.int64) - cb % p) % p
        assert np.array_equal(R[i], row), f"row {i}"
    for j in (0, 129, N - 1):
        col = (D0[:, j].astype(np.int64) - (Ci @ Bi[:, j]) % p) % p
        assert np.array_equal(R[:, j], col), f"col {j}"
    # every entry: R v == D0 v - C (B v) mod p
    for _ in range(2):
        v = rng.integers(0, p, size=N, dtype=np.int64)
        bv = np.zeros(K, np.int64)
        for k0 in range(0, K, 4096):
            bv[k0:k0 + 4096] = (Bi[k0:k0 + 4096] @ v) % p
        cbv = np.zeros(M, np.int64)
        rv = np.zeros(M, np.int64)
        dv = np.zeros(M, np.int64)
        for i0 in range(0, M, 2048):
            cbv[i0:i0 + 2048] = (Ci[i0:i0 + 2048] @ bv) % p
            rv[i0:i0 + 2048] = (R[i0:i0 + 2048] @ v) % p
            dv[i0:i0 + 2048] = (D0[i0:i0 + 2048].astype(np.int64) @ v) % p
        assert np.array_equal(rv, (dv - cbv) % p)


@pytest.mark.parametrize("p", PRIMES)
def test_c3_dense_rref_planted_rank(p):
    d = flgen.dense_planted_rank(16384, 16384, 12288, p, seed=31 + p)
    res = {}
    for mode in (fl.FL_MFMA_I8, fl.FL_PLAIN):
        D = _dev16(d["D"])
        ech = fl.echelon_d(D, p, 16384, 16384, mode)
        torch.cuda.synchronize()
        res[mode] = (D, ech)
    D, ech = res[fl.FL_MFMA_I8]
    rank = int(ech.rank.cpu().numpy().view(np.uint32)[0])
    assert rank == 12288
    assert np.array_equal(ech.pivcol.cpu().numpy().view(np.uint32)[:rank], d["pivcols"])
    out = _u16(D)
    assert np.array_equal(out[:rank], d["V"])
    assert not out[rank:].any()
    Dp, ep = res[fl.FL_PLAIN]
    assert torch.equal(Dp, D)
    assert torch.equal(ep.pivcol, ech.pivcol) and torch.equal(ep.rank, ech.rank)
