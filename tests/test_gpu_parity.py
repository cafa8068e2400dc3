"""Parity of the device path (through the C ABI) with the CPU oracle.

Every comparison is bit-exact: all arithmetic is exact modular integer
arithmetic, so the tolerance is zero mismatches.  Inputs are seeded and
synthetic (flgen); sizes span several tiles with ragged tails.
"""
import numpy as np
import pytest
import torch

import flgen
import oracle
import paper_1602_06097_amd as fl

pytestmark = pytest.mark.gpu

MODES = [fl.FL_PLAIN, fl.FL_MFMA_I8]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fl.load()


def up(g):
    d = torch.device("cuda")
    return (torch.from_numpy(g["row_ptr"].view(np.int64).copy()).to(d),
            torch.from_numpy(g["col"].view(np.int32).copy()).to(d),
            torch.from_numpy(g["val"].view(np.int16).copy()).to(d))


def u16(t):
    return t.cpu().numpy().view(np.uint16)


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def u64(t):
    return t.cpu().numpy().view(np.uint64)


def _cases():
    c = {}
    c["tiny_p7"] = flgen.random_sparse(9, 13, 0.4, 7, seed=1, zero_rows=0.1, dup_rows=0.2)
    c["tiny_p2"] = flgen.random_sparse(12, 10, 0.5, 2, seed=2, zero_rows=0.1)
    c["nonmonic_p65521"] = flgen.random_sparse(180, 260, 0.06, 65521, seed=3, zero_rows=0.05,
                                               dup_rows=0.1)
    c["nonmonic_p251"] = flgen.random_sparse(150, 150, 0.08, 251, seed=4, dup_rows=0.2)
    c["planted_ragged"] = flgen.fl_matrix(m=1300, n=1900, npiv=950, rank_d=230, density=0.05,
                                          p=65521, seed=11)
    c["planted_p251"] = flgen.fl_matrix(m=700, n=1000, npiv=500, rank_d=150, density=0.06,
                                        p=251, seed=12)
    c["full_rank_d"] = flgen.fl_matrix(m=600, n=700, npiv=400, rank_d=200, density=0.05,
                                       p=65521, seed=13)
    c["zero_d"] = flgen.fl_matrix(m=500, n=700, npiv=400, rank_d=0, density=0.05, p=65521, seed=14)
    c["no_nonpivot_rows"] = flgen.fl_matrix(m=300, n=500, npiv=300, rank_d=0, density=0.05,
                                            p=65521, seed=15)
    c["identity_like"] = _identity(70, 65521)
    return c


def _identity(n, p):
    import scipy.sparse as sp
    a = sp.identity(n, dtype=np.int64, format="csr")
    return dict(m=n, n=n, p=p, row_ptr=a.indptr.astype(np.uint64), col=a.indices.astype(np.uint32),
                val=a.data.astype(np.uint16))


CASES = _cases()
_ORACLE = {}


def ref(name):
    if name not in _ORACLE:
        _ORACLE[name] = oracle.fl_rref(CASES[name])
    return _ORACLE[name]


def _strict_upper(A, npiv):
    """Oracle A without its unit diagonal (the device stores only the rest)."""
    rp, ci, v = A
    keep = np.ones(len(ci), bool)
    for i in range(npiv):
        keep[int(rp[i])] = False  # first entry of row i is the diagonal
    counts = np.diff(rp.astype(np.int64)) - 1
    nrp = np.zeros(npiv + 1, np.uint64)
    nrp[1:] = np.cumsum(counts)
    return nrp, ci[keep], v[keep]


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("w", [1, 2, 4, 8])
def test_split_parity(name, w):
    g, r = CASES[name], ref(name)
    s = r["split"]
    sp = fl.split(*up(g), g["m"], g["n"], g["p"], ml_width=w)
    torch.cuda.synchronize()
    assert (sp.npiv, sp.mD, sp.nB) == (s["npiv"], s["mD"], s["nB"])
    b = sp.bufs
    assert np.array_equal(u32(b["row_perm"])[:g["m"]], s["row_perm"])
    assert np.array_equal(u32(b["col_perm"])[:g["n"]], s["col_perm"])
    npiv, mD = s["npiv"], s["mD"]
    for key, rows in (("b", npiv), ("d", mD)):
        orp, oci, ov = s[key.upper()]
        assert np.array_equal(u64(b[f"{key}_ptr"])[:rows + 1], orp)
        k = int(orp[-1])
        assert np.array_equal(u32(b[f"{key}_col"])[:k], oci)
        assert np.array_equal(u16(b[f"{key}_val"])[:k], ov)
    assert sp.info.nnzB == int(s["B"][0][-1]) and sp.info.nnzD == int(s["D"][0][-1])
    # A (strictly upper) and C as w-multilines, against the oracle's packer
    for key, csr3, rows, length in (("a", _strict_upper(s["A"], npiv), npiv, sp.info.lenA),
                                    ("c", s["C"], mD, sp.info.lenC)):
        gptr, pos, val = oracle.multiline(csr3, rows, npiv, w)
        ng = (rows + w - 1) // w
        assert np.array_equal(u64(b[f"{key}_gptr"])[:ng + 1], gptr)
        assert length == len(pos)
        assert np.array_equal(u32(b[f"{key}_pos"])[:len(pos)], pos)
        assert np.array_equal(u16(b[f"{key}_val"])[:len(val)], val)
    assert sp.info.nnzA == int(s["A"][0][-1]) - npiv
    assert sp.info.nnzC == int(s["C"][0][-1])


@pytest.fixture(scope="module")
def runs():
    cache = {}

    def get(name, mode, w=2):
        key = (name, mode, w)
        if key not in cache:
            g = CASES[name]
            res = fl.fl_reduce(*up(g), g["m"], g["n"], g["p"], mode=mode, ml_width=w, keep=True)
            torch.cuda.synchronize()
            cache[key] = res
        return cache[key]
    return get


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("w", [1, 2, 8])
@pytest.mark.parametrize("mode", MODES)
def test_trsm_parity(name, w, mode, runs):
    r = ref(name)
    res = runs(name, mode, w)
    s = r["split"]
    if s["npiv"] and s["nB"]:
        assert np.array_equal(u16(res["X"])[:s["npiv"], :s["nB"]], r["X"])


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("mode", MODES)
def test_reduce_parity(name, mode, runs):
    r = ref(name)
    res = runs(name, mode)
    s = r["split"]
    if s["mD"] and s["nB"]:
        assert np.array_equal(u16(res["Dt"])[:s["mD"], :s["nB"]], r["Dt"])


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("mode", MODES)
def test_echelon_and_rref_parity(name, mode, runs):
    r = ref(name)
    res = runs(name, mode)
    s = r["split"]
    mD, nB, npiv = s["mD"], s["nB"], s["npiv"]
    if mD and nB:
        rank = int(u32(res["echelon"].rank)[0])
        assert rank == r["rank_d"]
        assert np.array_equal(u32(res["echelon"].pivcol)[:rank], r["pivcols"])
        RD = u16(res["RD"])[:mD, :nB]
        assert np.array_equal(RD[:rank], r["RD"])
        assert not RD[rank:].any()
    if npiv and nB:
        assert np.array_equal(u16(res["Xp"])[:npiv, :nB], r["Xp"])
    orp, oci, ov, rank = res["rref"]
    assert rank == r["rank"]
    erp, eci, ev = r["rref"]
    assert np.array_equal(u64(orp), erp)
    assert np.array_equal(u32(oci)[:len(eci)], eci)
    assert np.array_equal(u16(ov)[:len(ev)], ev)


@pytest.mark.parametrize("mode", MODES)
def test_echelon_dense_planted(mode):
    """Dense RREF with several 1024-row chunks and a ragged last panel."""
    p = 65521
    d = flgen.dense_planted_rank(2500, 700, 470, p, seed=21)
    ld = 704
    D = torch.zeros((2500, ld), dtype=torch.int16, device="cuda")
    D[:, :700] = torch.from_numpy(d["D"].view(np.int16))
    ech = fl.echelon_d(D, p, 2500, 700, mode)
    torch.cuda.synchronize()
    rank = int(u32(ech.rank)[0])
    assert rank == 470
    assert np.array_equal(u32(ech.pivcol)[:rank], d["pivcols"])
    out = u16(D)[:, :700]
    assert np.array_equal(out[:rank], d["V"])
    assert not out[rank:].any()
    assert not u16(D)[:, 700:].any()  # padding columns untouched


@pytest.mark.parametrize("p", [65521, 251, 2])
@pytest.mark.parametrize("shape", [(130, 300, 200), (257, 129, 1000), (64, 64, 64), (1, 5, 3)])
def test_matmul_sub_both_forms(p, shape):
    M, N, K = shape
    rng = np.random.default_rng(M * 7 + N + K + p)
    C = rng.integers(0, p, size=(M, K), dtype=np.int64)
    X = rng.integers(0, p, size=(K, N), dtype=np.int64)
    D0 = rng.integers(0, p, size=(M, N), dtype=np.int64)
    want = (D0 - (C @ X) % p) % p
    ldc, ldx = (K + 7) // 8 * 8, (N + 3) // 4 * 4
    for mode in MODES:
        tc = torch.zeros((M, ldc), dtype=torch.int16)
        tc[:, :K] = torch.from_numpy(C.astype(np.uint16).view(np.int16))
        tx = torch.zeros((K, ldx), dtype=torch.int16)
        tx[:, :N] = torch.from_numpy(X.astype(np.uint16).view(np.int16))
        td = torch.zeros((M, ldx), dtype=torch.int16)
        td[:, :N] = torch.from_numpy(D0.astype(np.uint16).view(np.int16))
        tc, tx, td = tc.cuda(), tx.cuda(), td.cuda()
        fl.matmul_sub(p, tc, tx, td, M, N, K, mode)
        torch.cuda.synchronize()
        assert np.array_equal(u16(td)[:, :N].astype(np.int64), want), mode


@pytest.mark.parametrize("value", [32640, 32639, 65520, 1])
def test_matmul_sub_limb_extremes(value):
    """Extreme limbs (32640 -> r = -32881 -> h = -128, l = -113; 32639 -> 127,
    127) with K beyond one int32 chunk of the MFMA form."""
    p, M, N, K = 65521, 32, 40, 70000
    C = np.full((M, K), value, np.int64)
    X = np.full((K, N), value, np.int64)
    X[::3] = 32640
    want = (-(C @ X)) % p
    for mode in MODES:
        tc = torch.from_numpy(C.astype(np.uint16).view(np.int16)).cuda()
        tx = torch.from_numpy(X.astype(np.uint16).view(np.int16)).cuda()
        td = torch.zeros((M, N), dtype=torch.int16, device="cuda")
        fl.matmul_sub(p, tc, tx, td, M, N, K, mode)
        torch.cuda.synchronize()
        assert np.array_equal(u16(td).astype(np.int64), want), mode


@pytest.mark.parametrize("p,value", [(251, 125), (251, 126), (251, 250), (241, 121), (3, 2), (2, 1)])
def test_matmul_sub_single_limb_extremes(p, value):
    """p < 256: each residue is one symmetric int8 limb ((p - 1) / 2 stays,
    (p + 1) / 2 becomes -(p - 1) / 2) and the MFMA GEMM runs the single
    product; K beyond one int32 chunk."""
    M, N, K = 32, 40, 70000
    C = np.full((M, K), value, np.int64)
    X = np.full((K, N), value, np.int64)
    X[::3] = (p + 1) // 2 % p
    want = (-(C @ X)) % p
    for mode in MODES:
        tc = torch.from_numpy(C.astype(np.uint16).view(np.int16)).cuda()
        tx = torch.from_numpy(X.astype(np.uint16).view(np.int16)).cuda()
        td = torch.zeros((M, N), dtype=torch.int16, device="cuda")
        fl.matmul_sub(p, tc, tx, td, M, N, K, mode)
        torch.cuda.synchronize()
        assert np.array_equal(u16(td).astype(np.int64), want), mode


def test_modular_reduction_exhaustive_on_device():
    """The kernels' Barrett reduction equals x % p for every x < 2^32, and
    the limb combines (the general one, the p >= 256 one with 24-bit
    products, the single-limb one for p < 256) equal S mod p over their
    input ranges; 257 is the smallest prime of the 24-bit form."""
    primes = [2, 3, 251, 257, 32749, 65521]
    assert fl.check_modp(primes) == [0] * len(primes)


@pytest.mark.parametrize("field,value,code", [("col", 10**6, 4), ("val", 0, 6), ("val", 65521, 6)])
def test_split_reports_data_errors(field, value, code):
    g = flgen.random_sparse(20, 30, 0.3, 65521, seed=5)
    g = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in g.items()}
    k = int(g["row_ptr"][3]) + 1
    g[field][k] = value
    assert oracle.validate(g) != oracle.OR_OK
    with pytest.raises(fl.FlError) as e:
        fl.split(*up(g), g["m"], g["n"], g["p"])
    assert e.value.status == code


def test_split_reports_unsorted_columns():
    g = flgen.random_sparse(20, 30, 0.4, 65521, seed=6)
    g = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in g.items()}
    s = int(g["row_ptr"][2])
    g["col"][s + 1] = g["col"][s]
    with pytest.raises(fl.FlError) as e:
        fl.split(*up(g), g["m"], g["n"], g["p"])
    assert e.value.status == 5


def test_trsm_many_blocks_both_forms():
    """Several 128-row TRSM blocks with bands reaching far right (long rows)."""
    g = flgen.fl_matrix(m=1400, n=1700, npiv=1100, rank_d=150, density=0.12, p=65521, seed=51)
    r = oracle.fl_rref(g)
    for mode in MODES:
        for w in (2, 4):
            sp = fl.split(*up(g), g["m"], g["n"], g["p"], ml_width=w)
            X = fl.trsm(sp, mode)
            torch.cuda.synchronize()
            assert np.array_equal(u16(X)[:sp.npiv, :sp.nB], r["X"]), (mode, w)


@pytest.mark.parametrize("p", [65521, 251])
def test_trsm_lookahead_far_update(p):
    """A band reaching past the superblock below (wide row supports): the
    MFMA form's far update is split by K between the main stream and a
    second stream; both parts and their ordering against the block solves
    are checked, twice in a row (no race between the streams).  p = 251
    runs the single-limb GEMM."""
    g = flgen.fl_matrix(m=2600, n=3400, npiv=2200, rank_d=200, density=0.06, p=p, seed=61,
                        rho_loc=0.05)
    s = oracle.split(g)
    Xr = oracle.trsm(s)
    for mode in MODES:
        for w in (1, 2):
            sp = fl.split(*up(g), g["m"], g["n"], g["p"], ml_width=w)
            X1 = fl.trsm(sp, mode)
            X2 = fl.trsm(sp, mode)
            torch.cuda.synchronize()
            assert np.array_equal(u16(X1)[:sp.npiv, :sp.nB], Xr), (mode, w)
            assert np.array_equal(u16(X2)[:sp.npiv, :sp.nB], Xr), (mode, w)


@pytest.mark.parametrize("p", [251, 241])
def test_single_limb_pipeline_many_blocks(p):
    """The whole MFMA-form path for p < 256 (single-limb GEMM in the TRSM
    band, the reduce and the second pass; single limbs through the rank-k
    tiles) on a matrix with several TRSM superblocks and echelon blocks,
    against the oracle and the plain form."""
    g = flgen.fl_matrix(m=2600, n=3400, npiv=2000, rank_d=420, density=0.05, p=p, seed=71 + p,
                        rho_loc=0.08)
    r = oracle.fl_rref(g)
    outs = {}
    for mode in MODES:
        res = fl.fl_reduce(*up(g), g["m"], g["n"], g["p"], mode=mode, keep=True)
        torch.cuda.synchronize()
        sp = res["split"]
        assert np.array_equal(u16(res["X"])[:sp.npiv, :sp.nB], r["X"]), mode
        assert np.array_equal(u16(res["Dt"])[:sp.mD, :sp.nB], r["Dt"]), mode
        assert np.array_equal(u16(res["Xp"])[:sp.npiv, :sp.nB], r["Xp"]), mode
        outs[mode] = [t.cpu() for t in res["rref"][:3]]
    for a, b in zip(outs[fl.FL_PLAIN], outs[fl.FL_MFMA_I8]):
        assert torch.equal(a, b)


def test_repeat_runs_identical():
    """Two runs of the whole path give identical bytes (no data races)."""
    g = CASES["planted_ragged"]
    a = fl.fl_reduce(*up(g), g["m"], g["n"], g["p"], mode=fl.FL_MFMA_I8)
    b = fl.fl_reduce(*up(g), g["m"], g["n"], g["p"], mode=fl.FL_MFMA_I8)
    torch.cuda.synchronize()
    for x, y in zip(a["rref"][:3], b["rref"][:3]):
        assert torch.equal(x, y)


@pytest.mark.parametrize("mode", MODES)
def test_echelon_probe_misses_rows(mode):
    """The first rows span only a 3-dimensional space, so the probe basis of
    each panel is incomplete and the flagged-row merge must finish the panel
    (more than 1024 flagged rows: several collection rounds)."""
    p = 65521
    rng = np.random.default_rng(31)
    rows, cols = 2600, 200
    base = rng.integers(0, p, size=(3, cols))
    D = np.zeros((rows, cols), np.int64)
    D[:400] = (rng.integers(0, p, size=(400, 3)) @ base) % p
    D[400:] = rng.integers(0, p, size=(rows - 400, cols))
    R, r, pc = oracle.rref_dense(D.astype(np.uint16), p)
    T = torch.zeros((rows, 200), dtype=torch.int16)
    T[:] = torch.from_numpy(D.astype(np.uint16).view(np.int16))
    T = T.cuda()
    ech = fl.echelon_d(T, p, rows, cols, mode)
    torch.cuda.synchronize()
    rank = int(u32(ech.rank)[0])
    assert rank == r == 200
    assert np.array_equal(u32(ech.pivcol)[:rank], pc)
    assert np.array_equal(u16(T)[:rank], R[:rank])
    assert not u16(T)[rank:].any()


@pytest.mark.parametrize("mode", MODES)
def test_echelon_flagged_rows_never_dropped(mode):
    """Regression: the merge lists flagged rows window by window; a window
    that overflowed the list used to be skipped past.  Rows [0, 1024) are
    multiples of v0 (the probe basis), 500 rows of the next window and 900 of
    the one after are in span(v0, v1), and one row deep in the third window is
    the only one with a third direction."""
    p = 65521
    rng = np.random.default_rng(41)
    rows, cols = 3100, 64
    v0, v1, w = (rng.integers(1, p, size=cols) for _ in range(3))
    D = np.zeros((rows, cols), np.int64)
    D[:1024] = np.outer(rng.integers(1, p, size=1024), v0) % p
    r1 = 1024 + np.sort(rng.choice(1024, 500, replace=False))
    r2 = 2048 + np.sort(rng.choice(1024, 900, replace=False))
    for idx in (r1, r2):
        D[idx] = (np.outer(rng.integers(1, p, size=len(idx)), v0)
                  + np.outer(rng.integers(1, p, size=len(idx)), v1)) % p
    D[r2[699]] = w
    R, r, pc = oracle.rref_dense(D.astype(np.uint16), p)
    assert r == 3
    T = torch.from_numpy(D.astype(np.uint16).view(np.int16)).cuda()
    ech = fl.echelon_d(T, p, rows, cols, mode)
    torch.cuda.synchronize()
    rank = int(u32(ech.rank)[0])
    assert rank == 3
    assert np.array_equal(u32(ech.pivcol)[:rank], pc)
    assert np.array_equal(u16(T)[:rank], R[:rank])
    assert not u16(T)[rank:].any()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("w", [1, 2, 4])
@pytest.mark.parametrize("mode", MODES)
def test_reduce_neworder_parity(name, w, mode):
    """Sec. 4.3: D - C A^{-1} B without X, equal to the oracle's reduction
    (which itself equals the paper's row-by-row Algorithm of Sec. 4.3)."""
    g, r = CASES[name], ref(name)
    s = r["split"]
    sp = fl.split(*up(g), g["m"], g["n"], g["p"], ml_width=w)
    Dt = fl.reduce_neworder(sp, mode)
    torch.cuda.synchronize()
    assert np.array_equal(u16(Dt)[:s["mD"], :s["nB"]], r["Dt"])


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("w", [1, 2])
def test_reduce_from_trsm_planes(name, w):
    """Dt from the limb planes of X that the MFMA-form TRSM leaves in its
    workspace (fl_trsm_planes + fl_reduce_cd_planes) equals the oracle's,
    and X itself is unchanged by keeping the planes."""
    g, r = CASES[name], ref(name)
    s = r["split"]
    sp = fl.split(*up(g), g["m"], g["n"], g["p"], ml_width=w)
    if not (s["npiv"] and s["nB"]):  # no X: no planes
        with pytest.raises(fl.FlError):
            fl.trsm(sp, fl.FL_MFMA_I8, keep_planes=True)
        return
    X, planes = fl.trsm(sp, fl.FL_MFMA_I8, keep_planes=True)
    Dt = fl.reduce_cd_planes(sp, planes)
    torch.cuda.synchronize()
    assert np.array_equal(u16(X)[:s["npiv"], :s["nB"]], r["X"])
    if s["mD"]:
        assert np.array_equal(u16(Dt)[:s["mD"], :s["nB"]], r["Dt"])


def test_reduce_from_trsm_planes_many_blocks():
    """Planes of a TRSM with several superblocks, ragged nB and npiv, and a
    reduce whose 128-row tiles span several K ranges."""
    g = flgen.fl_matrix(m=1500, n=1800, npiv=1100, rank_d=250, density=0.04, p=65521, seed=43)
    r = oracle.fl_rref(g)
    sp = fl.split(*up(g), g["m"], g["n"], g["p"], ml_width=2)
    X, planes = fl.trsm(sp, fl.FL_MFMA_I8, keep_planes=True)
    Dt = fl.reduce_cd_planes(sp, planes)
    Dt2 = fl.reduce_cd(sp, X, fl.FL_MFMA_I8)
    torch.cuda.synchronize()
    assert np.array_equal(u16(Dt)[:sp.mD, :sp.nB], r["Dt"])
    assert np.array_equal(u16(Dt2)[:sp.mD, :sp.nB], r["Dt"])


@pytest.mark.parametrize("mode", MODES)
def test_reduce_neworder_many_blocks(mode):
    """Several TRSM blocks in the transposed solve, a K range beyond one
    128-column tile, and rank-only use: RREF of the new-order Dt."""
    g = flgen.fl_matrix(m=1500, n=1800, npiv=1100, rank_d=250, density=0.04, p=65521, seed=41)
    r = oracle.fl_rref(g)
    sp = fl.split(*up(g), g["m"], g["n"], g["p"], ml_width=2)
    Dt = fl.reduce_neworder(sp, mode)
    torch.cuda.synchronize()
    assert np.array_equal(u16(Dt)[:sp.mD, :sp.nB], r["Dt"])
    ech = fl.echelon_d(Dt, g["p"], sp.mD, sp.nB, mode)
    torch.cuda.synchronize()
    assert int(u32(ech.rank)[0]) == r["rank_d"]
