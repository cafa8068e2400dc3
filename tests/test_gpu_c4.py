"""The whole batch workload: 256 FL matrices over F_65521 with rows
log-uniform in [500, 20,000] (columns 1.3-1.6 x rows, 70-85% pivot rows,
density 2-15%, planted Schur complements), 1.75e9 nonzeros in all, reduced
by one batched plan and run.

  * every matrix: the batched CSR of RREF(M) is bit-identical to the
    single-matrix path on the same device input;
  * every matrix: rank(M) = pivot rows + planted rank, the rows of RREF(M)
    whose pivot is not a pivot column of A are zero on those columns and
    equal the planted RREF V of the Schur complement on the others, and the
    rowspace certificate (RREF structure + Freivalds) holds;
  * a seeded subset including the smallest and the largest matrix: SHA-256
    of the CSR arrays equal to the CPU oracle's (stored digests, written by
    tests/golden/make_c4_oracle_digests.py from the oracle alone: the
    largest matrix takes the oracle several minutes)."""
import hashlib
import json
import os

import numpy as np
import pytest
import torch

import flgen
import paper_1602_06097_amd as fl
from certify import certify_rref, csr

pytestmark = pytest.mark.gpu

P = 65521
CHUNKS = 8
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def c4():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fl.load()
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    mats = flgen.config_batch("c4", workers=workers)
    d = torch.device("cuda")
    dev = [(torch.from_numpy(g["row_ptr"].view(np.int64)).to(d), torch.from_numpy(g["col"].view(np.int32)).to(d),
            torch.from_numpy(g["val"].view(np.int16)).to(d), g["m"], g["n"]) for g in mats]
    b = fl.batch_plan(dev, P, None)
    fl.batch_run(b)
    res = fl.batch_results(b)
    yield mats, dev, b, res
    del b, res, dev
    torch.cuda.empty_cache()


def _host(r):
    if r["rank"] == 0:
        return np.zeros(1, np.uint64), np.zeros(0, np.uint32), np.zeros(0, np.uint16)
    return (r["row_ptr"].cpu().numpy().view(np.uint64), r["col"].cpu().numpy().view(np.uint32),
            r["val"].cpu().numpy().view(np.uint16))


def test_c4_shape(c4):
    mats, _, _, res = c4
    assert len(mats) == len(res) == 256
    rows = [g["m"] for g in mats]
    assert min(rows) >= 500 and max(rows) <= 20000
    assert sum(len(g["col"]) for g in mats) > 1.5e9
    assert all(r["status"] == 0 for r in res)


def test_c4_batched_equals_single_matrix_path(c4):
    mats, dev, _, res = c4
    for i, (rp, ci, vv, m, n) in enumerate(dev):
        one = fl.fl_reduce(rp, ci, vv, m, n, P, mode=fl.FL_MFMA_I8)
        orp, oci, ov, rank = one["rref"]
        r = res[i]
        assert r["rank"] == rank, i
        nnz = int(orp[-1].item()) if rank else 0
        assert r["nnz"] == nnz, i
        if rank:
            assert torch.equal(r["row_ptr"], orp[:rank + 1]), i
            assert torch.equal(r["col"], oci[:nnz]), i
            assert torch.equal(r["val"], ov[:nnz]), i
        del one, orp, oci, ov


@pytest.mark.parametrize("chunk", range(CHUNKS))
def test_c4_planted_rank_V_and_certificate(c4, chunk):
    mats, _, _, res = c4
    for i in range(chunk, len(mats), CHUNKS):
        g, r = mats[i], res[i]
        npiv = len(g["piv_cols"])
        assert r["rank"] == npiv + g["rank_d"], i
        rp, ci, v = _host(r)
        R = csr(rp, ci, v, r["rank"], g["n"])
        M = csr(g["row_ptr"], g["col"], g["val"], g["m"], g["n"])
        certify_rref(M, R, P, r["rank"], trials=2, seed=i)
        # rows of RREF(M) led by a column outside the pivot columns of A
        lead = ci[rp[:-1].astype(np.int64)] if r["rank"] else np.zeros(0, np.uint32)
        is_piv = np.zeros(g["n"], bool)
        is_piv[g["piv_cols"]] = True
        d_rows = np.nonzero(~is_piv[lead])[0]
        assert len(d_rows) == g["rank_d"], i
        RD = R[d_rows]
        assert RD[:, g["piv_cols"]].nnz == 0, i
        V = RD[:, g["nonpiv_cols"]].tocsr()
        V.sort_indices()
        Vp = g["V"].tocsr()
        Vp.sort_indices()
        assert V.shape == Vp.shape, i
        assert np.array_equal(V.indptr, Vp.indptr), i
        assert np.array_equal(V.indices, Vp.indices), i
        assert np.array_equal(V.data.astype(np.int64), Vp.data.astype(np.int64)), i


def test_c4_subset_equals_oracle(c4):
    mats, _, _, res = c4
    with open(os.path.join(HERE, "golden", "c4_oracle_digests.json")) as f:
        ref = json.load(f)
    rows = [g["m"] for g in mats]
    subset = {int(k): v for k, v in ref["matrices"].items()}
    assert int(np.argmin(rows)) in subset and int(np.argmax(rows)) in subset
    for i, o in subset.items():
        g, r = mats[i], res[i]
        assert (g["m"], g["n"], len(g["col"])) == (o["m"], o["n"], o["nnz_in"]), i
        assert (r["rank"], r["nnz"]) == (o["rank"], o["nnz"]), i
        rp, ci, v = _host(r)
        assert hashlib.sha256(rp.tobytes()).hexdigest() == o["row_ptr_sha256"], i
        assert hashlib.sha256(ci.tobytes()).hexdigest() == o["col_sha256"], i
        assert hashlib.sha256(v.tobytes()).hexdigest() == o["val_sha256"], i
