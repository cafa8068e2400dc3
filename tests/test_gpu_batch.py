"""Parity of the batched form (many matrices of uneven sizes in one plan and
one run) with the CPU oracle, for several configurations, for graph replays
and for the autotuned configuration.  Every comparison is bit-exact."""
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


def _batch_inputs():
    mats = flgen.batch_matrices(14, 60, 1500, P, seed=flgen.BASE_SEED + 40)
    mats.append(flgen.random_sparse(180, 260, 0.06, P, seed=3, zero_rows=0.05, dup_rows=0.1))
    mats.append(flgen.fl_matrix(m=300, n=500, npiv=300, rank_d=0, density=0.05, p=P, seed=15))
    mats.append(flgen.fl_matrix(m=500, n=700, npiv=400, rank_d=0, density=0.05, p=P, seed=14))
    empty_rows = flgen.random_sparse(40, 30, 0.0, P, seed=5)          # no nonzero at all
    mats.append(empty_rows)
    mats.append(dict(m=0, n=17, p=P, row_ptr=np.zeros(1, np.uint64), col=np.zeros(0, np.uint32),
                     val=np.zeros(0, np.uint16)))                     # no rows
    mats.append(flgen.fl_matrix(m=1300, n=1900, npiv=950, rank_d=230, density=0.05, p=P, seed=11))
    return mats


MATS = _batch_inputs()
_REF = {}


def ref(i):
    if i not in _REF:
        _REF[i] = oracle.fl_rref(MATS[i], keep=False)
    return _REF[i]


def _up(mats):
    d = torch.device("cuda")
    out = []
    for g in mats:
        out.append((torch.from_numpy(g["row_ptr"].view(np.int64).copy()).to(d),
                    torch.from_numpy(g["col"].view(np.int32).copy()).to(d),
                    torch.from_numpy(g["val"].view(np.int16).copy()).to(d), g["m"], g["n"]))
    return out


def _check_all(results, mats=MATS, skip=()):
    assert len(results) == len(mats)
    for i, r in enumerate(results):
        if i in skip:
            continue
        o = ref(i)
        assert r["status"] == 0, i
        assert r["rank"] == o["rank"], i
        orp, oci, ov = o["rref"]
        assert r["nnz"] == int(orp[-1]), i
        if r["rank"] == 0:
            continue
        assert np.array_equal(r["row_ptr"].cpu().numpy().view(np.uint64), orp), i
        assert np.array_equal(r["col"].cpu().numpy().view(np.uint32), oci), i
        assert np.array_equal(r["val"].cpu().numpy().view(np.uint16), ov), i


CONFIGS = [
    None,
    dict(ml_width=2, streams=8, mfma_min_entries=0),
    dict(ml_width=1, streams=1, mfma_min_entries=1),               # everything MFMA, one branch
    dict(ml_width=4, streams=3, mfma_min_entries=(1 << 64) - 1),   # everything VALU
    dict(ml_width=8, streams=16, mfma_min_entries=1 << 16),
    # work-queue launches: one workgroup per unit (most tasks per workgroup),
    # four, and one workgroup per tile; far-update column groups
    dict(ml_width=2, streams=4, mfma_min_entries=1 << 16, queue_per_cu=1, far_groups=7),
    dict(ml_width=2, streams=4, mfma_min_entries=1, queue_per_cu=4, far_groups=512),
    dict(ml_width=2, streams=4, mfma_min_entries=(1 << 64) - 1, queue_per_cu=1),
    dict(ml_width=2, streams=4, mfma_min_entries=1 << 16, queue_per_cu=fl.FL_BATCH_DIRECT),
]


@pytest.mark.parametrize("cfg", CONFIGS, ids=["tuned-or-default", "default", "w1-s1-mfma", "w4-s3-plain",
                                              "w8-s16-mixed", "queue1-g7", "queue4-g512-mfma",
                                              "queue1-plain", "direct"])
def test_batch_equals_oracle(cfg):
    b = fl.batch_plan(_up(MATS), P, cfg)
    fl.batch_run(b)
    _check_all(fl.batch_results(b))


def test_batch_modes_follow_threshold():
    b = fl.batch_plan(_up(MATS), P, dict(ml_width=2, streams=4, mfma_min_entries=1 << 16))
    fl.batch_run(b)
    res = fl.batch_results(b)
    for r in res:
        dense = (r["npiv"] + r["mD"]) * r["nB"]
        assert r["mode"] == (fl.FL_MFMA_I8 if dense >= (1 << 16) else fl.FL_PLAIN)
    _check_all(res)


def test_batch_graph_replays_match_eager():
    """The captured run replayed several times, with unrelated eager work and
    a wipe of the result region between replays: every replay must rebuild
    the same results."""
    b = fl.batch_plan(_up(MATS), P, dict(ml_width=2, streams=4, mfma_min_entries=1 << 16))
    fl.batch_graph_build(b)
    torch.cuda.synchronize()
    for rep in range(3):
        b.run_arena.fill_(0xA5 if rep % 2 else 0)
        junk = torch.arange(1 << 20, device="cuda", dtype=torch.int32).sum()
        fl.batch_graph_launch(b)
        torch.cuda.synchronize()
        assert int(junk) >= 0
        _check_all(fl.batch_results(b))


def test_batch_reports_bad_matrix_and_reduces_the_rest():
    mats = MATS[:4] + [dict(MATS[4])] + MATS[5:8]
    bad = dict(mats[4])
    col = bad["col"].copy()
    col[len(col) // 2] = bad["n"] + 5  # column out of range
    bad["col"] = col
    mats[4] = bad
    b = fl.batch_plan(_up(mats), P, dict(ml_width=2, streams=2, mfma_min_entries=1 << 16))
    fl.batch_run(b)
    res = fl.batch_results(b)
    assert res[4]["status"] != 0 and res[4]["rank"] == 0 and res[4]["nnz"] == 0
    _check_all(res, mats=mats, skip=(4,))


def test_batch_autotune_choice_is_used_and_exact():
    mats = _up(MATS)
    cfg, ms = fl.batch_autotune(mats, P)
    assert cfg["ml_width"] in (1, 2, 4) and 1 <= cfg["streams"] <= 16 and ms > 0
    assert cfg["queue_per_cu"] in (fl.FL_BATCH_DIRECT, 1, 2, 4) and cfg["far_groups"] in (32, 128, 512)
    b = fl.batch_plan(mats, P, None)
    assert fl.batch_config(b) == cfg
    fl.batch_run(b)
    _check_all(fl.batch_results(b))
