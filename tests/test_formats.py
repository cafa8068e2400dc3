"""The binary matrix formats of Sec. 3.2: host-side layout parse (CPU) and
the device decode (GPU), round-tripped through the writers."""
import ctypes as ct
import os

import numpy as np
import pytest

import flgen
import oracle
import paper_1602_06097_amd as fl
from paper_1602_06097_amd import formats


def _parse(path, fmt):
    lib = fl.load()
    raw = np.fromfile(path, dtype=np.uint8)
    lay = fl.FlFileLayout()
    st = lib.fl_file_layout_parse(raw.ctypes.data_as(ct.c_void_p), raw.size, fmt, ct.byref(lay))
    return st, lay, raw


def _mat(seed=3):
    return flgen.random_sparse(60, 90, 0.15, 65521, seed=seed, zero_rows=0.1, dup_rows=0.3)


def _runs_example():
    # rows: {0,1,2,5}, {}, {7}, {3,4}
    rp = np.array([0, 4, 4, 5, 7], np.uint64)
    col = np.array([0, 1, 2, 5, 7, 3, 4], np.uint32)
    val = np.array([1, 2, 3, 4, 1, 2, 3], np.uint16)
    return dict(m=4, n=8, p=7, row_ptr=rp, col=col, val=val)


def test_format1_layout(tmp_path):
    g = _mat()
    path = os.path.join(tmp_path, "m1.bin")
    formats.write_format1(path, g["m"], g["n"], g["p"], g["row_ptr"], g["col"], g["val"])
    st, lay, raw = _parse(path, 1)
    assert st == 0
    nnz = int(g["row_ptr"][-1])
    assert (lay.m, lay.n, lay.p, lay.nnz) == (g["m"], g["n"], g["p"], nnz)
    assert lay.bytes == raw.size == 20 + 6 * nnz + 4 * g["m"]
    assert np.array_equal(np.frombuffer(raw, np.uint16, nnz, lay.off_data), g["val"])
    assert np.array_equal(np.frombuffer(raw, np.uint32, nnz, lay.off_cols), g["col"])


def test_format2_layout_and_encoding(tmp_path):
    g = _runs_example()
    path = os.path.join(tmp_path, "m2.bin")
    formats.write_format2(path, g["m"], g["n"], g["p"], g["row_ptr"], g["col"], g["val"], version=5)
    st, lay, raw = _parse(path, 2)
    assert st == 0
    assert (lay.m, lay.n, lay.p, lay.nnz, lay.elem_bytes, lay.elem_signed, lay.version) == (4, 8, 7, 7, 2, 0, 5)
    colid = np.frombuffer(raw, np.uint64, lay.k, lay.off_colid)
    # runs: (0, 3), 5 | 2^31 ; 7 | 2^31 ; (3, 2)
    assert list(colid) == [0, 3, 5 | (1 << 31), 7 | (1 << 31), 3, 2]
    # rows {1,2,3,4}, {1}, {2,3}: three distinct coefficient vectors, the empty row a fourth
    assert lay.pnb == 4 and lay.pnnz == 7


@pytest.mark.parametrize("fmt", [1, 2])
def test_layout_rejects_truncated_and_inconsistent_files(tmp_path, fmt):
    g = _mat(5)
    path = os.path.join(tmp_path, "m.bin")
    w = formats.write_format1 if fmt == 1 else formats.write_format2
    w(path, g["m"], g["n"], g["p"], g["row_ptr"], g["col"], g["val"])
    raw = np.fromfile(path, dtype=np.uint8)
    lib = fl.load()
    lay = fl.FlFileLayout()
    for cut in (3, 19, raw.size // 2, raw.size - 1):
        part = raw[:cut].copy()
        assert lib.fl_file_layout_parse(part.ctypes.data_as(ct.c_void_p), part.size, fmt, ct.byref(lay)) == 1
    bad = raw.copy()
    off = 20 + 6 * int(g["row_ptr"][-1]) if fmt == 1 else 28
    bad[off] ^= 1  # one row length off by one: lengths no longer add up to nnz
    assert lib.fl_file_layout_parse(bad.ctypes.data_as(ct.c_void_p), bad.size, fmt, ct.byref(lay)) == 1
    assert b"nnz" in lib.fl_last_error()
    assert lib.fl_file_layout_parse(raw.ctypes.data_as(ct.c_void_p), raw.size, 3, ct.byref(lay)) == 1


@pytest.mark.gpu
@pytest.mark.parametrize("fmt,elem", [(1, "u16"), (2, "u16"), (2, "i16"), (2, "u8"), (2, "i32"), (2, "u64")])
def test_device_decode_round_trip(tmp_path, fmt, elem):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = 251 if elem in ("u8",) else 65521
    g = flgen.fl_matrix(m=400, n=560, npiv=300, rank_d=60, density=0.06, p=p, seed=17)
    path = os.path.join(tmp_path, "m.bin")
    if fmt == 1:
        formats.write_format1(path, g["m"], g["n"], p, g["row_ptr"], g["col"], g["val"])
    else:
        formats.write_format2(path, g["m"], g["n"], p, g["row_ptr"], g["col"], g["val"], elem=elem)
    rp, ci, vv, (m, n, pp) = formats.read_matrix(path, fmt)
    assert (m, n, pp) == (g["m"], g["n"], p)
    assert np.array_equal(rp.cpu().numpy().view(np.uint64), g["row_ptr"])
    assert np.array_equal(ci.cpu().numpy().view(np.uint32), g["col"])
    assert np.array_equal(vv.cpu().numpy().view(np.uint16), g["val"])
    # and the reduction of the decoded matrix
    res = fl.fl_reduce(rp, ci, vv, m, n, p, mode=fl.FL_MFMA_I8)
    torch.cuda.synchronize()
    o = oracle.fl_rref(g, keep=False)
    orp, oci, ov = o["rref"]
    frp, fci, fvv, rank = res["rref"]
    assert rank == o["rank"]
    assert np.array_equal(frp.cpu().numpy().view(np.uint64), orp)
    assert np.array_equal(fci.cpu().numpy().view(np.uint32), oci)
    assert np.array_equal(fvv.cpu().numpy().view(np.uint16), ov)


@pytest.mark.gpu
def test_device_decode_reports_a_run_past_the_row_data(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    g = _runs_example()
    path = os.path.join(tmp_path, "m2.bin")
    formats.write_format2(path, g["m"], g["n"], g["p"], g["row_ptr"], g["col"], g["val"])
    raw = np.fromfile(path, dtype=np.uint8)
    st, lay, _ = _parse(path, 2)
    colid = np.frombuffer(raw, np.uint64, lay.k, lay.off_colid).copy()
    colid[1] = 30  # run of 30 columns: beyond nnz and n
    raw[lay.off_colid:lay.off_colid + 8 * lay.k] = colid.view(np.uint8)
    raw.tofile(path)
    with pytest.raises(fl.FlError):
        formats.read_matrix(path, 2)
