"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point that include/fl.h declares, and rejects host-checkable
argument errors before touching the device."""
import ctypes as ct
import os
import re

import pytest

import paper_1602_06097_amd as fl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fl.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fl_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_five_steps():
    names = _declared()
    for n in ("fl_split", "fl_trsm", "fl_reduce_cd", "fl_echelon_d", "fl_rref",
              "fl_rref_csr_size", "fl_rref_to_csr", "fl_matmul_sub"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ct.CDLL(fl.lib_path)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_and_version():
    lib = fl.load()
    assert lib.fl_version().decode().startswith("fl-gfx950")
    for s in range(8):
        assert lib.fl_status_string(s)
    assert lib.fl_status_string(0).decode() == "ok"


def test_workspace_sizes_are_host_computable():
    lib = fl.load()
    assert lib.fl_split_workspace(60000, 80000, 137_000_000, 2) > 0
    assert lib.fl_echelon_d_workspace(15000, 35000, fl.FL_PLAIN) > 0
    assert lib.fl_echelon_d_workspace(15000, 35000, fl.FL_MFMA_I8) > lib.fl_echelon_d_workspace(
        15000, 35000, fl.FL_PLAIN)
    assert lib.fl_matmul_sub_workspace(100, 100, 100, fl.FL_PLAIN) == 0
    assert lib.fl_matmul_sub_workspace(100, 100, 100, fl.FL_MFMA_I8) >= 2 * 128 * 128 * 2
    info = fl.FlSplitInfo(p=65521, m=10, n=12, ml_width=2, npiv=6, nB=6, mD=4)
    assert lib.fl_rref_workspace(ct.byref(info), fl.FL_PLAIN) > 0
    assert lib.fl_rref_csr_workspace(ct.byref(info)) > 0


def _split_call(p=65521, w=2, ws_bytes=1 << 20, rows=4, with_out=True, csr_null=False):
    lib = fl.load()
    M = fl.FlCsr(rows, 5, 3, ct.c_void_p(None if csr_null else 8), ct.c_void_p(8), ct.c_void_p(8))
    out = fl.FlSplitOut(**{f: ct.c_void_p(8) for f, _ in fl.FlSplitOut._fields_}) if with_out else None
    info = fl.FlSplitInfo()
    return lib.fl_split(ct.byref(M), p, w, ct.byref(out) if with_out else None, ct.byref(info),
                        ct.c_void_p(8 if ws_bytes else None), ws_bytes, None)


@pytest.mark.parametrize("kw,code", [
    (dict(p=1), 1), (dict(p=65537), 1), (dict(w=3), 1), (dict(w=16), 1),
    (dict(with_out=False), 1), (dict(csr_null=True), 1), (dict(ws_bytes=0), 2), (dict(ws_bytes=16), 2),
])
def test_split_rejects_bad_arguments_on_the_host(kw, code):
    assert _split_call(**kw) == code
    assert fl.load().fl_last_error()


def test_split_of_empty_matrix_needs_no_device():
    lib = fl.load()
    M = fl.FlCsr(0, 0, 0, None, None, None)
    out = fl.FlSplitOut()
    info = fl.FlSplitInfo()
    ws = ct.create_string_buffer(4096)
    need = lib.fl_split_workspace(0, 0, 0, 2)
    assert need <= 4096
    assert lib.fl_split(ct.byref(M), 7, 2, ct.byref(out), ct.byref(info), ct.cast(ws, ct.c_void_p),
                        4096, None) == 0
    assert info.npiv == 0 and info.nB == 0 and info.mD == 0 and info.p == 7


def test_dense_entry_points_reject_bad_arguments():
    lib = fl.load()
    # p out of range, bad mode, misaligned / short leading dimensions
    assert lib.fl_echelon_d(70000, 4, 4, ct.c_void_p(8), 4, ct.c_void_p(8), ct.c_void_p(8), 0, None, 0, None) == 1
    assert lib.fl_echelon_d(7, 4, 4, ct.c_void_p(8), 4, ct.c_void_p(8), ct.c_void_p(8), 5, None, 0, None) == 1
    assert lib.fl_echelon_d(7, 4, 6, ct.c_void_p(8), 6, ct.c_void_p(8), ct.c_void_p(8), 0, None, 0, None) == 1
    assert lib.fl_echelon_d(7, 4, 4, ct.c_void_p(8), 4, ct.c_void_p(8), ct.c_void_p(8), 0, None, 0, None) == 2
    assert lib.fl_matmul_sub(7, 4, 4, 4, ct.c_void_p(8), 4, ct.c_void_p(8), 2, ct.c_void_p(8), 4, 0, None, 0, None) == 1
    assert lib.fl_matmul_sub(7, 4, 4, 4, ct.c_void_p(8), 4, ct.c_void_p(8), 4, ct.c_void_p(8), 4, 1, None, 0, None) == 2
    info = fl.FlSplitInfo(p=7, m=10, n=12, ml_width=2, npiv=6, nB=6, mD=4, status=3)
    assert lib.fl_trsm(ct.byref(info), ct.byref(fl.FlSplitOut()), ct.c_void_p(8), 8, 0, None, 0, None) == 1
    info.status = 0
    assert lib.fl_trsm(ct.byref(info), ct.byref(fl.FlSplitOut()), ct.c_void_p(8), 6, 0, None, 0, None) == 1
    assert lib.fl_trsm(ct.byref(info), ct.byref(fl.FlSplitOut()), ct.c_void_p(8), 8, 7, None, 0, None) == 1


def _batch_csr(count=3):
    arr = (fl.FlCsr * count)()
    for i in range(count):
        arr[i] = fl.FlCsr(100 + 50 * i, 150 + 60 * i, 1000 * (i + 1), ct.c_void_p(8), ct.c_void_p(8),
                          ct.c_void_p(8))
    return arr


def test_batch_split_workspace_is_host_computable():
    lib = fl.load()
    arr = _batch_csr()
    w1, w2, w4 = (lib.fl_batch_split_workspace(arr, 3, w) for w in (1, 2, 4))
    assert 0 < w1 < w2 < w4
    assert lib.fl_batch_split_workspace(arr, 0, 2) == 0


def test_batch_host_argument_errors():
    lib = fl.load()
    arr = _batch_csr()
    h = ct.c_void_p()
    need = lib.fl_batch_split_workspace(arr, 3, 2)
    cfg = fl.FlBatchConfig(2, 4, 0)
    ARG, WS = 1, 2
    assert lib.fl_batch_plan(arr, 0, 65521, ct.byref(cfg), ct.c_void_p(256), need, ct.byref(h), None) == ARG
    assert lib.fl_batch_plan(arr, 3, 1, ct.byref(cfg), ct.c_void_p(256), need, ct.byref(h), None) == ARG
    bad_w = fl.FlBatchConfig(3, 4, 0)
    assert lib.fl_batch_plan(arr, 3, 65521, ct.byref(bad_w), ct.c_void_p(256), need, ct.byref(h), None) == ARG
    bad_s = fl.FlBatchConfig(2, 17, 0)
    assert lib.fl_batch_plan(arr, 3, 65521, ct.byref(bad_s), ct.c_void_p(256), need, ct.byref(h), None) == ARG
    assert lib.fl_batch_plan(arr, 3, 65521, ct.byref(cfg), ct.c_void_p(256), need - 1, ct.byref(h), None) == WS
    assert lib.fl_batch_plan(arr, 3, 65521, ct.byref(cfg), None, need, ct.byref(h), None) == WS
    assert not h.value
    assert lib.fl_batch_run(None, ct.c_void_p(256), 1 << 20, None) == ARG
    assert lib.fl_batch_graph_launch(None, None) == ARG
    assert lib.fl_batch_run_workspace(None) == 0
    lib.fl_batch_free(None)
