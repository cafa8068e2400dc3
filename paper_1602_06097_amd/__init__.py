"""Python binding of libfl, the gfx950 Faugere-Lachartre reduction library.

Argument marshalling only: every step of the reduction runs in the device
library's HIP kernels.  PyTorch provides device memory (``torch.empty`` on
``cuda``, which is HIP on ROCm) and the current stream handle.  If libfl.so
is missing the import of any entry point raises -- there is no CPU fallback.

The function names mirror the C ABI in include/fl.h:

    sp = split(M, p, ml_width)            # FL step 1 (syncs once)
    X  = trsm(sp)                         # step 2: X = A^{-1} B
    Dt = reduce_cd(sp, X, mode)           # step 3: Dt = D - C X
    ech = echelon_d(Dt, p, mD, nB, mode)  # step 4: RREF(Dt) in place
    rref(sp, X, Dt, ech, mode)            # second pass: X <- X'
    R = rref_to_csr(sp, X, Dt, ech)       # step 5: RREF(M) as CSR
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass

import torch

__all__ = ["FL_PLAIN", "FL_MFMA_I8", "FlError", "lib_path", "load", "split", "trsm", "reduce_cd", "reduce_cd_planes", "Planes",
           "reduce_neworder",
           "echelon_d", "rref", "rref_to_csr", "matmul_sub", "fl_reduce", "check_modp", "prof_report",
           "version", "Split", "Echelon", "Batch", "batch_plan", "batch_run", "batch_graph_build",
           "batch_graph_launch", "batch_results", "batch_autotune", "batch_config"]

FL_PLAIN, FL_MFMA_I8 = 0, 1
_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libfl.so")
_lib = None

c_u32, c_u64, c_vp, c_sz = ct.c_uint32, ct.c_uint64, ct.c_void_p, ct.c_size_t


class FlError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


class FlCsr(ct.Structure):
    _fields_ = [("rows", c_u32), ("cols", c_u32), ("nnz", c_u64), ("row_ptr", c_vp),
                ("col", c_vp), ("val", c_vp)]


class FlSplitOut(ct.Structure):
    _fields_ = [(n, c_vp) for n in ("row_perm", "col_perm", "a_gptr", "a_pos", "a_val", "b_ptr",
                                    "b_col", "b_val", "c_gptr", "c_pos", "c_val", "d_ptr", "d_col",
                                    "d_val")]


class FlSplitInfo(ct.Structure):
    _fields_ = [("p", c_u32), ("m", c_u32), ("n", c_u32), ("ml_width", c_u32), ("npiv", c_u32),
                ("nB", c_u32), ("mD", c_u32), ("status", c_u32), ("nnz", c_u64), ("nnzA", c_u64),
                ("nnzB", c_u64), ("nnzC", c_u64), ("nnzD", c_u64), ("lenA", c_u64),
                ("lenC", c_u64)]


FL_BATCH_DIRECT = 0xFFFF


class FlBatchConfig(ct.Structure):
    _fields_ = [("ml_width", c_u32), ("streams", c_u32), ("mfma_min_entries", c_u64), ("queue_per_cu", c_u32),
                ("far_groups", c_u32)]


class FlBatchMatrix(ct.Structure):
    _fields_ = [("row_ptr", c_vp), ("col", c_vp), ("val", c_vp), ("nnz_cap", c_u64), ("rank_max", c_u32),
                ("npiv", c_u32), ("mD", c_u32), ("nB", c_u32), ("mode", ct.c_int), ("status", ct.c_int)]


class FlFileLayout(ct.Structure):
    _fields_ = [("format", c_u32), ("m", c_u32), ("n", c_u32), ("p", c_u64), ("nnz", c_u64), ("b", c_u32),
                ("elem_bytes", c_u32), ("elem_signed", c_u32), ("version", c_u32), ("k", c_u64), ("pnb", c_u64),
                ("pnnz", c_u64), ("off_data", c_u64), ("off_cols", c_u64), ("off_rows", c_u64),
                ("off_polmap", c_u64), ("off_colid", c_u64), ("off_prow", c_u64), ("off_pdata", c_u64),
                ("bytes", c_u64)]


def load():
    """Load libfl.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(lib_path):
        raise ImportError(f"{lib_path} not built: run __graft_entry__.build() "
                          "or python -m paper_1602_06097_amd.build")
    lib = ct.CDLL(lib_path)
    P = ct.POINTER
    sigs = {
        "fl_split": (ct.c_int, [P(FlCsr), c_u32, c_u32, P(FlSplitOut), P(FlSplitInfo), c_vp, c_sz, c_vp]),
        "fl_split_workspace": (c_sz, [c_u32, c_u32, c_u64, c_u32]),
        "fl_trsm": (ct.c_int, [P(FlSplitInfo), P(FlSplitOut), c_vp, c_u64, ct.c_int, c_vp, c_sz, c_vp]),
        "fl_trsm_workspace": (c_sz, [P(FlSplitInfo), ct.c_int]),
        "fl_reduce_cd": (ct.c_int, [P(FlSplitInfo), P(FlSplitOut), c_vp, c_u64, c_vp, c_u64, ct.c_int,
                                    c_vp, c_sz, c_vp]),
        "fl_reduce_cd_workspace": (c_sz, [P(FlSplitInfo), ct.c_int]),
        "fl_trsm_planes": (ct.c_int, [P(FlSplitInfo), c_vp, c_sz, P(c_vp), P(c_vp), P(c_u64), P(c_vp)]),
        "fl_reduce_cd_planes": (ct.c_int, [P(FlSplitInfo), P(FlSplitOut), c_vp, c_vp, c_u64, c_vp, c_vp,
                                           c_u64, c_vp, c_sz, c_vp]),
        "fl_reduce_cd_planes_workspace": (c_sz, [P(FlSplitInfo)]),
        "fl_reduce_neworder": (ct.c_int, [P(FlSplitInfo), P(FlSplitOut), c_vp, c_u64, ct.c_int, c_vp, c_sz, c_vp]),
        "fl_reduce_neworder_workspace": (c_sz, [P(FlSplitInfo), ct.c_int]),
        "fl_echelon_d": (ct.c_int, [c_u32, c_u32, c_u32, c_vp, c_u64, c_vp, c_vp, ct.c_int, c_vp, c_sz,
                                    c_vp]),
        "fl_echelon_d_workspace": (c_sz, [c_u32, c_u32, ct.c_int]),
        "fl_rref": (ct.c_int, [P(FlSplitInfo), P(FlSplitOut), c_vp, c_u64, c_vp, c_u64, c_vp, c_vp,
                               ct.c_int, c_vp, c_sz, c_vp]),
        "fl_rref_workspace": (c_sz, [P(FlSplitInfo), ct.c_int]),
        "fl_rref_csr_size": (ct.c_int, [P(FlSplitInfo), P(FlSplitOut), c_vp, c_u64, c_vp, c_u64, c_vp,
                                        c_vp, c_vp, P(c_u32), P(c_u64), c_vp, c_sz, c_vp]),
        "fl_rref_to_csr": (ct.c_int, [P(FlSplitInfo), P(FlSplitOut), c_vp, c_u64, c_vp, c_u64, c_vp,
                                      c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
        "fl_rref_csr_workspace": (c_sz, [P(FlSplitInfo)]),
        "fl_rref_csr_size_noalloc": (ct.c_int, [P(FlSplitInfo), P(FlSplitOut), c_vp, c_u64, c_vp, c_u64, c_vp,
                                                c_vp, c_vp, P(c_u32), P(c_u64), c_vp]),
        "fl_rref_csr_noalloc_scratch_bytes": (c_sz, []),
        "fl_split32": (ct.c_int, [P(FlCsr), c_u32, c_u32, P(FlSplitOut), P(FlSplitInfo), c_vp, c_sz, c_vp]),
        "fl_trsm32": (ct.c_int, [P(FlSplitInfo), P(FlSplitOut), c_vp, c_u64, ct.c_int, c_vp, c_sz, c_vp]),
        "fl_trsm32_workspace": (c_sz, [P(FlSplitInfo), ct.c_int]),
        "fl_reduce_cd32": (ct.c_int, [P(FlSplitInfo), P(FlSplitOut), c_vp, c_u64, c_vp, c_u64, ct.c_int,
                                      c_vp, c_sz, c_vp]),
        "fl_reduce_cd32_workspace": (c_sz, [P(FlSplitInfo), ct.c_int]),
        "fl_echelon_d32": (ct.c_int, [c_u32, c_u32, c_u32, c_vp, c_u64, c_vp, c_vp, ct.c_int, c_vp, c_sz,
                                      c_vp]),
        "fl_echelon_d32_workspace": (c_sz, [c_u32, c_u32, ct.c_int]),
        "fl_rref32": (ct.c_int, [P(FlSplitInfo), P(FlSplitOut), c_vp, c_u64, c_vp, c_u64, c_vp, c_vp,
                                 ct.c_int, c_vp, c_sz, c_vp]),
        "fl_rref32_workspace": (c_sz, [P(FlSplitInfo), ct.c_int]),
        "fl_rref32_csr_size": (ct.c_int, [P(FlSplitInfo), P(FlSplitOut), c_vp, c_u64, c_vp, c_u64, c_vp,
                                          c_vp, c_vp, P(c_u32), P(c_u64), c_vp, c_sz, c_vp]),
        "fl_rref32_to_csr": (ct.c_int, [P(FlSplitInfo), P(FlSplitOut), c_vp, c_u64, c_vp, c_u64, c_vp,
                                        c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
        "fl_rref32_csr_workspace": (c_sz, [P(FlSplitInfo)]),
        "fl_matmul_sub": (ct.c_int, [c_u32, c_u32, c_u32, c_u32, c_vp, c_u64, c_vp, c_u64, c_vp, c_u64,
                                     ct.c_int, c_vp, c_sz, c_vp]),
        "fl_matmul_sub_workspace": (c_sz, [c_u32, c_u32, c_u32, ct.c_int]),
        "fl_status_string": (ct.c_char_p, [ct.c_int]),
        "fl_last_error": (ct.c_char_p, []),
        "fl_version": (ct.c_char_p, []),
        "fl_check_modp": (ct.c_int, [P(c_u32), c_u32, c_vp, c_vp]),
        "fl_batch_split_workspace": (c_sz, [P(FlCsr), c_u32, c_u32]),
        "fl_batch_plan": (ct.c_int, [P(FlCsr), c_u32, c_u32, P(FlBatchConfig), c_vp, c_sz, P(c_vp), c_vp]),
        "fl_batch_run_workspace": (c_sz, [c_vp]),
        "fl_batch_run": (ct.c_int, [c_vp, c_vp, c_sz, c_vp]),
        "fl_batch_graph_build": (ct.c_int, [c_vp, c_vp, c_sz, c_vp]),
        "fl_batch_graph_launch": (ct.c_int, [c_vp, c_vp]),
        "fl_batch_summary": (c_vp, [c_vp, c_vp]),
        "fl_batch_matrix_info": (ct.c_int, [c_vp, c_u32, c_vp, P(FlBatchMatrix)]),
        "fl_batch_get_config": (None, [c_vp, P(FlBatchConfig)]),
        "fl_batch_autotune": (ct.c_int, [P(FlCsr), c_u32, c_u32, c_vp, c_sz, c_vp, c_sz, P(FlBatchConfig),
                                         P(ct.c_double), c_vp]),
        "fl_batch_free": (None, [c_vp]),
        "fl_file_layout_parse": (ct.c_int, [c_vp, c_u64, c_u32, P(FlFileLayout)]),
        "fl_file_decode_workspace": (c_sz, [P(FlFileLayout)]),
        "fl_file_decode": (ct.c_int, [P(FlFileLayout), c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
        "fl_prof_enable": (None, [ct.c_int]),
        "fl_prof_reset": (None, []),
        "fl_prof_report": (c_sz, [ct.c_char_p, c_sz]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(lib, name)
        f.restype, f.argtypes = res, args
    _lib = lib
    return lib


def version() -> str:
    return load().fl_version().decode()


def _check(st: int, where: str):
    if st != 0:
        lib = load()
        raise FlError(st, where, f"{lib.fl_status_string(st).decode()}; {lib.fl_last_error().decode()}")


def _stream():
    return c_vp(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return c_vp(t.data_ptr()) if t is not None and t.numel() else c_vp(None)


def _dev():
    return torch.device("cuda")


def _ws(nbytes: int):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=_dev())


def _ld(cols: int) -> int:
    """Leading dimension used for dense buffers: a multiple of 64 elements."""
    return max(64, (cols + 63) // 64 * 64)


@dataclass
class Split:
    info: FlSplitInfo
    out: FlSplitOut
    bufs: dict

    @property
    def npiv(self): return self.info.npiv

    @property
    def mD(self): return self.info.mD

    @property
    def nB(self): return self.info.nB

    @property
    def p(self): return self.info.p


@dataclass
class Echelon:
    rank: torch.Tensor    # device uint32 [1]
    pivcol: torch.Tensor  # device uint32 [min(rows, cols)]
    rows: int
    cols: int


def split(row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, m: int, n: int, p: int,
          ml_width: int = 2) -> Split:
    """FL step 1 on a device CSR matrix (row_ptr uint64 [m+1], col uint32/int32
    [nnz], val uint16/int16 [nnz]).  Allocates the outputs at their upper-bound
    capacities and returns the sizes after the library's single sync."""
    lib = load()
    nnz = int(col.numel())
    w = int(ml_width)
    G = (m + w - 1) // w + 1
    d = _dev()

    def e(n_, dt):
        return torch.empty(max(n_, 1), dtype=dt, device=d)

    bufs = dict(row_perm=e(m, torch.int32), col_perm=e(n, torch.int32),
                a_gptr=e(G, torch.int64), a_pos=e(nnz, torch.int32), a_val=e(w * nnz, torch.int16),
                b_ptr=e(m + 1, torch.int64), b_col=e(nnz, torch.int32), b_val=e(nnz, torch.int16),
                c_gptr=e(G, torch.int64), c_pos=e(nnz, torch.int32), c_val=e(w * nnz, torch.int16),
                d_ptr=e(m + 1, torch.int64), d_col=e(nnz, torch.int32), d_val=e(nnz, torch.int16))
    out = FlSplitOut(**{k: c_vp(v.data_ptr()) for k, v in bufs.items()})
    M = FlCsr(m, n, nnz, _ptr(row_ptr), _ptr(col), _ptr(val))
    info = FlSplitInfo()
    ws = _ws(lib.fl_split_workspace(m, n, nnz, w))
    st = lib.fl_split(ct.byref(M), p, w, ct.byref(out), ct.byref(info), _ptr(ws), ws.numel(), _stream())
    _check(st, "fl_split")
    bufs["_input"] = (row_ptr, col, val)
    return Split(info=info, out=out, bufs=bufs)


class Planes:
    """The int8 limb planes of X left in an MFMA-form TRSM workspace (which
    this object keeps alive): Xh/Xl device addresses and their row stride."""

    def __init__(self, ws, xh: int, xl: int, ldp: int, row_end: int | None = None):
        self.ws, self.xh, self.xl, self.ldp, self.row_end = ws, xh, xl, ldp, row_end


def trsm(sp: Split, mode: int = FL_PLAIN, keep_planes: bool = False):
    """X = A^{-1} B as a dense (npiv x ld) uint16 tensor (int16 storage).
    With keep_planes (FL_MFMA_I8 only) returns (X, Planes): the limb planes of
    X in the TRSM workspace, for reduce_cd_planes."""
    lib = load()
    ld = _ld(sp.nB)
    X = torch.empty((max(sp.npiv, 1), ld), dtype=torch.int16, device=_dev())
    ws = _ws(lib.fl_trsm_workspace(ct.byref(sp.info), mode))
    st = lib.fl_trsm(ct.byref(sp.info), ct.byref(sp.out), _ptr(X), ld, mode, _ptr(ws), ws.numel(),
                     _stream())
    _check(st, "fl_trsm")
    if not keep_planes:
        return X
    if mode != FL_MFMA_I8:
        raise ValueError("trsm: keep_planes needs the FL_MFMA_I8 form")
    xh, xl, ldp, rend = ct.c_void_p(), ct.c_void_p(), c_u64(), ct.c_void_p()
    st = lib.fl_trsm_planes(ct.byref(sp.info), _ptr(ws), ws.numel(), ct.byref(xh), ct.byref(xl), ct.byref(ldp),
                            ct.byref(rend))
    _check(st, "fl_trsm_planes")
    return X, Planes(ws, xh.value, xl.value, ldp.value, rend.value)


def reduce_cd_planes(sp: Split, planes: Planes) -> torch.Tensor:
    """reduce_cd (FL_MFMA_I8) from the limb planes of X that trsm kept."""
    lib = load()
    ld = _ld(sp.nB)
    Dt = torch.empty((max(sp.mD, 1), ld), dtype=torch.int16, device=_dev())
    ws = _ws(lib.fl_reduce_cd_planes_workspace(ct.byref(sp.info)))
    st = lib.fl_reduce_cd_planes(ct.byref(sp.info), ct.byref(sp.out), planes.xh, planes.xl, planes.ldp,
                                 planes.row_end, _ptr(Dt), ld, _ptr(ws), ws.numel(), _stream())
    _check(st, "fl_reduce_cd_planes")
    return Dt


def reduce_cd(sp: Split, X: torch.Tensor, mode: int = FL_PLAIN) -> torch.Tensor:
    lib = load()
    ld = _ld(sp.nB)
    Dt = torch.empty((max(sp.mD, 1), ld), dtype=torch.int16, device=_dev())
    ws = _ws(lib.fl_reduce_cd_workspace(ct.byref(sp.info), mode))
    st = lib.fl_reduce_cd(ct.byref(sp.info), ct.byref(sp.out), _ptr(X), X.shape[1], _ptr(Dt), ld,
                          mode, _ptr(ws), ws.numel(), _stream())
    _check(st, "fl_reduce_cd")
    return Dt


def reduce_neworder(sp: Split, mode: int = FL_PLAIN) -> torch.Tensor:
    """Dt = D - C A^{-1} B without X (Sec. 4.3), dense (mD x ld) uint16."""
    lib = load()
    ld = _ld(sp.nB)
    Dt = torch.empty((max(sp.mD, 1), ld), dtype=torch.int16, device=_dev())
    ws = _ws(lib.fl_reduce_neworder_workspace(ct.byref(sp.info), mode))
    st = lib.fl_reduce_neworder(ct.byref(sp.info), ct.byref(sp.out), _ptr(Dt), ld, mode, _ptr(ws), ws.numel(),
                                _stream())
    _check(st, "fl_reduce_neworder")
    return Dt


def echelon_d(Dt: torch.Tensor, p: int, rows: int, cols: int, mode: int = FL_PLAIN) -> Echelon:
    lib = load()
    d = _dev()
    rank = torch.zeros(1, dtype=torch.int32, device=d)
    piv = torch.zeros(max(min(rows, cols), 1), dtype=torch.int32, device=d)
    ws = _ws(lib.fl_echelon_d_workspace(rows, cols, mode))
    st = lib.fl_echelon_d(p, rows, cols, _ptr(Dt), Dt.shape[1], _ptr(rank), _ptr(piv), mode,
                          _ptr(ws), ws.numel(), _stream())
    _check(st, "fl_echelon_d")
    return Echelon(rank=rank, pivcol=piv, rows=rows, cols=cols)


def rref(sp: Split, X: torch.Tensor, Dt: torch.Tensor, ech: Echelon, mode: int = FL_PLAIN) -> None:
    lib = load()
    ws = _ws(lib.fl_rref_workspace(ct.byref(sp.info), mode))
    st = lib.fl_rref(ct.byref(sp.info), ct.byref(sp.out), _ptr(X), X.shape[1], _ptr(Dt), Dt.shape[1],
                     _ptr(ech.rank), _ptr(ech.pivcol), mode, _ptr(ws), ws.numel(), _stream())
    _check(st, "fl_rref")


def rref_to_csr(sp: Split, Xp: torch.Tensor, Dt: torch.Tensor, ech: Echelon):
    """RREF(M) in original column order: (row_ptr int64, col int32, val int16, rank)."""
    lib = load()
    maxr = min(sp.mD, sp.nB)
    row_ptr = torch.empty(sp.npiv + maxr + 1, dtype=torch.int64, device=_dev())
    ws = _ws(lib.fl_rref_csr_workspace(ct.byref(sp.info)))
    h_rank, h_nnz = c_u32(0), c_u64(0)
    args = (ct.byref(sp.info), ct.byref(sp.out), _ptr(Xp), Xp.shape[1], _ptr(Dt), Dt.shape[1],
            _ptr(ech.rank), _ptr(ech.pivcol))
    st = lib.fl_rref_csr_size(*args, _ptr(row_ptr), ct.byref(h_rank), ct.byref(h_nnz), _ptr(ws),
                              ws.numel(), _stream())
    _check(st, "fl_rref_csr_size")
    nnz = int(h_nnz.value)
    col = torch.empty(max(nnz, 1), dtype=torch.int32, device=_dev())
    val = torch.empty(max(nnz, 1), dtype=torch.int16, device=_dev())
    st = lib.fl_rref_to_csr(*args, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(ws), ws.numel(), _stream())
    _check(st, "fl_rref_to_csr")
    rank = int(h_rank.value)
    return row_ptr[:rank + 1], col[:nnz], val[:nnz], rank


def rref_to_csr_noalloc(sp: Split, Xp: torch.Tensor, Dt: torch.Tensor, ech: Echelon, row_ptr: torch.Tensor,
                        col: torch.Tensor, val: torch.Tensor):
    """rref_to_csr into caller-provided outputs, with no device allocation by
    the library: the size query runs on the library's static scratch
    (fl_rref_csr_size_noalloc).  row_ptr must hold npiv + min(mD, nB) + 1
    entries and col/val the nonzeros.  Returns (nnz, rank)."""
    lib = load()
    h_rank, h_nnz = c_u32(0), c_u64(0)
    args = (ct.byref(sp.info), ct.byref(sp.out), _ptr(Xp), Xp.shape[1], _ptr(Dt), Dt.shape[1],
            _ptr(ech.rank), _ptr(ech.pivcol))
    st = lib.fl_rref_csr_size_noalloc(*args, _ptr(row_ptr), ct.byref(h_rank), ct.byref(h_nnz), _stream())
    _check(st, "fl_rref_csr_size_noalloc")
    nnz = int(h_nnz.value)
    if nnz > min(col.numel(), val.numel()):
        raise ValueError(f"col/val hold {min(col.numel(), val.numel())} entries, RREF(M) has {nnz}")
    st = lib.fl_rref_to_csr(*args, _ptr(row_ptr), _ptr(col), _ptr(val), None, 0, _stream())
    _check(st, "fl_rref_to_csr")
    return nnz, int(h_rank.value)


def matmul_sub(p: int, C: torch.Tensor, X: torch.Tensor, D: torch.Tensor, M: int, N: int, K: int,
               mode: int = FL_PLAIN) -> None:
    """D[:M, :N] -= C[:M, :K] X[:K, :N] mod p, in place (dense uint16 in int16 storage)."""
    lib = load()
    ws = _ws(lib.fl_matmul_sub_workspace(M, N, K, mode))
    st = lib.fl_matmul_sub(p, M, N, K, _ptr(C), C.shape[1], _ptr(X), X.shape[1], _ptr(D), D.shape[1],
                           mode, _ptr(ws), ws.numel(), _stream())
    _check(st, "fl_matmul_sub")


def fl_reduce(row_ptr, col, val, m: int, n: int, p: int, mode: int = FL_PLAIN, ml_width: int = 2,
              keep: bool = False) -> dict:
    """The whole hot path on one matrix already resident on the device.
    With keep=True, copies of X = A^{-1}B and Dt = D - C X are returned too."""
    sp = split(row_ptr, col, val, m, n, p, ml_width)
    X = trsm(sp, mode)
    Dt = reduce_cd(sp, X, mode)
    res = dict(split=sp)
    if keep:
        res["X"], res["Dt"] = X.clone(), Dt.clone()
    ech = echelon_d(Dt, p, sp.mD, sp.nB, mode)
    rref(sp, X, Dt, ech, mode)
    res.update(echelon=ech, Xp=X, RD=Dt, rref=rref_to_csr(sp, X, Dt, ech))
    return res


class Batch:
    """A planned batch: the library's plan object plus the two device arenas
    (the split arena must outlive the plan; the run arena holds every
    result)."""

    def __init__(self, handle, count, split_arena, run_arena, inputs):
        self.handle, self.count = handle, count
        self.split_arena, self.run_arena, self._inputs = split_arena, run_arena, inputs

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.fl_batch_free(self.handle)
            self.handle = None


def _csr_array(mats):
    arr = (FlCsr * len(mats))()
    for i, (rp, ci, vv, m, n) in enumerate(mats):
        arr[i] = FlCsr(m, n, int(ci.numel()) if m else 0, _ptr(rp), _ptr(ci), _ptr(vv))
    return arr


def _config(cfg):
    if cfg is None:
        return None
    return FlBatchConfig(int(cfg.get("ml_width", 0)), int(cfg.get("streams", 0)),
                         int(cfg.get("mfma_min_entries", 0)), int(cfg.get("queue_per_cu", 0)),
                         int(cfg.get("far_groups", 0)))


def batch_plan(mats, p: int, config: dict | None = None) -> Batch:
    """Plan a batch of device CSR matrices [(row_ptr, col, val, m, n), ...]:
    splits all of them with one synchronisation.  config: dict with
    ml_width / streams / mfma_min_entries (0 = default); None = the autotuned
    configuration for batches of this shape, else the defaults."""
    lib = load()
    arr = _csr_array(mats)
    cfg = _config(config)
    w_alloc = (cfg.ml_width or 2) if cfg is not None else 4
    split_arena = _ws(lib.fl_batch_split_workspace(arr, len(mats), w_alloc))
    h = c_vp()
    st = lib.fl_batch_plan(arr, len(mats), p, ct.byref(cfg) if cfg is not None else None,
                           _ptr(split_arena), split_arena.numel(), ct.byref(h), _stream())
    _check(st, "fl_batch_plan")
    run_arena = _ws(lib.fl_batch_run_workspace(h))
    return Batch(h, len(mats), split_arena, run_arena, list(mats))


def batch_run(b: Batch) -> None:
    lib = load()
    _check(lib.fl_batch_run(b.handle, _ptr(b.run_arena), b.run_arena.numel(), _stream()), "fl_batch_run")


def batch_graph_build(b: Batch) -> None:
    lib = load()
    _check(lib.fl_batch_graph_build(b.handle, _ptr(b.run_arena), b.run_arena.numel(), _stream()),
           "fl_batch_graph_build")


def batch_graph_launch(b: Batch) -> None:
    lib = load()
    _check(lib.fl_batch_graph_launch(b.handle, _stream()), "fl_batch_graph_launch")


def batch_config(b: Batch) -> dict:
    lib = load()
    c = FlBatchConfig()
    lib.fl_batch_get_config(b.handle, ct.byref(c))
    return dict(ml_width=c.ml_width, streams=c.streams, mfma_min_entries=c.mfma_min_entries,
                queue_per_cu=c.queue_per_cu, far_groups=c.far_groups)


def batch_results(b: Batch) -> list:
    """Per matrix: dict(rank, nnz, status, mode, row_ptr, col, val) with the
    CSR of RREF(M) as views of the run arena (synchronises the stream)."""
    lib = load()
    torch.cuda.current_stream().synchronize()
    base = b.run_arena.data_ptr()
    sp = lib.fl_batch_summary(b.handle, _ptr(b.run_arena))
    off = sp - base
    summ = b.run_arena[off:off + 32 * b.count].view(torch.int64).view(b.count, 4).cpu().numpy()
    out = []
    for i in range(b.count):
        info = FlBatchMatrix()
        _check(lib.fl_batch_matrix_info(b.handle, i, _ptr(b.run_arena), ct.byref(info)),
               "fl_batch_matrix_info")
        rank, nnz, status = int(summ[i, 0]), int(summ[i, 1]), int(summ[i, 2])
        d = dict(rank=rank, nnz=nnz, status=status, mode=int(info.mode), npiv=info.npiv, mD=info.mD,
                 nB=info.nB)
        if info.row_ptr:
            o = info.row_ptr - base
            d["row_ptr"] = b.run_arena[o:o + 8 * (rank + 1)].view(torch.int64)
            o = info.col - base
            d["col"] = b.run_arena[o:o + 4 * nnz].view(torch.int32)
            o = info.val - base
            d["val"] = b.run_arena[o:o + 2 * nnz].view(torch.int16)
        out.append(d)
    return out


def batch_autotune(mats, p: int, run_bytes: int | None = None):
    """Time candidate configurations on this batch; returns (config, ms).
    The choice is remembered for batch_plan(config=None) on batches of the
    same shape."""
    lib = load()
    arr = _csr_array(mats)
    split_arena = _ws(lib.fl_batch_split_workspace(arr, len(mats), 4))
    if run_bytes is None:
        # the largest run arena among the candidates: plan the all-MFMA,
        # 16-branch configuration to size it
        h = c_vp()
        cfg = FlBatchConfig(2, 16, 1)
        _check(lib.fl_batch_plan(arr, len(mats), p, ct.byref(cfg), _ptr(split_arena), split_arena.numel(),
                                 ct.byref(h), _stream()), "fl_batch_plan")
        run_bytes = int(lib.fl_batch_run_workspace(h) * 1.25)
        lib.fl_batch_free(h)
    run_arena = _ws(run_bytes)
    best, ms = FlBatchConfig(), ct.c_double(0)
    st = lib.fl_batch_autotune(arr, len(mats), p, _ptr(split_arena), split_arena.numel(), _ptr(run_arena),
                               run_arena.numel(), ct.byref(best), ct.byref(ms), _stream())
    _check(st, "fl_batch_autotune")
    return dict(ml_width=best.ml_width, streams=best.streams, mfma_min_entries=best.mfma_min_entries,
                queue_per_cu=best.queue_per_cu, far_groups=best.far_groups), ms.value


def prof_report() -> dict:
    """Per-site launch profile collected while fl_prof_enable(1) was set:
    {site: {"count": launches, "total_ms": summed HIP-event time}}."""
    import json
    lib = load()
    need = lib.fl_prof_report(None, 0)
    buf = ct.create_string_buffer(need)
    lib.fl_prof_report(buf, need)
    out = json.loads(buf.value.decode())
    for v in out.values():
        v["avg_ms"] = v["total_ms"] / max(v["count"], 1)
    return out


def check_modp(primes) -> list:
    lib = load()
    arr = (c_u32 * len(primes))(*primes)
    out = torch.zeros(len(primes), dtype=torch.int64, device=_dev())
    st = lib.fl_check_modp(arr, len(primes), _ptr(out), _stream())
    _check(st, "fl_check_modp")
    torch.cuda.synchronize()
    return [int(x) for x in out.cpu()]


# ---- 32-bit field characteristic (uint32 residues, p < 2^32) --------------------
# fl_csr32 / fl_split_out32 have the layouts of fl_csr / fl_split_out (every
# array is a pointer), so the same ctypes structures marshal them.

def split32(row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, m: int, n: int, p: int,
            ml_width: int = 2) -> Split:
    """split over uint32 residues (val: int32 storage of uint32 values)."""
    lib = load()
    nnz = int(col.numel())
    w = int(ml_width)
    G = (m + w - 1) // w + 1
    d = _dev()

    def e(n_, dt):
        return torch.empty(max(n_, 1), dtype=dt, device=d)

    bufs = dict(row_perm=e(m, torch.int32), col_perm=e(n, torch.int32),
                a_gptr=e(G, torch.int64), a_pos=e(nnz, torch.int32), a_val=e(w * nnz, torch.int32),
                b_ptr=e(m + 1, torch.int64), b_col=e(nnz, torch.int32), b_val=e(nnz, torch.int32),
                c_gptr=e(G, torch.int64), c_pos=e(nnz, torch.int32), c_val=e(w * nnz, torch.int32),
                d_ptr=e(m + 1, torch.int64), d_col=e(nnz, torch.int32), d_val=e(nnz, torch.int32))
    out = FlSplitOut(**{k: c_vp(v.data_ptr()) for k, v in bufs.items()})
    M = FlCsr(m, n, nnz, _ptr(row_ptr), _ptr(col), _ptr(val))
    info = FlSplitInfo()
    ws = _ws(lib.fl_split_workspace(m, n, nnz, w))
    st = lib.fl_split32(ct.byref(M), p, w, ct.byref(out), ct.byref(info), _ptr(ws), ws.numel(), _stream())
    _check(st, "fl_split32")
    bufs["_input"] = (row_ptr, col, val)
    return Split(info=info, out=out, bufs=bufs)


def trsm32(sp: Split, mode: int = FL_PLAIN) -> torch.Tensor:
    lib = load()
    ld = _ld(sp.nB)
    X = torch.empty((max(sp.npiv, 1), ld), dtype=torch.int32, device=_dev())
    ws = _ws(lib.fl_trsm32_workspace(ct.byref(sp.info), mode))
    _check(lib.fl_trsm32(ct.byref(sp.info), ct.byref(sp.out), _ptr(X), ld, mode, _ptr(ws), ws.numel(), _stream()),
           "fl_trsm32")
    return X


def reduce_cd32(sp: Split, X: torch.Tensor, mode: int = FL_PLAIN) -> torch.Tensor:
    lib = load()
    ld = _ld(sp.nB)
    Dt = torch.empty((max(sp.mD, 1), ld), dtype=torch.int32, device=_dev())
    ws = _ws(lib.fl_reduce_cd32_workspace(ct.byref(sp.info), mode))
    _check(lib.fl_reduce_cd32(ct.byref(sp.info), ct.byref(sp.out), _ptr(X), X.shape[1], _ptr(Dt), ld, mode,
                              _ptr(ws), ws.numel(), _stream()), "fl_reduce_cd32")
    return Dt


def echelon_d32(Dt: torch.Tensor, p: int, rows: int, cols: int, mode: int = FL_PLAIN) -> Echelon:
    lib = load()
    d = _dev()
    rank = torch.zeros(1, dtype=torch.int32, device=d)
    piv = torch.zeros(max(min(rows, cols), 1), dtype=torch.int32, device=d)
    ws = _ws(lib.fl_echelon_d32_workspace(rows, cols, mode))
    _check(lib.fl_echelon_d32(p, rows, cols, _ptr(Dt), Dt.shape[1], _ptr(rank), _ptr(piv), mode, _ptr(ws),
                              ws.numel(), _stream()), "fl_echelon_d32")
    return Echelon(rank=rank, pivcol=piv, rows=rows, cols=cols)


def rref32(sp: Split, X: torch.Tensor, Dt: torch.Tensor, ech: Echelon, mode: int = FL_PLAIN) -> None:
    lib = load()
    ws = _ws(lib.fl_rref32_workspace(ct.byref(sp.info), mode))
    _check(lib.fl_rref32(ct.byref(sp.info), ct.byref(sp.out), _ptr(X), X.shape[1], _ptr(Dt), Dt.shape[1],
                         _ptr(ech.rank), _ptr(ech.pivcol), mode, _ptr(ws), ws.numel(), _stream()), "fl_rref32")


def rref32_to_csr(sp: Split, Xp: torch.Tensor, Dt: torch.Tensor, ech: Echelon):
    """RREF(M) in original column order: (row_ptr int64, col int32, val int32 (uint32 values), rank)."""
    lib = load()
    maxr = min(sp.mD, sp.nB)
    row_ptr = torch.empty(sp.npiv + maxr + 1, dtype=torch.int64, device=_dev())
    ws = _ws(lib.fl_rref32_csr_workspace(ct.byref(sp.info)))
    h_rank, h_nnz = c_u32(0), c_u64(0)
    args = (ct.byref(sp.info), ct.byref(sp.out), _ptr(Xp), Xp.shape[1], _ptr(Dt), Dt.shape[1],
            _ptr(ech.rank), _ptr(ech.pivcol))
    _check(lib.fl_rref32_csr_size(*args, _ptr(row_ptr), ct.byref(h_rank), ct.byref(h_nnz), _ptr(ws), ws.numel(),
                                  _stream()), "fl_rref32_csr_size")
    nnz = int(h_nnz.value)
    col = torch.empty(max(nnz, 1), dtype=torch.int32, device=_dev())
    val = torch.empty(max(nnz, 1), dtype=torch.int32, device=_dev())
    _check(lib.fl_rref32_to_csr(*args, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(ws), ws.numel(), _stream()),
           "fl_rref32_to_csr")
    rank = int(h_rank.value)
    return row_ptr[:rank + 1], col[:nnz], val[:nnz], rank


def fl_reduce32(row_ptr, col, val, m: int, n: int, p: int, mode: int = FL_PLAIN, ml_width: int = 2,
                keep: bool = False) -> dict:
    """The whole hot path over uint32 residues on one device-resident matrix."""
    sp = split32(row_ptr, col, val, m, n, p, ml_width)
    X = trsm32(sp, mode)
    Dt = reduce_cd32(sp, X, mode)
    res = dict(split=sp)
    if keep:
        res["X"], res["Dt"] = X.clone(), Dt.clone()
    ech = echelon_d32(Dt, p, sp.mD, sp.nB, mode)
    rref32(sp, X, Dt, ech, mode)
    res.update(echelon=ech, Xp=X, RD=Dt, rref=rref32_to_csr(sp, X, Dt, ech))
    return res
