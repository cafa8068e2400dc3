"""Writers and a reader for the binary matrix formats of Sec. 3.2.

The writers are host code (numpy); the reader parses the header with the
library (fl_file_layout_parse, which also checks the section sizes) and
decodes the sections on the device (fl_file_decode).
"""
from __future__ import annotations

import ctypes as ct

import numpy as np

_SINGLE = 1 << 31


def write_format1(path: str, m: int, n: int, p: int, row_ptr, col, val) -> None:
    """Format 1: m, n, p (u32), nnz (u64), data (u16), cols (u32), rows (u32 lengths)."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    nnz = int(rp[-1]) if len(rp) else 0
    with open(path, "wb") as f:
        f.write(np.array([m, n, p], dtype=np.uint32).tobytes())
        f.write(np.array([nnz], dtype=np.uint64).tobytes())
        f.write(np.asarray(val, dtype=np.uint16)[:nnz].tobytes())
        f.write(np.asarray(col, dtype=np.uint32)[:nnz].tobytes())
        f.write(np.diff(rp).astype(np.uint32).tobytes())


def _runs(cols: np.ndarray) -> list:
    """colid items of one row: runs of consecutive columns."""
    out = []
    i = 0
    while i < len(cols):
        j = i + 1
        while j < len(cols) and cols[j] == cols[j - 1] + 1:
            j += 1
        if j - i > 1:
            out += [int(cols[i]), j - i]
        else:
            out.append(int(cols[i]) | _SINGLE)
        i = j
    return out


def write_format2(path: str, m: int, n: int, p: int, row_ptr, col, val, elem: str = "u16",
                  version: int = 0) -> None:
    """Format 2: rows with equal coefficient vectors share one polynomial."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.uint32)
    val = np.asarray(val, dtype=np.uint16)
    types = {"u8": (np.uint8, 0, 0), "i8": (np.int8, 1, 0), "u16": (np.uint16, 0, 1), "i16": (np.int16, 1, 1),
             "u32": (np.uint32, 0, 2), "i32": (np.int32, 1, 2), "u64": (np.uint64, 0, 3), "i64": (np.int64, 1, 3)}
    dt, signed, v = types[elem]
    b = signed | (v << 1) | (version << 3)
    polys, polmap, colid = {}, [], []
    for i in range(m):
        s, e = int(rp[i]), int(rp[i + 1])
        key = val[s:e].tobytes()
        if key not in polys:
            polys[key] = len(polys)
        polmap.append(polys[key])
        colid += _runs(col[s:e])
    order = sorted(polys.items(), key=lambda kv: kv[1])
    prow = [len(k) // 2 for k, _ in order]
    pdata = np.concatenate([np.frombuffer(k, dtype=np.uint16) for k, _ in order]) if order else np.zeros(0, np.uint16)
    if signed:  # store residues above p/2 as negative numbers
        pd = pdata.astype(np.int64)
        pd = np.where(pd > p // 2, pd - p, pd)
    else:
        pd = pdata.astype(np.int64)
    with open(path, "wb") as f:
        f.write(np.array([b, m, n], dtype=np.uint32).tobytes())
        f.write(np.array([p, int(rp[-1]) if len(rp) else 0], dtype=np.uint64).tobytes())
        f.write(np.diff(rp).astype(np.uint32).tobytes())
        f.write(np.array(polmap, dtype=np.uint32).tobytes())
        f.write(np.array([len(colid)], dtype=np.uint64).tobytes())
        f.write(np.array(colid, dtype=np.uint64).tobytes())
        f.write(np.array([len(prow)], dtype=np.uint32).tobytes())
        f.write(np.array([len(pd)], dtype=np.uint64).tobytes())
        f.write(np.array(prow, dtype=np.uint32).tobytes())
        f.write(pd.astype(dt).tobytes())


def read_matrix(path: str, fmt: int):
    """Decode a Format 1 or 2 file on the device: returns (row_ptr int64,
    col int32, val int16) device tensors and (m, n, p)."""
    import torch

    from . import FlFileLayout, FlError, _check, _ptr, _stream, _ws, load

    lib = load()
    raw = np.fromfile(path, dtype=np.uint8)
    lay = FlFileLayout()
    st = lib.fl_file_layout_parse(raw.ctypes.data_as(ct.c_void_p), raw.size, fmt, ct.byref(lay))
    _check(st, "fl_file_layout_parse")
    dev = torch.device("cuda")

    def section(off, count, dtype):
        a = np.frombuffer(raw, dtype=dtype, count=count, offset=off) if count else np.zeros(0, dtype)
        return torch.from_numpy(a.copy()).to(dev)

    m, nnz = lay.m, lay.nnz
    row_ptr = torch.empty(m + 1, dtype=torch.int64, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = _ws(lib.fl_file_decode_workspace(ct.byref(lay)))
    if fmt == 1:
        val = section(lay.off_data, nnz, np.int16)
        col = section(lay.off_cols, nnz, np.int32)
        rows = section(lay.off_rows, m, np.int32)
        secs = [val, col, rows]
    else:
        rows = section(lay.off_rows, m, np.int32)
        polmap = section(lay.off_polmap, m, np.int32)
        colid = section(lay.off_colid, lay.k, np.int64)
        prow = section(lay.off_prow, lay.pnb, np.int32)
        pdata = section(lay.off_pdata, lay.pnnz * lay.elem_bytes, np.uint8)
        secs = [rows, polmap, colid, prow, pdata]
        col = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
        val = torch.empty(max(nnz, 1), dtype=torch.int16, device=dev)
    arr = (ct.c_void_p * len(secs))(*[_ptr(s) for s in secs])
    st = lib.fl_file_decode(ct.byref(lay), arr, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(status), _ptr(ws),
                            ws.numel(), _stream())
    _check(st, "fl_file_decode")
    torch.cuda.current_stream().synchronize()
    code = int(status.item())
    if code:
        raise FlError(code, "fl_file_decode", f"malformed file (status bits {code:#x})")
    return row_ptr, col[:nnz], val[:nnz], (m, lay.n, int(lay.p))
