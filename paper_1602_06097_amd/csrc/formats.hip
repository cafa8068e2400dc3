// formats.hip -- the binary matrix file formats of the paper (Sec. 3.2):
// host-side layout parse, device-side decode to CSR.
//
// Format 1 is CSR with row lengths: m, n, p (u32), nnz (u64), data (u16 x nnz),
// cols (u32 x nnz), rows (u32 x m).
// Format 2 separates positions and coefficients: b (u32: element type in the
// low 3 bits), m, n (u32), p, nnz (u64), rows (u32 x m, row lengths), polmap
// (u32 x m: the polynomial whose coefficients fill row i), k (u64), colid
// (u64 x k: column runs -- a run of s > 1 consecutive columns from f is the
// pair f, s; a single column f is stored as f | 2^31), pnb (u32), pnnz (u64),
// prow (u32 x pnb: polynomial sizes), pdata (pnnz elements of the type in b).
//
// Decoding Format 2 on the device: the colid stream is a sequence of tokens of
// one or two items; which items start a token is a prefix property (an item
// follows a pair start or not), found by a scan over the two-state transition
// functions of the items.  Token lengths are scanned into output positions
// and every token writes its columns; coefficients are copied row by row
// from the row's polynomial, with the element type converted to a residue.
#include <hipcub/hipcub.hpp>
#include <string.h>

#include "fl_internal.h"

namespace {

// A transition function of the token parser on the states {0: token start
// expected, 1: run length expected}, as bit 0 = f(0), bit 1 = f(1).
struct Compose {
    __host__ __device__ uint8_t operator()(uint8_t a, uint8_t b) const {
        const uint8_t r0 = (b >> ((a >> 0) & 1)) & 1, r1 = (b >> ((a >> 1) & 1)) & 1;
        return (uint8_t)(r0 | (r1 << 1));
    }
};
constexpr uint8_t kIdentity = 2;  // f(0) = 0, f(1) = 1

constexpr uint64_t kSingle = (uint64_t)1 << 31;

__global__ void k_item_fn(uint64_t k, const uint64_t *__restrict__ colid, uint8_t *fn) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= k) return;
    // from "start": a single column stays at "start", a pair start goes to
    // "length"; from "length" always back to "start"
    fn[t] = (colid[t] & kSingle) ? 0 : 1;
}

// Token lengths (0 for items that are not token starts); errors: a pair
// start without its length item.
__global__ void k_token_len(uint64_t k, const uint64_t *__restrict__ colid, const uint8_t *__restrict__ state,
                            uint64_t *len, uint32_t *status) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= k) return;
    uint64_t L = 0;
    if ((state[t] & 1) == 0) {  // state before item t is "start"
        if (colid[t] & kSingle) {
            L = 1;
        } else if (t + 1 < k) {
            L = colid[t + 1];
        } else {
            atomicOr(status, 1u);
        }
    }
    len[t] = L;
}

__global__ void k_token_emit(uint64_t k, uint64_t nnz, uint32_t n, const uint64_t *__restrict__ colid,
                             const uint64_t *__restrict__ len, const uint64_t *__restrict__ at, uint32_t *col,
                             uint32_t *status) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= k) return;
    const uint64_t L = len[t];
    if (!L) return;
    const uint64_t f = colid[t] & (kSingle - 1), o = at[t];
    if (o + L > nnz || f + L > n) {
        atomicOr(status, 2u);
        return;
    }
    for (uint64_t r = 0; r < L; r++) col[o + r] = (uint32_t)(f + r);
}

// Coefficients of row i = the coefficients of polynomial polmap[i].
__global__ __launch_bounds__(256) void k_rows_values(uint32_t m, uint32_t p, uint32_t pnb, uint32_t elem_bytes,
                                                     int elem_signed, const uint32_t *__restrict__ rows,
                                                     const uint64_t *__restrict__ row_ptr,
                                                     const uint32_t *__restrict__ polmap,
                                                     const uint32_t *__restrict__ prow,
                                                     const uint64_t *__restrict__ poff, const uint8_t *__restrict__ pdata,
                                                     uint16_t *val, uint32_t *status) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= m) return;
    const uint32_t pm = polmap[i];
    if (pm >= pnb || prow[pm] != rows[i]) {
        if (lane == 0) atomicOr(status, 4u);
        return;
    }
    const uint64_t src = poff[pm], dst = row_ptr[i];
    for (uint32_t r = lane; r < rows[i]; r += 64) {
        const uint8_t *e = pdata + (src + r) * elem_bytes;
        int64_t v;
        if (elem_bytes == 1) v = elem_signed ? (int64_t)(int8_t)e[0] : (int64_t)e[0];
        else if (elem_bytes == 2) v = elem_signed ? (int64_t)*(const int16_t *)e : (int64_t)*(const uint16_t *)e;
        else if (elem_bytes == 4) v = elem_signed ? (int64_t)*(const int32_t *)e : (int64_t)*(const uint32_t *)e;
        else v = *(const int64_t *)e;
        if (elem_bytes == 8 && !elem_signed) v = (int64_t)((uint64_t)v % p);
        int64_t rmod = v % (int64_t)p;
        if (rmod < 0) rmod += p;
        val[dst + r] = (uint16_t)rmod;
    }
}

__global__ void k_u32_to_u64(uint64_t n, const uint32_t *__restrict__ in, uint64_t *out) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[t] = in[t];
}

template <class T> bool rd(const uint8_t *b, uint64_t size, uint64_t off, T *v) {
    if (off + sizeof(T) > size) return false;
    memcpy(v, b + off, sizeof(T));
    return true;
}

inline unsigned grid(uint64_t n) { return (unsigned)((n + 255) / 256); }

struct F2Ws {
    uint8_t *fn, *state;
    uint64_t *len, *at, *poff, *prow64, *rows64, *scantmp;
    void *cub;
    size_t cub_bytes;
};

size_t f2_layout(const fl_file_layout *L, void *ws, F2Ws *out) {
    WsCarve c(ws);
    F2Ws w = {};
    const uint64_t k = L->k ? L->k : 1, m = L->m ? L->m : 1, pnb = L->pnb ? L->pnb : 1;
    w.fn = c.take<uint8_t>(k);
    w.state = c.take<uint8_t>(k);
    w.len = c.take<uint64_t>(k + 1);
    w.at = c.take<uint64_t>(k + 1);
    w.poff = c.take<uint64_t>(pnb + 1);
    w.prow64 = c.take<uint64_t>(pnb + 1);
    w.rows64 = c.take<uint64_t>(m + 1);
    uint64_t big = k + 1 > m + 1 ? k + 1 : m + 1;
    if (pnb + 1 > big) big = pnb + 1;
    w.scantmp = c.take<uint64_t>(fl_scan_tmp_elems(big));
    size_t b = 0;
    (void)hipcub::DeviceScan::ExclusiveScan(nullptr, b, (const uint8_t *)nullptr, (uint8_t *)nullptr, Compose(),
                                            kIdentity, (int)k, (hipStream_t)0);
    w.cub_bytes = b;
    w.cub = c.take<char>(b);
    if (out) *out = w;
    return c.off;
}

}  // namespace

extern "C" fl_status fl_file_layout_parse(const void *file, uint64_t bytes, uint32_t format, fl_file_layout *out) {
    FL_ARG(file && out, "fl_file_layout_parse: NULL argument");
    FL_ARG(format == 1 || format == 2, "fl_file_layout_parse: format must be 1 or 2");
    const uint8_t *b = (const uint8_t *)file;
    fl_file_layout L = {};
    L.format = format;
    uint64_t o = 0;
    auto bad = [&](const char *what) {
        fl_set_error(what);
        return FL_ERR_ARG;
    };
    if (format == 1) {
        uint32_t m, n, p;
        uint64_t nnz;
        if (!rd(b, bytes, 0, &m) || !rd(b, bytes, 4, &n) || !rd(b, bytes, 8, &p) || !rd(b, bytes, 12, &nnz))
            return bad("fl_file_layout_parse: truncated Format 1 header");
        if (nnz > bytes) return bad("fl_file_layout_parse: nnz exceeds the file size");
        L.m = m;
        L.n = n;
        L.p = p;
        L.nnz = nnz;
        o = 20;
        L.off_data = o;
        o += 2 * nnz;
        L.off_cols = o;
        o += 4 * nnz;
        L.off_rows = o;
        o += 4 * (uint64_t)m;
    } else {
        uint32_t bb, m, n, pnb;
        uint64_t p, nnz, k, pnnz;
        if (!rd(b, bytes, 0, &bb) || !rd(b, bytes, 4, &m) || !rd(b, bytes, 8, &n) || !rd(b, bytes, 12, &p) ||
            !rd(b, bytes, 20, &nnz))
            return bad("fl_file_layout_parse: truncated Format 2 header");
        L.b = bb;
        L.elem_signed = bb & 1;
        L.elem_bytes = 1u << ((bb >> 1) & 3);
        L.version = bb >> 3;
        L.m = m;
        L.n = n;
        L.p = p;
        L.nnz = nnz;
        o = 28;
        L.off_rows = o;
        o += 4 * (uint64_t)m;
        L.off_polmap = o;
        o += 4 * (uint64_t)m;
        if (nnz > bytes || o > bytes) return bad("fl_file_layout_parse: sizes exceed the file size");
        if (!rd(b, bytes, o, &k)) return bad("fl_file_layout_parse: truncated Format 2 (k)");
        if (k > bytes) return bad("fl_file_layout_parse: k exceeds the file size");
        L.k = k;
        o += 8;
        L.off_colid = o;
        o += 8 * k;
        if (!rd(b, bytes, o, &pnb) || !rd(b, bytes, o + 4, &pnnz))
            return bad("fl_file_layout_parse: truncated Format 2 (pnb, pnnz)");
        if (pnnz > bytes) return bad("fl_file_layout_parse: pnnz exceeds the file size");
        L.pnb = pnb;
        L.pnnz = pnnz;
        o += 12;
        L.off_prow = o;
        o += 4 * (uint64_t)pnb;
        L.off_pdata = o;
        o += (uint64_t)L.elem_bytes * pnnz;
    }
    L.bytes = o;
    if (o > bytes) return bad("fl_file_layout_parse: file shorter than its header implies");
    if (L.p < 2 || L.p > 65521) return bad("fl_file_layout_parse: p must be in [2, 65521]");
    if (L.m >= (1u << 31) || L.n >= (1u << 31)) return bad("fl_file_layout_parse: dimensions must be < 2^31");
    // the sizes the device decode relies on: row lengths add up to nnz, the
    // polynomial sizes to pnnz, and every row names an existing polynomial of
    // its own length
    uint64_t sum = 0;
    for (uint64_t i = 0; i < L.m; i++) {
        uint32_t r;
        memcpy(&r, b + L.off_rows + 4 * i, 4);
        sum += r;
    }
    if (sum != L.nnz) return bad("fl_file_layout_parse: row lengths do not add up to nnz");
    if (format == 2) {
        uint64_t ps = 0;
        for (uint64_t j = 0; j < L.pnb; j++) {
            uint32_t r;
            memcpy(&r, b + L.off_prow + 4 * j, 4);
            ps += r;
        }
        if (ps != L.pnnz) return bad("fl_file_layout_parse: polynomial sizes do not add up to pnnz");
        for (uint64_t i = 0; i < L.m; i++) {
            uint32_t pm, r, pr;
            memcpy(&pm, b + L.off_polmap + 4 * i, 4);
            memcpy(&r, b + L.off_rows + 4 * i, 4);
            if (pm >= L.pnb) return bad("fl_file_layout_parse: polmap names a missing polynomial");
            memcpy(&pr, b + L.off_prow + 4 * (uint64_t)pm, 4);
            if (pr != r) return bad("fl_file_layout_parse: a row and its polynomial differ in length");
        }
    }
    *out = L;
    return FL_OK;
}

extern "C" size_t fl_file_decode_workspace(const fl_file_layout *L) {
    if (!L) return 0;
    if (L->format == 1) {
        WsCarve c(nullptr);
        c.take<uint64_t>((uint64_t)L->m + 1);
        c.take<uint64_t>(fl_scan_tmp_elems((uint64_t)L->m + 1));
        return c.off;
    }
    return f2_layout(L, nullptr, nullptr);
}

extern "C" fl_status fl_file_decode(const fl_file_layout *L, const void *const *d_sections, uint64_t *row_ptr,
                                    uint32_t *col, uint16_t *val, uint32_t *d_status, void *ws, size_t ws_bytes,
                                    hipStream_t stream) {
    FL_ARG(L && d_sections && row_ptr && d_status, "fl_file_decode: NULL argument");
    FL_ARG(L->format == 1 || L->format == 2, "fl_file_decode: bad layout");
    const uint64_t m = L->m, nnz = L->nnz;
    const size_t need = fl_file_decode_workspace(L);
    if (!ws || ws_bytes < need) {
        fl_set_error("fl_file_decode: workspace too small");
        return FL_ERR_WORKSPACE;
    }
    FL_HIP(fl_fill_u32(d_status, 0, 1, stream));
    if (L->format == 1) {
        // sections: [0] data (u16, copied by the caller into val), [1] cols, [2] rows
        const uint32_t *rows = (const uint32_t *)d_sections[2];
        WsCarve c(ws);
        uint64_t *rows64 = c.take<uint64_t>(m + 1);
        uint64_t *tmp = c.take<uint64_t>(fl_scan_tmp_elems(m + 1));
        if (m) {
            hipLaunchKernelGGL(k_u32_to_u64, dim3(grid(m)), dim3(256), 0, stream, m, rows, rows64);
            FL_LAUNCH_CHECK("k_u32_to_u64");
        }
        FL_HIP(fl_fill_u64(rows64 + m, 0, 1, stream));
        FL_HIP(fl_exclusive_scan_u64(rows64, row_ptr, m + 1, tmp, nullptr, stream));
        (void)col;
        (void)val;
        return FL_OK;
    }
    // Format 2: sections [0] rows, [1] polmap, [2] colid, [3] prow, [4] pdata
    FL_ARG(nnz == 0 || (col && val), "fl_file_decode: NULL col/val");
    FL_ARG(L->k < (1ull << 31), "fl_file_decode: more than 2^31 column items");
    const uint32_t *rows = (const uint32_t *)d_sections[0];
    const uint32_t *polmap = (const uint32_t *)d_sections[1];
    const uint64_t *colid = (const uint64_t *)d_sections[2];
    const uint32_t *prow = (const uint32_t *)d_sections[3];
    const uint8_t *pdata = (const uint8_t *)d_sections[4];
    F2Ws w;
    f2_layout(L, ws, &w);
    const uint64_t k = L->k, pnb = L->pnb;
    // row pointers
    if (m) {
        hipLaunchKernelGGL(k_u32_to_u64, dim3(grid(m)), dim3(256), 0, stream, m, rows, w.rows64);
        FL_LAUNCH_CHECK("k_u32_to_u64");
    }
    FL_HIP(fl_fill_u64(w.rows64 + m, 0, 1, stream));
    FL_HIP(fl_exclusive_scan_u64(w.rows64, row_ptr, m + 1, w.scantmp, nullptr, stream));
    // columns: parse the token stream
    if (k) {
        hipLaunchKernelGGL(k_item_fn, dim3(grid(k)), dim3(256), 0, stream, k, colid, w.fn);
        FL_LAUNCH_CHECK("k_item_fn");
        size_t b = w.cub_bytes;
        FL_HIP(hipcub::DeviceScan::ExclusiveScan(w.cub, b, w.fn, w.state, Compose(), kIdentity, (int)k, stream));
        hipLaunchKernelGGL(k_token_len, dim3(grid(k)), dim3(256), 0, stream, k, colid, (const uint8_t *)w.state,
                           w.len, d_status);
        FL_LAUNCH_CHECK("k_token_len");
        FL_HIP(fl_fill_u64(w.len + k, 0, 1, stream));
        FL_HIP(fl_exclusive_scan_u64(w.len, w.at, k + 1, w.scantmp, nullptr, stream));
        hipLaunchKernelGGL(k_token_emit, dim3(grid(k)), dim3(256), 0, stream, k, nnz, L->n, colid,
                           (const uint64_t *)w.len, (const uint64_t *)w.at, col, d_status);
        FL_LAUNCH_CHECK("k_token_emit");
    }
    // coefficients
    if (pnb) {
        hipLaunchKernelGGL(k_u32_to_u64, dim3(grid(pnb)), dim3(256), 0, stream, pnb, prow, w.prow64);
        FL_LAUNCH_CHECK("k_u32_to_u64");
    }
    FL_HIP(fl_fill_u64(w.prow64 + pnb, 0, 1, stream));
    FL_HIP(fl_exclusive_scan_u64(w.prow64, w.poff, pnb + 1, w.scantmp, nullptr, stream));
    if (m) {
        hipLaunchKernelGGL(k_rows_values, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, stream, (uint32_t)m,
                           (uint32_t)L->p, (uint32_t)pnb, L->elem_bytes, (int)L->elem_signed, rows,
                           (const uint64_t *)row_ptr, polmap, prow, (const uint64_t *)w.poff, pdata, val, d_status);
        FL_LAUNCH_CHECK("k_rows_values");
    }
    return FL_OK;
}
