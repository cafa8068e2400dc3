// split.hip -- FL step 1: validation, pivot selection and the splice
// [A B; C D] (paper Sec. 3.1 and Sec. 4.1 step 1), with A and C packed as
// w-multiline vectors (Sec. 4.2, the multiline Definition).
//
// Kernels, in stream order (all sizes that depend on the pivot count live on
// the device; grids are launched for upper bounds and exit early):
//   k_rows         one wave per input row: validate, leading column, and
//                  atomicMin of (row nnz << 32 | row) on the pivot key of the
//                  leading column  -> pivot row = fewest nonzeros, lowest index
//   k_colflag      pivot-column flags; exclusive scan -> npiv
//   k_colmap       col_map (input -> new column) and col_perm
//   k_rowflag      non-pivot row flags; exclusive scan
//   k_rowmap       row_perm / row position of every input row
//   k_count_bd     one wave per input row: entries in non-pivot columns
//   (scan)         -> CSR row pointers of B and D
//   k_scatter_bd   one wave per input row: scatter B/D entries (pivot rows
//                  made monic)
//   k_ml_count     one block per multiline group of A or C: size of the
//                  union of the group's column supports (LDS bitmap)
//   (scan)         -> multiline group pointers
//   k_ml_fill      one block per group: pos list and interleaved values
//   k_info         sizes for the host
#include "fl_internal.h"
#include "wide.h"

namespace {
// The field arithmetic the split needs (scaling pivot rows by the inverse of
// their lead): uint16 residues with 32-bit Barrett, or uint32 residues with
// 64-bit Barrett (the 32-bit field path).
struct FieldU16 {
    using V = uint16_t;
    fl::Mod md;
    uint32_t p() const { return md.p; }
    __device__ uint32_t mul(uint32_t a, uint32_t b) const { return fl::mulmod(a, b, md); }
    __device__ uint32_t inv(uint32_t a) const { return fl::invmod(a, md); }
};
struct FieldU32 {
    using V = uint32_t;
    flw::Mod64 md;
    uint32_t p() const { return md.p; }
    __device__ uint32_t mul(uint32_t a, uint32_t b) const { return flw::mulw(a, b, md); }
    __device__ uint32_t inv(uint32_t a) const { return flw::invw(a, md); }
};
}  // namespace

namespace {

constexpr uint32_t kNone = 0xffffffffu;
constexpr uint64_t kKeyNone = ~(uint64_t)0;
constexpr int kWinWords = 2048;              // LDS bitmap window: 65536 columns
constexpr uint32_t kWinBits = kWinWords * 32;

struct SplitDev {
    // validation
    uint64_t *errkey;    // [1] min over (row << 33 | offset << 2 | sub)
    // columns
    uint64_t *pivkey;    // [n]
    uint64_t *colscan;   // [n]  flag, then exclusive scan
    uint32_t *colmap;    // [n]
    uint32_t *cbits;     // [n / 32 + 1] pivot-column flags, 32 columns per word
    uint32_t *cbase;     // [n / 32 + 1] pivot columns before each word (colscan at its first column)
    // rows
    uint32_t *lead;      // [m]  leading column or kNone
    uint64_t *rowscan;   // [m]  non-pivot flag, then exclusive scan
    uint32_t *rowpos;    // [m]  new row position of each input row
    uint64_t *cnt;       // [m]  B/D counts by new row position, then scan
    uint32_t *rspan;     // [2m] by new row position: least and greatest new column of
                         //      the row's multiline entries (kNone, 0: none)
    uint64_t *glen;      // [G+1] multiline union sizes, then scan
    uint64_t *tot;       // [8]  0: npiv, 1: #nonpiv rows, 2: nnz(B)+nnz(D), 3: total ml len,
                         //      4: nnz(A) strictly upper, 5: nnz(C)
    uint64_t *scantmp;
};

__device__ __forceinline__ bool failed(const uint64_t *errkey) { return *errkey != kKeyNone; }

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
    for (int d = 32; d >= 1; d >>= 1) {
        uint32_t lo = __shfl_xor((uint32_t)v, d, 64), hi = __shfl_xor((uint32_t)(v >> 32), d, 64);
        uint64_t o = ((uint64_t)hi << 32) | lo;
        v = o < v ? o : v;
    }
    return v;
}

template <class V>
__global__ __launch_bounds__(256) void k_rows(uint32_t m, uint32_t n, uint64_t nnz,
                                              const uint64_t *__restrict__ rp,
                                              const uint32_t *__restrict__ ci,
                                              const V *__restrict__ v, uint32_t p,
                                              SplitDev d) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= m) return;
    uint64_t s = rp[i], e = rp[i + 1];
    uint64_t key = kKeyNone;
    bool rowbad = (i == 0 && s != 0) || e < s || e > nnz || (i == m - 1 && e != nnz);
    if (rowbad) {
        if (lane == 0) atomicMin((unsigned long long *)d.errkey, (unsigned long long)((uint64_t)i << 33));
        if (lane == 0) d.lead[i] = kNone;
        return;
    }
    for (uint64_t k = s + lane; k < e; k += 64) {
        uint32_t c = ci[k];
        uint32_t x = v[k];
        uint64_t off = (k - s) << 2;
        uint64_t base = ((uint64_t)i << 33) | off;
        uint64_t kk = kKeyNone;
        if (c >= n) kk = base | 1;
        else if (k > s && ci[k - 1] >= c) kk = base | 2;
        else if (x == 0 || x >= p) kk = base | 3;
        key = kk < key ? kk : key;
    }
    key = wave_min_u64(key);
    if (lane == 0) {
        if (key != kKeyNone) atomicMin((unsigned long long *)d.errkey, (unsigned long long)key);
        uint32_t ld = kNone;
        if (e > s) {
            ld = ci[s];
            if (ld < n)
                atomicMin((unsigned long long *)&d.pivkey[ld],
                          (unsigned long long)(((e - s) << 32) | i));
            else
                ld = kNone;
        }
        d.lead[i] = ld;
    }
}

__global__ void k_colflag(uint32_t n, SplitDev d) {
    uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) d.colscan[c] = d.pivkey[c] != kKeyNone ? 1 : 0;
}

__global__ void k_colmap(uint32_t n, SplitDev d, uint32_t *col_perm) {
    uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (failed(d.errkey)) return;
    {  // the compact map (colmap_of): one word of flags and its base per 32 columns
        const uint64_t m = __ballot(c < n && d.pivkey[c] != kKeyNone);
        if ((threadIdx.x & 31) == 0 && c < n) {
            d.cbits[c >> 5] = (uint32_t)(m >> (threadIdx.x & 32));
            d.cbase[c >> 5] = (uint32_t)d.colscan[c];
        }
    }
    if (c >= n) return;
    uint32_t npiv = (uint32_t)d.tot[0];
    uint32_t before = (uint32_t)d.colscan[c];
    uint32_t nc = d.pivkey[c] != kKeyNone ? before : npiv + (c - before);
    d.colmap[c] = nc;
    col_perm[nc] = c;
}

// New column of input column c, from the compact map written by k_colmap
// (equal to colmap[c]): pivot columns take their rank among the pivot
// columns, the others follow in order after npiv.  The entries of a row
// are in increasing column order, so 64 consecutive entries read a few
// words of the map (a few cache lines) where colmap would take one line per
// entry.
__device__ __forceinline__ uint32_t colmap_of(const SplitDev &d, uint32_t c, uint32_t npiv) {
    const uint32_t w = c >> 5, b = c & 31u, bits = d.cbits[w];
    const uint32_t lo = d.cbase[w] + (uint32_t)__popc(bits & ((1u << b) - 1u));
    return (bits >> b) & 1u ? lo : npiv + c - lo;
}

__device__ __forceinline__ bool is_pivot_row(uint32_t i, const SplitDev &d) {
    uint32_t ld = d.lead[i];
    return ld != kNone && (uint32_t)(d.pivkey[ld] & 0xffffffffu) == i;
}

__global__ void k_rowflag(uint32_t m, SplitDev d) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    d.rowscan[i] = (!failed(d.errkey) && !is_pivot_row(i, d)) ? 1 : 0;
}

__global__ void k_rowmap(uint32_t m, SplitDev d, uint32_t *row_perm) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m || failed(d.errkey)) return;
    uint32_t npiv = (uint32_t)d.tot[0];
    uint32_t pos = is_pivot_row(i, d) ? d.colmap[d.lead[i]] : npiv + (uint32_t)d.rowscan[i];
    d.rowpos[i] = pos;
    row_perm[pos] = i;
}

// Entry (k) of input row `orig` at new row position `pos` belongs to the
// multiline iff it lies in a pivot column and is not A's unit diagonal.
__device__ __forceinline__ bool ml_entry(uint32_t nc, uint32_t npiv, bool is_a, uint32_t pos) {
    return nc < npiv && !(is_a && nc == pos);
}

// Number of entries of input row i in non-pivot columns, stored at the row's
// new position (pivot rows: B counts at [0, npiv); others: D counts after);
// also the span of its multiline entries (pivot columns, A's unit diagonal
// excluded), which the multiline packing reads instead of the row.
__global__ __launch_bounds__(256) void k_count_bd(uint32_t m, const uint64_t *__restrict__ rp,
                                                  const uint32_t *__restrict__ ci, SplitDev d) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= m || failed(d.errkey)) return;
    uint32_t npiv = (uint32_t)d.tot[0];
    const uint32_t pos = d.rowpos[i];
    const bool is_a = pos < npiv;
    uint64_t s = rp[i], e = rp[i + 1];
    uint32_t cnt = 0, mn = kNone, mx = 0;
    // four entries per lane in flight: the column loads, then the map lookups
    for (uint64_t k0 = s + lane; k0 < e; k0 += 256) {
        uint32_t c[4];
#pragma unroll
        for (int u = 0; u < 4; u++) c[u] = k0 + 64 * u < e ? ci[k0 + 64 * u] : 0;
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const uint32_t nc = colmap_of(d, c[u], npiv);
            const bool in = k0 + 64 * u < e;
            cnt += in && nc >= npiv ? 1 : 0;
            if (in && ml_entry(nc, npiv, is_a, pos)) {
                mn = nc < mn ? nc : mn;
                mx = nc > mx ? nc : mx;
            }
        }
    }
    for (int dd = 32; dd >= 1; dd >>= 1) {
        cnt += __shfl_xor(cnt, dd, 64);
        const uint32_t omn = __shfl_xor(mn, dd, 64), omx = __shfl_xor(mx, dd, 64);
        mn = omn < mn ? omn : mn;
        mx = omx > mx ? omx : mx;
    }
    if (lane == 0) {
        d.rspan[2 * (uint64_t)pos] = mn;
        d.rspan[2 * (uint64_t)pos + 1] = mx;
        d.cnt[pos] = cnt;
        uint64_t in_piv = (e - s) - cnt;  // entries in pivot columns
        if (pos < npiv) atomicAdd((unsigned long long *)&d.tot[4], (unsigned long long)(in_piv - 1));
        else if (in_piv) atomicAdd((unsigned long long *)&d.tot[5], (unsigned long long)in_piv);
    }
}

__global__ void k_bd_ptr(uint32_t m, SplitDev d, uint64_t *b_ptr, uint64_t *d_ptr) {
    uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > m || failed(d.errkey)) return;
    uint32_t npiv = (uint32_t)d.tot[0];
    uint64_t total = d.tot[2];
    uint64_t v = k < m ? d.cnt[k] : total;
    uint64_t bend = npiv < m ? d.cnt[npiv] : total;
    if (k <= npiv) b_ptr[k] = v;
    if (k >= npiv) d_ptr[k - npiv] = v - bend;
}

__device__ __forceinline__ uint32_t lane_prefix_count(bool pred, uint32_t lane) {
    uint64_t mask = __ballot(pred);
    uint64_t below = lane == 0 ? 0 : (mask & (~(uint64_t)0 >> (64 - lane)));
    return __popcll(below);
}

template <class F>
__global__ __launch_bounds__(256) void k_scatter_bd(uint32_t m, F f,
                                                    const uint64_t *__restrict__ rp,
                                                    const uint32_t *__restrict__ ci,
                                                    const typename F::V *__restrict__ v, SplitDev d,
                                                    uint32_t *b_col, typename F::V *b_val,
                                                    uint32_t *d_col, typename F::V *d_val) {
    using V = typename F::V;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= m || failed(d.errkey)) return;
    uint32_t npiv = (uint32_t)d.tot[0];
    uint32_t pos = d.rowpos[i];
    bool top = pos < npiv;
    uint64_t s = rp[i], e = rp[i + 1];
    uint32_t scale = 1;
    if (top) scale = f.inv(v[s]);
    uint64_t bstart = top ? 0 : (npiv < m ? d.cnt[npiv] : d.tot[2]);
    uint64_t out = d.cnt[pos] - bstart;
    uint32_t *oc = top ? b_col : d_col;
    V *ov = top ? b_val : d_val;
    // four chunks of 64 entries at a time: their loads and map lookups are
    // issued before the chunks are compacted in order
    for (uint64_t k0 = s; k0 < e; k0 += 256) {
        uint32_t c[4], x[4], nc[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const uint64_t k = k0 + 64 * u + lane;
            c[u] = k < e ? ci[k] : 0;
            x[u] = k < e ? v[k] : 0;
        }
#pragma unroll
        for (int u = 0; u < 4; u++) nc[u] = colmap_of(d, c[u], npiv);
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const bool take = k0 + 64 * u + lane < e && nc[u] >= npiv;
            const uint32_t before = lane_prefix_count(take, lane);
            if (take) {
                oc[out + before] = nc[u] - npiv;
                ov[out + before] = (V)(top ? f.mul(x[u], scale) : x[u]);
            }
            out += __popcll(__ballot(take));
        }
    }
}

// ---- multiline packing of A (strictly upper, pivot rows made monic) and C ----

struct GroupInfo {
    bool is_a;
    uint32_t g;        // group index within A or C
    uint32_t r0, r1;   // new row positions [r0, r1)
};

__device__ __forceinline__ bool group_of(uint32_t gid, uint32_t w, uint32_t npiv, uint32_t m,
                                         GroupInfo &gi) {
    uint32_t ga = (npiv + w - 1) / w, gc = (m - npiv + w - 1) / w;
    if (gid < ga) {
        gi.is_a = true; gi.g = gid; gi.r0 = gid * w;
        gi.r1 = gi.r0 + w < npiv ? gi.r0 + w : npiv;
        return true;
    }
    if (gid < ga + gc) {
        gi.is_a = false; gi.g = gid - ga; gi.r0 = npiv + gi.g * w;
        gi.r1 = gi.r0 + w < m ? gi.r0 + w : m;
        return true;
    }
    return false;
}

// Block-wide min / max / sum of uint32 through LDS.
__device__ inline uint32_t block_reduce(uint32_t v, int op, uint32_t *red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int dd = 32; dd >= 1; dd >>= 1) {
        uint32_t o = __shfl_xor(v, dd, 64);
        v = op == 0 ? (o < v ? o : v) : op == 1 ? (o > v ? o : v) : v + o;
    }
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    uint32_t r = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); w++)
        r = op == 0 ? (red[w] < r ? red[w] : r) : op == 1 ? (red[w] > r ? red[w] : r) : r + red[w];
    __syncthreads();
    return r;
}


// The span of the group's multiline columns, from the rows' spans (the same
// in every thread).
__device__ __forceinline__ void group_span(const GroupInfo &gi, const SplitDev &d, uint32_t &lo, uint32_t &hi) {
    lo = kNone;
    hi = 0;
    for (uint32_t r = gi.r0; r < gi.r1; r++) {
        const uint32_t a = d.rspan[2 * (uint64_t)r], b = d.rspan[2 * (uint64_t)r + 1];
        lo = a < lo ? a : lo;
        hi = b > hi ? b : hi;
    }
}

// Words of the window at w0 that the span [w0, hi] touches.
__device__ __forceinline__ uint32_t window_words(uint32_t w0, uint32_t hi) {
    return ((hi - w0 < kWinBits ? hi - w0 : kWinBits - 1) >> 5) + 1;
}

__global__ __launch_bounds__(256) void k_ml_count(uint32_t m, uint32_t w,
                                                  const uint64_t *__restrict__ rp,
                                                  const uint32_t *__restrict__ ci,
                                                  const uint32_t *__restrict__ row_perm,
                                                  SplitDev d) {
    __shared__ uint32_t bits[kWinWords];
    __shared__ uint32_t red[8];
    if (failed(d.errkey)) return;
    uint32_t npiv = (uint32_t)d.tot[0];
    GroupInfo gi;
    if (!group_of(blockIdx.x, w, npiv, m, gi)) return;
    uint32_t lo, hi;
    group_span(gi, d, lo, hi);
    uint32_t total = 0;
    if (lo != kNone) {
        for (uint32_t w0 = lo; w0 <= hi; w0 += kWinBits) {
            const uint32_t nwords = window_words(w0, hi);
            for (uint32_t k = threadIdx.x; k < nwords; k += blockDim.x) bits[k] = 0;
            __syncthreads();
            for (uint32_t r = gi.r0; r < gi.r1; r++) {
                uint32_t orig = row_perm[r];
                uint64_t s = rp[orig], e = rp[orig + 1];
                for (uint64_t k0 = s + threadIdx.x; k0 < e; k0 += 4 * (uint64_t)blockDim.x) {
                    uint32_t c[4];
#pragma unroll
                    for (int u = 0; u < 4; u++) c[u] = k0 + u * blockDim.x < e ? ci[k0 + u * blockDim.x] : 0;
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                        const uint32_t nc = colmap_of(d, c[u], npiv);
                        if (k0 + u * blockDim.x < e && ml_entry(nc, npiv, gi.is_a, r) && nc >= w0 &&
                            nc - w0 < kWinBits)
                            atomicOr(&bits[(nc - w0) >> 5], 1u << ((nc - w0) & 31));
                    }
                }
            }
            __syncthreads();
            uint32_t c = 0;
            for (uint32_t k = threadIdx.x; k < nwords; k += blockDim.x) c += __popc(bits[k]);
            total += block_reduce(c, 2, red);
            if (hi - w0 < kWinBits) break;
        }
    }
    if (threadIdx.x == 0) d.glen[blockIdx.x] = total;
}

__global__ void k_ml_ptr(uint32_t m, uint32_t w, SplitDev d, uint64_t *a_gptr, uint64_t *c_gptr) {
    uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (failed(d.errkey)) return;
    uint32_t npiv = (uint32_t)d.tot[0];
    uint32_t ga = (npiv + w - 1) / w, gc = (m - npiv + w - 1) / w;
    uint64_t total = d.tot[3];
    if (k <= ga) a_gptr[k] = k < ga + gc ? d.glen[k] : total;
    if (k <= gc) {
        uint64_t base = ga < ga + gc ? d.glen[ga] : total;
        uint64_t v = (ga + k) < ga + gc ? d.glen[ga + k] : total;
        c_gptr[k] = v - base;
    }
}

template <class F>
__global__ __launch_bounds__(256) void k_ml_fill(uint32_t m, uint32_t w, F f,
                                                 const uint64_t *__restrict__ rp,
                                                 const uint32_t *__restrict__ ci,
                                                 const typename F::V *__restrict__ v,
                                                 const uint32_t *__restrict__ row_perm,
                                                 SplitDev d, uint32_t *a_pos, typename F::V *a_val,
                                                 uint32_t *c_pos, typename F::V *c_val) {
    using V = typename F::V;
    __shared__ uint32_t bits[kWinWords];
    __shared__ uint32_t pre[kWinWords];
    __shared__ uint32_t red[8];
    __shared__ uint32_t scale_s[8];
    if (failed(d.errkey)) return;
    uint32_t npiv = (uint32_t)d.tot[0];
    GroupInfo gi;
    if (!group_of(blockIdx.x, w, npiv, m, gi)) return;
    uint32_t ga = (npiv + w - 1) / w;
    uint64_t base = d.glen[blockIdx.x] - (gi.is_a ? 0 : (ga < gridDim.x ? d.glen[ga] : 0));
    uint32_t *pos = gi.is_a ? a_pos : c_pos;
    V *val = gi.is_a ? a_val : c_val;
    if (threadIdx.x < gi.r1 - gi.r0) {
        uint32_t orig = row_perm[gi.r0 + threadIdx.x];
        scale_s[threadIdx.x] = gi.is_a ? f.inv(v[rp[orig]]) : 1u;
    }
    uint32_t lo, hi;
    group_span(gi, d, lo, hi);
    if (lo == kNone) return;
    uint64_t out = base;
    for (uint32_t w0 = lo; w0 <= hi; w0 += kWinBits) {
        const uint32_t nwords = window_words(w0, hi);
        for (uint32_t k = threadIdx.x; k < nwords; k += blockDim.x) bits[k] = 0;
        __syncthreads();  // (also publishes scale_s)
        for (uint32_t r = gi.r0; r < gi.r1; r++) {
            uint32_t orig = row_perm[r];
            uint64_t s = rp[orig], e = rp[orig + 1];
            for (uint64_t k0 = s + threadIdx.x; k0 < e; k0 += 4 * (uint64_t)blockDim.x) {
                uint32_t c[4];
#pragma unroll
                for (int u = 0; u < 4; u++) c[u] = k0 + u * blockDim.x < e ? ci[k0 + u * blockDim.x] : 0;
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const uint32_t nc = colmap_of(d, c[u], npiv);
                    if (k0 + u * blockDim.x < e && ml_entry(nc, npiv, gi.is_a, r) && nc >= w0 &&
                        nc - w0 < kWinBits)
                        atomicOr(&bits[(nc - w0) >> 5], 1u << ((nc - w0) & 31));
                }
            }
        }
        __syncthreads();
        // exclusive prefix of popcounts over the window words (serial per
        // thread chunk + block scan of chunk sums)
        constexpr int kPer = kWinWords / 256;
        uint32_t csum = 0;
        const int w_lo = threadIdx.x * kPer;
        for (int k = 0; k < kPer; k++) {
            pre[w_lo + k] = csum;
            csum += (uint32_t)(w_lo + k) < nwords ? __popc(bits[w_lo + k]) : 0;
        }
        // block exclusive scan of csum
        uint32_t incl = csum;
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        for (int dd = 1; dd < 64; dd <<= 1) {
            uint32_t o = __shfl_up(incl, dd, 64);
            if (lane >= dd) incl += o;
        }
        if (lane == 63) red[wave] = incl;
        __syncthreads();
        uint32_t wbefore = 0, wtot = 0;
        for (int ww = 0; ww < 4; ww++) {
            if (ww < wave) wbefore += red[ww];
            wtot += red[ww];
        }
        uint32_t excl = wbefore + incl - csum;
        for (int k = 0; k < kPer; k++) pre[w_lo + k] += excl;
        __syncthreads();
        // positions and zeroed value slots
        for (uint32_t k = threadIdx.x; k < nwords; k += blockDim.x) {
            uint32_t b = bits[k];
            uint32_t idx = pre[k];
            while (b) {
                int t = __ffs(b) - 1;
                b &= b - 1;
                pos[out + idx] = w0 + (uint32_t)k * 32 + t;
                for (uint32_t q = 0; q < w; q++) val[(out + idx) * w + q] = 0;
                idx++;
            }
        }
        __syncthreads();
        // values
        for (uint32_t r = gi.r0; r < gi.r1; r++) {
            uint32_t orig = row_perm[r];
            uint32_t sc = scale_s[r - gi.r0];
            uint64_t s = rp[orig], e = rp[orig + 1];
            for (uint64_t k0 = s + threadIdx.x; k0 < e; k0 += 4 * (uint64_t)blockDim.x) {
                uint32_t c[4], xv[4];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const uint64_t k = k0 + u * blockDim.x;
                    c[u] = k < e ? ci[k] : 0;
                    xv[u] = k < e ? v[k] : 0;
                }
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const uint32_t nc = colmap_of(d, c[u], npiv);
                    if (k0 + u * blockDim.x < e && ml_entry(nc, npiv, gi.is_a, r) && nc >= w0 &&
                        nc - w0 < kWinBits) {
                        uint32_t off = nc - w0;
                        uint32_t word = off >> 5, bit = off & 31;
                        uint32_t idx = pre[word] + __popc(bits[word] & ((1u << bit) - 1));
                        uint32_t x = gi.is_a ? f.mul(xv[u], sc) : xv[u];
                        val[(out + idx) * w + (r - gi.r0)] = (V)x;
                    }
                }
            }
        }
        out += wtot;
        __syncthreads();
        if (hi - w0 < kWinBits) break;
    }
}

__global__ void k_info(uint32_t m, uint32_t n, uint32_t w, SplitDev d, uint64_t *info) {
    // info: 0 status key, 1 npiv, 2 nnzB, 3 nnzD, 4 lenA, 5 lenC, 6 nnzA, 7 nnzC
    uint64_t key = *d.errkey;
    info[0] = key;
    if (key != kKeyNone) return;
    uint32_t npiv = (uint32_t)d.tot[0];
    uint64_t bdtot = d.tot[2];
    uint64_t bend = npiv < m ? d.cnt[npiv] : bdtot;
    info[1] = npiv;
    info[2] = bend;
    info[3] = bdtot - bend;
    uint32_t ga = (npiv + w - 1) / w, gc = (m - npiv + w - 1) / w;
    uint64_t mltot = d.tot[3];
    uint64_t aend = ga < ga + gc ? d.glen[ga] : mltot;
    info[4] = aend;
    info[5] = mltot - aend;
    info[6] = d.tot[4];
    info[7] = d.tot[5];
}

size_t split_ws_layout(uint32_t m, uint32_t n, uint32_t w, void *ws, SplitDev *d,
                       uint64_t **info) {
    WsCarve c(ws);
    size_t groups = (size_t)(m + w - 1) / w + 1;
    size_t big = (size_t)m > n ? m : n;
    if (groups + 1 > big) big = groups + 1;
    SplitDev t;
    t.errkey = c.take<uint64_t>(1);
    t.pivkey = c.take<uint64_t>(n ? n : 1);
    t.colscan = c.take<uint64_t>(n ? n : 1);
    t.colmap = c.take<uint32_t>(n ? n : 1);
    t.cbits = c.take<uint32_t>((size_t)n / 32 + 1);
    t.cbase = c.take<uint32_t>((size_t)n / 32 + 1);
    t.lead = c.take<uint32_t>(m ? m : 1);
    t.rowscan = c.take<uint64_t>(m ? m : 1);
    t.rowpos = c.take<uint32_t>(m ? m : 1);
    t.cnt = c.take<uint64_t>(m ? m : 1);
    t.rspan = c.take<uint32_t>(2 * (size_t)(m ? m : 1));
    t.glen = c.take<uint64_t>(groups);
    t.tot = c.take<uint64_t>(8);
    t.scantmp = c.take<uint64_t>(fl_scan_tmp_elems(big));
    uint64_t *inf = c.take<uint64_t>(8);
    if (d) *d = t;
    if (info) *info = inf;
    return c.off;
}

inline unsigned blocks(size_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

__global__ void k_iota(uint32_t n, uint32_t *out) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = i;
}

}  // namespace

extern "C" size_t fl_split_workspace(uint32_t m, uint32_t n, uint64_t nnz, uint32_t ml_width) {
    (void)nnz;
    if (ml_width == 0) ml_width = 1;
    return split_ws_layout(m, n, ml_width, nullptr, nullptr, nullptr);
}

// Output pointers of the split for value type V (fl_split_out for uint16,
// fl_split_out32 for uint32).
template <class V> struct SplitOutT {
    uint32_t *row_perm, *col_perm;
    uint64_t *a_gptr;
    uint32_t *a_pos;
    V *a_val;
    uint64_t *b_ptr;
    uint32_t *b_col;
    V *b_val;
    uint64_t *c_gptr;
    uint32_t *c_pos;
    V *c_val;
    uint64_t *d_ptr;
    uint32_t *d_col;
    V *d_val;
};
template <class O, class V> SplitOutT<V> out_view(const O *o) {
    return SplitOutT<V>{o->row_perm, o->col_perm, o->a_gptr, o->a_pos, o->a_val, o->b_ptr, o->b_col, o->b_val,
                        o->c_gptr, o->c_pos, o->c_val, o->d_ptr, o->d_col, o->d_val};
}

// Everything of the split but the final sync: validation, permutations, A, B,
// C, D.  The eight size words (see k_info) go to dinfo_out when it is
// non-NULL, else to the workspace.  With m == 0 nothing but col_perm is
// written and the size words are left alone.
template <class F>
fl_status split_enqueue(uint32_t m, uint32_t n, uint64_t nnz, const uint64_t *rp, const uint32_t *ci,
                        const typename F::V *v, F f, uint32_t ml_width, const SplitOutT<typename F::V> &o,
                        void *ws, size_t ws_bytes, uint64_t *dinfo_out, hipStream_t stream) {
    const uint32_t p = f.p();
    FL_ARG(ml_width == 1 || ml_width == 2 || ml_width == 4 || ml_width == 8,
           "fl_split: ml_width must be 1, 2, 4 or 8");
    FL_ARG(m < (1u << 31) && n < (1u << 31), "fl_split: dimensions must be < 2^31");
    const uint32_t w = ml_width;
    FL_ARG(m == 0 || (rp && (nnz == 0 || (ci && v))), "fl_split: NULL CSR array");
    FL_ARG(m == 0 || (o.row_perm && o.a_gptr && o.b_ptr && o.c_gptr && o.d_ptr), "fl_split: NULL output array");
    FL_ARG(n == 0 || o.col_perm, "fl_split: NULL col_perm");
    FL_ARG(nnz == 0 || (o.a_pos && o.a_val && o.b_col && o.b_val && o.c_pos && o.c_val && o.d_col && o.d_val),
           "fl_split: NULL output array");
    SplitDev d;
    uint64_t *dinfo;
    size_t need = split_ws_layout(m, n, w, ws, &d, &dinfo);
    if (!ws || ws_bytes < need) {
        fl_set_error("fl_split: workspace too small");
        return FL_ERR_WORKSPACE;
    }
    if (dinfo_out) dinfo = dinfo_out;
    if (m == 0) {  // no rows: no pivots, every column is a non-pivot column
        if (n) {
            hipLaunchKernelGGL(k_iota, dim3(blocks(n, 256)), dim3(256), 0, stream, n, o.col_perm);
            FL_LAUNCH_CHECK("k_iota");
        }
        return FL_OK;
    }
    const size_t groups = (size_t)(m + w - 1) / w + 1;

    FL_HIP(fl_fill_u64(d.errkey, ~(uint64_t)0, 1, stream));
    FL_HIP(fl_fill_u64(d.pivkey, ~(uint64_t)0, n, stream));
    FL_HIP(fl_fill_u64(d.tot, 0, 8, stream));
    hipLaunchKernelGGL(k_rows<typename F::V>, dim3(blocks(m, 4)), dim3(256), 0, stream, m, n, nnz, rp, ci, v,
                       p, d);
    FL_LAUNCH_CHECK("k_rows");
    if (n) {
        hipLaunchKernelGGL(k_colflag, dim3(blocks(n, 256)), dim3(256), 0, stream, n, d);
        FL_LAUNCH_CHECK("k_colflag");
        FL_HIP(fl_exclusive_scan_u64(d.colscan, d.colscan, n, d.scantmp, d.tot + 0, stream));
        hipLaunchKernelGGL(k_colmap, dim3(blocks(n, 256)), dim3(256), 0, stream, n, d, o.col_perm);
        FL_LAUNCH_CHECK("k_colmap");
    }
    hipLaunchKernelGGL(k_rowflag, dim3(blocks(m, 256)), dim3(256), 0, stream, m, d);
    FL_LAUNCH_CHECK("k_rowflag");
    FL_HIP(fl_exclusive_scan_u64(d.rowscan, d.rowscan, m, d.scantmp, d.tot + 1, stream));
    hipLaunchKernelGGL(k_rowmap, dim3(blocks(m, 256)), dim3(256), 0, stream, m, d, o.row_perm);
    FL_LAUNCH_CHECK("k_rowmap");
    hipLaunchKernelGGL(k_count_bd, dim3(blocks(m, 4)), dim3(256), 0, stream, m, rp, ci, d);
    FL_LAUNCH_CHECK("k_count_bd");
    FL_HIP(fl_exclusive_scan_u64(d.cnt, d.cnt, m, d.scantmp, d.tot + 2, stream));
    hipLaunchKernelGGL(k_bd_ptr, dim3(blocks(m + 1, 256)), dim3(256), 0, stream, m, d, o.b_ptr, o.d_ptr);
    FL_LAUNCH_CHECK("k_bd_ptr");
    hipLaunchKernelGGL(k_scatter_bd<F>, dim3(blocks(m, 4)), dim3(256), 0, stream, m, f, rp, ci, v, d, o.b_col,
                       o.b_val, o.d_col, o.d_val);
    FL_LAUNCH_CHECK("k_scatter_bd");
    // multiline groups: A groups then C groups, at most ceil(m/w) + 1 of them
    FL_HIP(fl_fill_u64(d.glen, 0, groups, stream));
    hipLaunchKernelGGL(k_ml_count, dim3((unsigned)groups), dim3(256), 0, stream, m, w, rp, ci, o.row_perm, d);
    FL_LAUNCH_CHECK("k_ml_count");
    FL_HIP(fl_exclusive_scan_u64(d.glen, d.glen, groups, d.scantmp, d.tot + 3, stream));
    hipLaunchKernelGGL(k_ml_ptr, dim3(blocks(groups + 1, 256)), dim3(256), 0, stream, m, w, d, o.a_gptr,
                       o.c_gptr);
    FL_LAUNCH_CHECK("k_ml_ptr");
    hipLaunchKernelGGL(k_ml_fill<F>, dim3((unsigned)groups), dim3(256), 0, stream, m, w, f, rp, ci, v, o.row_perm,
                       d, o.a_pos, o.a_val, o.c_pos, o.c_val);
    FL_LAUNCH_CHECK("k_ml_fill");
    hipLaunchKernelGGL(k_info, dim3(1), dim3(1), 0, stream, m, n, w, d, dinfo);
    FL_LAUNCH_CHECK("k_info");
    return FL_OK;
}

fl_status fl_split_enqueue(const fl_csr *M, uint32_t p, uint32_t ml_width, const fl_split_out *o,
                           void *ws, size_t ws_bytes, uint64_t *dinfo_out, hipStream_t stream) {
    FL_ARG(M && o, "fl_split: NULL argument");
    FL_ARG(p >= 2 && p <= 65521, "fl_split: p must be in [2, 65521]");
    return split_enqueue(M->rows, M->cols, M->nnz, M->row_ptr, M->col, M->val, FieldU16{fl::make_mod(p)},
                         ml_width, out_view<fl_split_out, uint16_t>(o), ws, ws_bytes, dinfo_out, stream);
}

// Host side of fl_split after the sync: the size words -> h_info.
fl_status fl_split_finish(const fl_csr *M, uint32_t p, uint32_t ml_width, const uint64_t hinf[8],
                          fl_split_info *h_info) {
    fl_split_info info = {};
    info.p = p; info.m = M->rows; info.n = M->cols; info.ml_width = ml_width; info.nnz = M->nnz;
    if (M->rows == 0) {
        info.nB = M->cols;
        *h_info = info;
        return FL_OK;
    }
    if (hinf[0] != ~(uint64_t)0) {
        static const fl_status codes[4] = {FL_ERR_DATA_ROWPTR, FL_ERR_DATA_COL_RANGE,
                                           FL_ERR_DATA_COL_ORDER, FL_ERR_DATA_VALUE};
        fl_status st = codes[hinf[0] & 3];
        info.status = st;
        *h_info = info;
        fl_set_error(fl_status_string(st));
        return st;
    }
    info.npiv = (uint32_t)hinf[1];
    info.nB = info.n - info.npiv;
    info.mD = info.m - info.npiv;
    info.nnzB = hinf[2];
    info.nnzD = hinf[3];
    info.lenA = hinf[4];
    info.lenC = hinf[5];
    info.nnzA = hinf[6];
    info.nnzC = hinf[7];
    *h_info = info;
    return FL_OK;
}

extern "C" fl_status fl_split(const fl_csr *M, uint32_t p, uint32_t ml_width,
                              const fl_split_out *o, fl_split_info *h_info, void *ws,
                              size_t ws_bytes, hipStream_t stream) {
    FL_ARG(M && o && h_info, "fl_split: NULL argument");
    fl_status st = fl_split_enqueue(M, p, ml_width, o, ws, ws_bytes, nullptr, stream);
    if (st != FL_OK) return st;
    uint64_t hinf[8] = {~(uint64_t)0, 0, 0, 0, 0, 0, 0, 0};
    if (M->rows) {
        SplitDev d;
        uint64_t *dinfo;
        split_ws_layout(M->rows, M->cols, ml_width, ws, &d, &dinfo);
        FL_HIP(hipMemcpyAsync(hinf, dinfo, sizeof(hinf), hipMemcpyDeviceToHost, stream));
        FL_HIP(hipStreamSynchronize(stream));
    }
    return fl_split_finish(M, p, ml_width, hinf, h_info);
}

// The 32-bit field path's split: the same steps over uint32 residues.
extern "C" fl_status fl_split32(const fl_csr32 *M, uint32_t p, uint32_t ml_width, const fl_split_out32 *o,
                                fl_split_info *h_info, void *ws, size_t ws_bytes, hipStream_t stream) {
    FL_ARG(M && o && h_info, "fl_split32: NULL argument");
    FL_ARG(p >= 2, "fl_split32: p must be >= 2");
    fl_status st = split_enqueue(M->rows, M->cols, M->nnz, M->row_ptr, M->col, M->val, FieldU32{flw::make_mod64(p)},
                                 ml_width, out_view<fl_split_out32, uint32_t>(o), ws, ws_bytes, nullptr, stream);
    if (st != FL_OK) return st;
    uint64_t hinf[8] = {~(uint64_t)0, 0, 0, 0, 0, 0, 0, 0};
    if (M->rows) {
        SplitDev d;
        uint64_t *dinfo;
        split_ws_layout(M->rows, M->cols, ml_width, ws, &d, &dinfo);
        FL_HIP(hipMemcpyAsync(hinf, dinfo, sizeof(hinf), hipMemcpyDeviceToHost, stream));
        FL_HIP(hipStreamSynchronize(stream));
    }
    fl_csr shape = {M->rows, M->cols, M->nnz, M->row_ptr, M->col, nullptr};
    return fl_split_finish(&shape, p, ml_width, hinf, h_info);
}
