// common.hip -- error plumbing, device scan and fill kernels, self-checks.
#include "fl_internal.h"
#include "mfma_tile.h"

#include <cstdio>
#include <cstring>

#include <map>
#include <mutex>
#include <string>
#include <vector>

static thread_local std::string g_last_error;

void fl_set_error(const char *msg) { g_last_error = msg ? msg : ""; }

fl_status fl_hip_fail(hipError_t e, const char *where) {
    g_last_error = std::string(where) + ": " + hipGetErrorString(e);
    return FL_ERR_HIP;
}

extern "C" const char *fl_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *fl_version(void) { return "fl-gfx950 0.1.0"; }

extern "C" const char *fl_status_string(fl_status s) {
    switch (s) {
    case FL_OK: return "ok";
    case FL_ERR_ARG: return "invalid argument";
    case FL_ERR_WORKSPACE: return "workspace too small";
    case FL_ERR_DATA_ROWPTR: return "row_ptr not monotone from 0 to nnz";
    case FL_ERR_DATA_COL_RANGE: return "column index out of range";
    case FL_ERR_DATA_COL_ORDER: return "columns of a row not strictly increasing";
    case FL_ERR_DATA_VALUE: return "value zero or not reduced mod p";
    case FL_ERR_HIP: return "HIP runtime error";
    }
    return "unknown status";
}

// ---- exclusive scan (uint64) ----------------------------------------------------
namespace {
constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;
constexpr size_t kScanTile = (size_t)kScanThreads * kScanPer;

__device__ inline uint64_t shfl_up_u64(uint64_t v, int d) {
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    lo = __shfl_up(lo, d, 64);
    hi = __shfl_up(hi, d, 64);
    return ((uint64_t)hi << 32) | lo;
}

// Inclusive scan of one value per thread over the block; returns the
// inclusive prefix, *block_total receives the sum of the block.
__device__ inline uint64_t block_incl_scan(uint64_t v, uint64_t *block_total) {
    __shared__ uint64_t wave_tot[kScanThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t o = shfl_up_u64(v, d);
        if (lane >= d) v += o;
    }
    if (lane == 63) wave_tot[wave] = v;
    __syncthreads();
    uint64_t before = 0, tot = 0;
    for (int w = 0; w < kScanThreads / 64; w++) {
        if (w < wave) before += wave_tot[w];
        tot += wave_tot[w];
    }
    __syncthreads();
    *block_total = tot;
    return v + before;
}

__global__ __launch_bounds__(kScanThreads) void k_tile_sum(const uint64_t *in, size_t n,
                                                           uint64_t *sums) {
    size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanPer;
    uint64_t s = 0;
    for (int k = 0; k < kScanPer; k++)
        if (base + k < n) s += in[base + k];
    uint64_t tot;
    block_incl_scan(s, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_tile_scan(const uint64_t *in, uint64_t *out,
                                                            size_t n, const uint64_t *offsets,
                                                            uint64_t *total) {
    size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanPer;
    uint64_t v[kScanPer];
    uint64_t s = 0;
    for (int k = 0; k < kScanPer; k++) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    uint64_t tot;
    uint64_t incl = block_incl_scan(s, &tot);
    uint64_t off = offsets ? offsets[blockIdx.x] : 0;
    uint64_t run = off + incl - s;
    for (int k = 0; k < kScanPer; k++) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) *total = off + tot;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u64(uint64_t *p, uint64_t v, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// One block row-chunk per blockIdx.y, columns in 4-element (8-byte) steps.
__global__ void k_zero_rows_u16(uint16_t *p, uint64_t ld, uint32_t rows, uint32_t cols) {
    for (uint32_t r = blockIdx.y; r < rows; r += gridDim.y) {
        uint16_t *row = p + (uint64_t)r * ld;
        for (uint32_t c = (blockIdx.x * blockDim.x + threadIdx.x) * 4; c < cols;
             c += gridDim.x * blockDim.x * 4) {
            if (c + 4 <= cols) *(uint64_t *)(row + c) = 0;
            else
                for (uint32_t k = c; k < cols; k++) row[k] = 0;
        }
    }
}

inline unsigned grid_for(size_t n, unsigned threads, unsigned cap = 65536) {
    size_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    return (unsigned)(g > cap ? cap : g);
}
}  // namespace

size_t fl_scan_tmp_elems(size_t n) {
    size_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb <= 1) return 1;
    return nb + fl_scan_tmp_elems(nb);
}

hipError_t fl_exclusive_scan_u64(const uint64_t *in, uint64_t *out, size_t n, uint64_t *tmp,
                                 uint64_t *total_out, hipStream_t s) {
    if (n == 0) {
        if (total_out) return fl_fill_u64(total_out, 0, 1, s);
        return hipSuccess;
    }
    size_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 1) {
        hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(kScanThreads), 0, s, in, out, n,
                           (const uint64_t *)nullptr, total_out);
        return hipGetLastError();
    }
    uint64_t *sums = tmp, *rest = tmp + nb;
    hipLaunchKernelGGL(k_tile_sum, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = fl_exclusive_scan_u64(sums, sums, nb, rest, nullptr, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tile_scan, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, n,
                       (const uint64_t *)sums, total_out);
    return hipGetLastError();
}

uint32_t fl_cu_count() {
    static int cus = [] {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
        return n;
    }();
    return (uint32_t)cus;
}

uint32_t fl_queue_grid(uint32_t total, uint32_t per_cu) {
    const uint64_t cap = (uint64_t)per_cu * (uint64_t)fl_cu_count();
    return (uint32_t)(cap < total ? cap : total);
}

hipError_t fl_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t fl_fill_u64(uint64_t *p, uint64_t v, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t fl_zero_rows_u16(uint16_t *p, uint64_t ld, uint32_t rows, uint32_t cols,
                            hipStream_t s) {
    if (rows == 0 || cols == 0) return hipSuccess;
    unsigned gx = (unsigned)((cols / 4 + 255) / 256);
    if (gx < 1) gx = 1;
    unsigned gy = rows < 4096 ? rows : 4096;
    hipLaunchKernelGGL(k_zero_rows_u16, dim3(gx, gy), dim3(256), 0, s, p, ld, rows, cols);
    return hipGetLastError();
}

// ---- self-check of the modular reductions ---------------------------------------
// Every 32-bit x through reduce32; with it, fold_pair(x, y) against 64-bit
// division for y = x times an odd constant (a spread of low words over the
// whole 2^41 range of 256 x + y), mulmod over the residue pairs (x mod 2^16
// mod p, x >> 16 mod p), and combine_limbs (with its p >= 256 form
// combine_limbs_2) over a grid of (S_hh, S_mid, S_ll) spanning the whole
// range its callers can produce (sums of up to kKChunk limb products, S_ll
// plus a folded residue), corners included; for p < 256 the single-limb
// combine_limbs_1 over the range of its sums instead.
namespace {
// Value i (of 2^bits) of a grid over [lo, hi]: the four values at each end,
// the four around zero, and a jittered linear spread in between.
__device__ int64_t grid_value(uint32_t i, uint32_t bits, int64_t lo, int64_t hi) {
    const uint32_t n = 1u << bits;
    if (i < 4) return lo + i;
    if (i >= n - 4) return hi - (int64_t)(n - 1 - i);
    if (i >= n / 2 - 2 && i < n / 2 + 2) return (int64_t)i - (int64_t)(n / 2);
    const uint64_t span = (uint64_t)(hi - lo);
    return lo + (int64_t)(span / n * i + (i * 2654435761u) % (span / n));
}

__global__ void k_check_modp(fl::Mod m, uint32_t bias, uint32_t c16, uint64_t *mismatch) {
    const uint64_t total = (uint64_t)1 << 32;
    const uint64_t nthreads = (uint64_t)gridDim.x * blockDim.x;
    const fl_mfma::LimbCombine lc = fl_mfma::limb_combine(m, bias, c16);
    const int64_t kMaxHH = (int64_t)fl_mfma::kKChunk * 16384;
    const int64_t kMaxMid = (int64_t)fl_mfma::kKChunk * 32512;
    const int64_t kMaxLL = kMaxHH + m.p - 1;
    uint64_t bad = 0;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += nthreads) {
        uint32_t v = (uint32_t)x;
        if (fl::reduce32(v, m) != v % m.p) bad++;
        const uint32_t y = v * 2654435761u;
        if (fl::fold_pair(v, y, m) != (uint32_t)((((uint64_t)v << 8) + y) % m.p)) bad++;
        const uint32_t a = (v & 0xffffu) % m.p, b = (v >> 16) % m.p;
        if (fl::mulmod(a, b, m) != a * b % m.p) bad++;
        const int64_t hh = grid_value(v >> 21, 11, -kMaxHH, kMaxHH);
        const int64_t mid = grid_value((v >> 10) & 2047u, 11, -kMaxMid, kMaxMid);
        const int64_t ll = grid_value(v & 1023u, 10, -kMaxHH, kMaxLL);
        const int64_t S = hh * 65536 + mid * 256 + ll;
        const int64_t want = ((S % (int64_t)m.p) + m.p) % m.p;
        if (fl_mfma::combine_limbs(lc, (int)hh, (int)mid, (int)ll) != (uint32_t)want) bad++;
        if (m.p >= 256) {  // the two-limb GEMM's combine (p >= 256 only)
            if (fl_mfma::combine_limbs_2(lc, (int)hh, (int)mid, (int)ll) != (uint32_t)want) bad++;
        } else {  // the single-limb GEMM's combine: S_ll of up to kKChunk products in [-127^2, 127^2]
            const int64_t kMaxOne = (int64_t)fl_mfma::kKChunk * 16129;
            const int64_t l1 = grid_value(v & 0x3fffffu, 22, -kMaxOne, kMaxOne + m.p - 1);
            const int64_t w1 = ((l1 % (int64_t)m.p) + m.p) % m.p;
            if (fl_mfma::combine_limbs_1(lc, (int)l1) != (uint32_t)w1) bad++;
        }
    }
    if (bad) atomicAdd((unsigned long long *)mismatch, (unsigned long long)bad);
}
}  // namespace

extern "C" fl_status fl_check_modp(const uint32_t *h_p_list, uint32_t count,
                                   uint64_t *d_mismatch, hipStream_t stream) {
    FL_ARG(h_p_list && d_mismatch, "fl_check_modp: NULL pointer");
    hipError_t e = fl_fill_u64(d_mismatch, 0, count, stream);
    if (e != hipSuccess) return fl_hip_fail(e, "fl_check_modp fill");
    for (uint32_t i = 0; i < count; i++) {
        FL_ARG(h_p_list[i] >= 2 && h_p_list[i] <= 65521, "fl_check_modp: p out of range");
        hipLaunchKernelGGL(k_check_modp, dim3(4096), dim3(256), 0, stream, fl::make_mod(h_p_list[i]),
                           fl_mfma::gemm_bias(h_p_list[i]), fl_mfma::gemm_c16(h_p_list[i]), d_mismatch + i);
        FL_LAUNCH_CHECK("k_check_modp");
    }
    return FL_OK;
}

// ---- launch profiler ---------------------------------------------------------------
// When enabled, selected kernel launches are bracketed by HIP events recorded
// on the launch stream; fl_prof_report aggregates elapsed times per site.
namespace {
struct ProfRec {
    std::string site;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t prof_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

int fl_prof_begin(const char *site, hipStream_t s) {
    if (!g_prof_on) return -1;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    ProfRec r;
    r.site = site;
    r.a = prof_event();
    r.b = prof_event();
    if (!r.a || !r.b) return -1;
    if (hipEventRecord(r.a, s) != hipSuccess) return -1;
    g_prof.push_back(r);
    return (int)g_prof.size() - 1;
}

void fl_prof_end(int tok, hipStream_t s) {
    if (tok < 0) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if ((size_t)tok < g_prof.size()) (void)hipEventRecord(g_prof[tok].b, s);
}

extern "C" void fl_prof_enable(int on) { g_prof_on = on != 0; }

bool fl_prof_set(bool on) {
    const bool old = g_prof_on;
    g_prof_on = on;
    return old;
}

extern "C" void fl_prof_reset(void) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto &r : g_prof) {
        g_event_pool.push_back(r.a);
        g_event_pool.push_back(r.b);
    }
    g_prof.clear();
}

extern "C" size_t fl_prof_report(char *buf, size_t len) {
    std::map<std::string, std::pair<uint64_t, double>> agg;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        for (auto &r : g_prof) {
            float ms = 0.f;
            if (hipEventSynchronize(r.b) != hipSuccess) continue;
            if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
            auto &e = agg[r.site];
            e.first += 1;
            e.second += ms;
        }
    }
    std::string out = "{";
    bool first = true;
    for (auto &kv : agg) {
        char tmp[256];
        snprintf(tmp, sizeof tmp, "%s\"%s\": {\"count\": %llu, \"total_ms\": %.6f}", first ? "" : ", ",
                 kv.first.c_str(), (unsigned long long)kv.second.first, kv.second.second);
        out += tmp;
        first = false;
    }
    out += "}";
    if (buf && len) {
        size_t n = out.size() < len - 1 ? out.size() : len - 1;
        memcpy(buf, out.data(), n);
        buf[n] = 0;
    }
    return out.size() + 1;
}

// ---- host -> device copies through kernel arguments ----------------------------
namespace {
struct UploadChunk {
    uint32_t n;          // 32-bit words in w
    uint32_t w[255];
};

__global__ void k_upload(uint32_t *dst, UploadChunk c) {
    for (uint32_t i = threadIdx.x; i < c.n; i += blockDim.x) dst[i] = c.w[i];
}
}  // namespace

hipError_t fl_upload(void *dst, const void *src, size_t bytes, hipStream_t s) {
    if ((bytes & 3) || ((uintptr_t)dst & 3)) return hipErrorInvalidValue;
    const uint32_t *in = (const uint32_t *)src;
    uint32_t *out = (uint32_t *)dst;
    size_t words = bytes / 4;
    for (size_t o = 0; o < words; o += 255) {
        UploadChunk c;
        c.n = (uint32_t)(words - o < 255 ? words - o : 255);
        memcpy(c.w, in + o, 4 * (size_t)c.n);
        hipLaunchKernelGGL(k_upload, dim3(1), dim3(256), 0, s, out + o, c);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

fl_status fl_aux_stream(uint32_t slot, hipStream_t *s, hipEvent_t *a, hipEvent_t *b) {
    struct Aux {
        hipStream_t s = nullptr;
        hipEvent_t a = nullptr, b = nullptr;
    };
    constexpr uint32_t kAuxSlots = 4;
    thread_local std::vector<Aux> cache;
    if (slot >= kAuxSlots) {
        fl_set_error("fl_aux_stream: bad slot");
        return FL_ERR_ARG;
    }
    int dev = 0;
    FL_HIP(hipGetDevice(&dev));
    if ((size_t)(dev + 1) * kAuxSlots > cache.size()) cache.resize((size_t)(dev + 1) * kAuxSlots);
    Aux &x = cache[(size_t)dev * kAuxSlots + slot];
    if (!x.s) {
        FL_HIP(hipEventCreateWithFlags(&x.a, hipEventDisableTiming));
        FL_HIP(hipEventCreateWithFlags(&x.b, hipEventDisableTiming));
        FL_HIP(hipStreamCreateWithFlags(&x.s, hipStreamNonBlocking));
    }
    *s = x.s;
    *a = x.a;
    *b = x.b;
    return FL_OK;
}
