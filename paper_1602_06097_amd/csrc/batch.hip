// batch.hip -- the batched form: many independent matrices of uneven sizes.
//
// An F4 computation hands over a sequence of matrices, most of them far too
// small to fill 256 compute units on their own (the F4 tables of Sec. 6.2
// range over three orders of magnitude).  The batch is reduced in two parts:
//
//   plan  every matrix is split (step 1 of Sec. 4.1) on the caller's stream
//         into its own slice of the split arena; the size words of all
//         matrices are read back with one synchronisation.  With every size
//         known, the plan lays out the run arena and picks each matrix's
//         arithmetic form (int8 MFMA above a size threshold, else VALU).
//   run   steps 2-5 of every matrix are enqueued on `streams` branches forked
//         from the caller's stream (matrices dealt largest first to the
//         branch with the least work so far), each branch reusing one
//         workspace sized for its largest matrix, and joined back.  Nothing
//         synchronises the host, so the run can be captured into a hipGraph
//         and replayed; a replay recomputes everything from the split.
//
// The autotuner times candidate configurations on the batch itself and
// remembers the best per batch shape.
#include <math.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fl_internal.h"

namespace {

constexpr uint32_t kMaxStreams = 16;
constexpr uint64_t kDefaultMfmaMin = (uint64_t)1 << 22;

inline uint64_t align256(uint64_t x) { return (x + 255) & ~(uint64_t)255; }
inline uint64_t ld64(uint32_t cols) { return cols ? ((uint64_t)cols + 63) / 64 * 64 : 64; }

// Byte layout of one matrix's fl_split outputs inside the split arena.
struct SplitSlice {
    uint64_t row_perm, col_perm, a_gptr, a_pos, a_val, b_ptr, b_col, b_val, c_gptr, c_pos, c_val,
        d_ptr, d_col, d_val, dinfo, end;
};

SplitSlice split_slice(uint64_t base, const fl_csr &M, uint32_t w) {
    SplitSlice s;
    const uint64_t m = M.rows, n = M.cols, nnz = M.nnz;
    const uint64_t G = (m + w - 1) / w + 1;
    uint64_t o = base;
    auto take = [&](uint64_t bytes) {
        const uint64_t at = o;
        o = align256(o + (bytes ? bytes : 1));
        return at;
    };
    s.row_perm = take(4 * m);
    s.col_perm = take(4 * n);
    s.a_gptr = take(8 * G);
    s.a_pos = take(4 * nnz);
    s.a_val = take(2 * w * nnz);
    s.b_ptr = take(8 * (m + 1));
    s.b_col = take(4 * nnz);
    s.b_val = take(2 * nnz);
    s.c_gptr = take(8 * G);
    s.c_pos = take(4 * nnz);
    s.c_val = take(2 * w * nnz);
    s.d_ptr = take(8 * (m + 1));
    s.d_col = take(4 * nnz);
    s.d_val = take(2 * nnz);
    s.dinfo = take(64);
    s.end = o;
    return s;
}

// Split workspace shared by all splits (they run one after another on one
// stream), placed after the slices.
size_t split_ws_max(const fl_csr *Ms, uint32_t count, uint32_t w) {
    size_t mx = 0;
    for (uint32_t i = 0; i < count; i++)
        mx = std::max(mx, fl_split_workspace(Ms[i].rows, Ms[i].cols, Ms[i].nnz, w));
    return mx;
}

size_t split_arena_bytes(const fl_csr *Ms, uint32_t count, uint32_t w) {
    uint64_t o = 0;
    for (uint32_t i = 0; i < count; i++) o = split_slice(o, Ms[i], w).end;
    return o + align256(split_ws_max(Ms, count, w));
}

// Summary table entry written at the end of each matrix's branch.
__global__ void k_batch_summary(uint64_t *row, uint32_t npiv, uint32_t maxr,
                                const uint32_t *__restrict__ d_rank,
                                const uint64_t *__restrict__ row_ptr, uint64_t status) {
    if (threadIdx.x) return;
    const uint32_t r = maxr ? *d_rank : 0;
    const uint32_t rank = npiv + r;
    row[0] = rank;
    row[1] = row_ptr[rank];
    row[2] = status;
    row[3] = 0;
}

__global__ void k_batch_skip(uint64_t *row, uint64_t status) {
    if (threadIdx.x) return;
    row[0] = 0;
    row[1] = 0;
    row[2] = status;
    row[3] = 0;
}

struct MatrixRun {
    fl_csr M;
    fl_split_out out;
    fl_split_info info;
    fl_status status;
    fl_mode mode;
    uint32_t branch;
    uint64_t ldx, ldd, maxr, nnz_cap;
    uint64_t off_X, off_Dt, off_rank, off_piv, off_rowptr, off_col, off_val;
    double cost;  // rough work estimate, for dealing matrices to branches
};

std::mutex g_tune_mu;
std::map<std::string, fl_batch_config> g_tuned;

std::string shape_key(const fl_csr *Ms, uint32_t count, uint32_t p) {
    uint64_t nnz = 0, mmax = 0;
    for (uint32_t i = 0; i < count; i++) {
        nnz += Ms[i].nnz;
        mmax = std::max<uint64_t>(mmax, Ms[i].rows);
    }
    char buf[96];
    snprintf(buf, sizeof buf, "%u/%u/%d/%d", count, p, (int)lround(log2((double)nnz + 1)),
             (int)lround(log2((double)mmax + 1)));
    return buf;
}

fl_batch_config resolve(const fl_batch_config *cfg, const fl_csr *Ms, uint32_t count, uint32_t p) {
    fl_batch_config c = {0, 0, 0};
    if (cfg) {
        c = *cfg;
    } else {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(shape_key(Ms, count, p));
        if (it != g_tuned.end()) c = it->second;
    }
    if (c.ml_width == 0) c.ml_width = 2;
    if (c.streams == 0) c.streams = 8;
    if (c.mfma_min_entries == 0) c.mfma_min_entries = kDefaultMfmaMin;
    return c;
}

}  // namespace

struct fl_batch {
    uint32_t count = 0, p = 0;
    fl_batch_config cfg = {};
    std::vector<MatrixRun> mats;
    std::vector<uint64_t> ws_off, ws_bytes;  // per branch
    uint64_t summary_off = 0, run_bytes = 0;
    hipStream_t streams[kMaxStreams] = {};
    hipStream_t capture = nullptr;  // graph capture when the caller passes the null stream
    hipEvent_t fork = nullptr, join[kMaxStreams] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

fl_status batch_init_streams(fl_batch *b) {
    FL_HIP(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
    FL_HIP(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
    for (uint32_t k = 0; k < b->cfg.streams; k++) {
        FL_HIP(hipStreamCreateWithFlags(&b->streams[k], hipStreamNonBlocking));
        FL_HIP(hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming));
    }
    return FL_OK;
}

// Lays out the run arena from the split sizes and deals matrices to branches.
void batch_layout(fl_batch *b) {
    const uint32_t S = b->cfg.streams;
    std::vector<uint64_t> ws_need(S, 0);
    std::vector<double> load(S, 0.0);
    std::vector<uint32_t> order(b->count);
    for (uint32_t i = 0; i < b->count; i++) order[i] = i;
    for (auto &mr : b->mats) {
        const fl_split_info &f = mr.info;
        mr.maxr = std::min(f.mD, f.nB);
        mr.cost = (double)f.nnzA * f.nB + (double)f.nnzC * f.nB +
                  (double)f.mD * f.nB * (double)std::min<uint64_t>(mr.maxr, 4096) +
                  (double)f.npiv * f.nB * (double)mr.maxr * 0.25 + (double)f.nnz;
        const uint64_t dense = ((uint64_t)f.npiv + f.mD) * f.nB;
        mr.mode = dense >= b->cfg.mfma_min_entries ? FL_MFMA_I8 : FL_PLAIN;
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t x, uint32_t y) { return b->mats[x].cost > b->mats[y].cost; });
    for (uint32_t i : order) {
        MatrixRun &mr = b->mats[i];
        uint32_t k = (uint32_t)(std::min_element(load.begin(), load.end()) - load.begin());
        mr.branch = k;
        load[k] += mr.cost + 2e6;  // per-matrix launch overhead, in work units
        if (mr.status != FL_OK) continue;
        const fl_split_info *f = &mr.info;
        size_t w = fl_trsm_workspace(f, mr.mode);
        w = std::max(w, fl_reduce_cd_workspace(f, mr.mode));
        w = std::max(w, fl_echelon_d_workspace(f->mD, f->nB, mr.mode));
        w = std::max(w, fl_rref_workspace(f, mr.mode));
        w = std::max(w, fl_rref_csr_workspace(f));
        ws_need[k] = std::max<uint64_t>(ws_need[k], w);
    }
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t at = o;
        o = align256(o + (bytes ? bytes : 1));
        return at;
    };
    b->summary_off = take(32ull * b->count);
    for (auto &mr : b->mats) {
        const fl_split_info &f = mr.info;
        mr.ldx = ld64(f.nB);
        mr.ldd = ld64(f.nB);
        mr.nnz_cap = ((uint64_t)f.npiv + mr.maxr) * ((uint64_t)f.nB + 1);
        if (mr.status != FL_OK) {
            mr.off_X = mr.off_Dt = mr.off_rank = mr.off_piv = mr.off_rowptr = mr.off_col = mr.off_val = 0;
            continue;
        }
        mr.off_X = take(2 * mr.ldx * std::max<uint64_t>(f.npiv, 1));
        mr.off_Dt = take(2 * mr.ldd * std::max<uint64_t>(f.mD, 1));
        mr.off_rank = take(4);
        mr.off_piv = take(4 * std::max<uint64_t>(mr.maxr, 1));
        mr.off_rowptr = take(8 * ((uint64_t)f.npiv + mr.maxr + 1));
        mr.off_col = take(4 * mr.nnz_cap);
        mr.off_val = take(2 * mr.nnz_cap);
    }
    b->ws_off.assign(S, 0);
    b->ws_bytes.assign(S, 0);
    for (uint32_t k = 0; k < S; k++) {
        b->ws_bytes[k] = std::max<uint64_t>(ws_need[k], 256);
        b->ws_off[k] = take(b->ws_bytes[k]);
    }
    b->run_bytes = o;
}

template <class T>
T *at(void *arena, uint64_t off) {
    return (T *)((char *)arena + off);
}

// Steps 2-5 of one matrix on stream s.
fl_status run_one(fl_batch *b, const MatrixRun &mr, void *arena, hipStream_t s) {
    uint64_t *sum = at<uint64_t>(arena, b->summary_off) + 4 * (size_t)(&mr - b->mats.data());
    if (mr.status != FL_OK) {
        hipLaunchKernelGGL(k_batch_skip, dim3(1), dim3(64), 0, s, sum, (uint64_t)mr.status);
        FL_LAUNCH_CHECK("k_batch_skip");
        return FL_OK;
    }
    const fl_split_info *f = &mr.info;
    uint16_t *X = at<uint16_t>(arena, mr.off_X);
    uint16_t *Dt = at<uint16_t>(arena, mr.off_Dt);
    uint32_t *rank = at<uint32_t>(arena, mr.off_rank);
    uint32_t *piv = at<uint32_t>(arena, mr.off_piv);
    uint64_t *rp = at<uint64_t>(arena, mr.off_rowptr);
    void *ws = at<char>(arena, b->ws_off[mr.branch]);
    const size_t wsb = b->ws_bytes[mr.branch];
    fl_status st;
    if ((st = fl_trsm(f, &mr.out, X, mr.ldx, mr.mode, ws, wsb, s)) != FL_OK) return st;
    if ((st = fl_reduce_cd(f, &mr.out, X, mr.ldx, Dt, mr.ldd, mr.mode, ws, wsb, s)) != FL_OK) return st;
    if ((st = fl_echelon_d(b->p, f->mD, f->nB, Dt, mr.ldd, rank, piv, mr.mode, ws, wsb, s)) != FL_OK)
        return st;
    if ((st = fl_rref(f, &mr.out, X, mr.ldx, Dt, mr.ldd, rank, piv, mr.mode, ws, wsb, s)) != FL_OK)
        return st;
    if ((st = fl_rref_csr_enqueue(f, &mr.out, X, mr.ldx, Dt, mr.ldd, rank, piv, rp,
                                  at<uint32_t>(arena, mr.off_col), at<uint16_t>(arena, mr.off_val), ws,
                                  wsb, s)) != FL_OK)
        return st;
    hipLaunchKernelGGL(k_batch_summary, dim3(1), dim3(64), 0, s, sum, f->npiv, (uint32_t)mr.maxr,
                       (const uint32_t *)rank, (const uint64_t *)rp, (uint64_t)FL_OK);
    FL_LAUNCH_CHECK("k_batch_summary");
    return FL_OK;
}

fl_status batch_run(fl_batch *b, void *arena, size_t bytes, hipStream_t stream) {
    FL_ARG(b && arena, "fl_batch_run: NULL argument");
    if (bytes < b->run_bytes) {
        fl_set_error("fl_batch_run: run arena too small");
        return FL_ERR_WORKSPACE;
    }
    const uint32_t S = b->cfg.streams;
    FL_HIP(hipEventRecord(b->fork, stream));
    for (uint32_t k = 0; k < S; k++) FL_HIP(hipStreamWaitEvent(b->streams[k], b->fork, 0));
    // largest matrices first on each branch, as dealt
    std::vector<uint32_t> order(b->count);
    for (uint32_t i = 0; i < b->count; i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t x, uint32_t y) { return b->mats[x].cost > b->mats[y].cost; });
    fl_status first = FL_OK;
    for (uint32_t i : order) {
        const MatrixRun &mr = b->mats[i];
        fl_status st = run_one(b, mr, arena, b->streams[mr.branch]);
        if (st != FL_OK && first == FL_OK) first = st;
    }
    for (uint32_t k = 0; k < S; k++) {
        FL_HIP(hipEventRecord(b->join[k], b->streams[k]));
        FL_HIP(hipStreamWaitEvent(stream, b->join[k], 0));
    }
    return first;
}

void batch_destroy(fl_batch *b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (uint32_t k = 0; k < kMaxStreams; k++) {
        if (b->streams[k]) (void)hipStreamDestroy(b->streams[k]);
        if (b->join[k]) (void)hipEventDestroy(b->join[k]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    delete b;
}

fl_status batch_plan(const fl_csr *Ms, uint32_t count, uint32_t p, const fl_batch_config *cfg,
                     void *split_arena, size_t split_bytes, fl_batch **out, hipStream_t stream) {
    FL_ARG(Ms && out && count, "fl_batch_plan: NULL argument or empty batch");
    FL_ARG(p >= 2 && p <= 65521, "fl_batch_plan: p must be in [2, 65521]");
    *out = nullptr;
    const fl_batch_config c = resolve(cfg, Ms, count, p);
    FL_ARG(c.ml_width == 1 || c.ml_width == 2 || c.ml_width == 4 || c.ml_width == 8,
           "fl_batch_plan: ml_width must be 1, 2, 4 or 8");
    FL_ARG(c.streams >= 1 && c.streams <= kMaxStreams, "fl_batch_plan: streams must be in [1, 16]");
    const uint32_t w = c.ml_width;
    if (!split_arena || split_bytes < split_arena_bytes(Ms, count, w)) {
        fl_set_error("fl_batch_plan: split arena too small");
        return FL_ERR_WORKSPACE;
    }
    fl_batch *b = new fl_batch;
    b->count = count;
    b->p = p;
    b->cfg = c;
    b->mats.resize(count);
    uint64_t o = 0;
    std::vector<SplitSlice> sl(count);
    for (uint32_t i = 0; i < count; i++) {
        sl[i] = split_slice(o, Ms[i], w);
        o = sl[i].end;
    }
    const uint64_t ws_off = o;
    const size_t ws_bytes = split_ws_max(Ms, count, w);
    char *base = (char *)split_arena;
    for (uint32_t i = 0; i < count; i++) {
        MatrixRun &mr = b->mats[i];
        mr.M = Ms[i];
        const SplitSlice &s = sl[i];
        fl_split_out &so = mr.out;
        so.row_perm = (uint32_t *)(base + s.row_perm);
        so.col_perm = (uint32_t *)(base + s.col_perm);
        so.a_gptr = (uint64_t *)(base + s.a_gptr);
        so.a_pos = (uint32_t *)(base + s.a_pos);
        so.a_val = (uint16_t *)(base + s.a_val);
        so.b_ptr = (uint64_t *)(base + s.b_ptr);
        so.b_col = (uint32_t *)(base + s.b_col);
        so.b_val = (uint16_t *)(base + s.b_val);
        so.c_gptr = (uint64_t *)(base + s.c_gptr);
        so.c_pos = (uint32_t *)(base + s.c_pos);
        so.c_val = (uint16_t *)(base + s.c_val);
        so.d_ptr = (uint64_t *)(base + s.d_ptr);
        so.d_col = (uint32_t *)(base + s.d_col);
        so.d_val = (uint16_t *)(base + s.d_val);
        fl_status st = fl_split_enqueue(&Ms[i], p, w, &so, base + ws_off, ws_bytes,
                                        (uint64_t *)(base + s.dinfo), stream);
        if (st != FL_OK) {
            batch_destroy(b);
            return st;
        }
    }
    // one synchronisation for the size words of every matrix
    std::vector<uint64_t> hinf(8 * (size_t)count);
    for (uint32_t i = 0; i < count; i++)
        if (Ms[i].rows) {
            hipError_t e = hipMemcpyAsync(&hinf[8 * (size_t)i], base + sl[i].dinfo, 64,
                                          hipMemcpyDeviceToHost, stream);
            if (e != hipSuccess) {
                batch_destroy(b);
                FL_HIP(e);
            }
        }
    {
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            batch_destroy(b);
            FL_HIP(e);
        }
    }
    for (uint32_t i = 0; i < count; i++) {
        MatrixRun &mr = b->mats[i];
        mr.status = fl_split_finish(&Ms[i], p, w, &hinf[8 * (size_t)i], &mr.info);
    }
    batch_layout(b);
    fl_status st = batch_init_streams(b);
    if (st != FL_OK) {
        batch_destroy(b);
        return st;
    }
    *out = b;
    return FL_OK;
}

}  // namespace

extern "C" size_t fl_batch_split_workspace(const fl_csr *Ms, uint32_t count, uint32_t ml_width) {
    if (!Ms || !count) return 0;
    if (ml_width == 0) ml_width = 2;
    return split_arena_bytes(Ms, count, ml_width);
}

extern "C" fl_status fl_batch_plan(const fl_csr *Ms, uint32_t count, uint32_t p,
                                   const fl_batch_config *cfg, void *split_arena, size_t split_bytes,
                                   fl_batch **plan, hipStream_t stream) {
    return batch_plan(Ms, count, p, cfg, split_arena, split_bytes, plan, stream);
}

extern "C" size_t fl_batch_run_workspace(const fl_batch *plan) { return plan ? plan->run_bytes : 0; }

extern "C" fl_status fl_batch_run(fl_batch *plan, void *run_arena, size_t run_bytes,
                                  hipStream_t stream) {
    return batch_run(plan, run_arena, run_bytes, stream);
}

extern "C" fl_status fl_batch_graph_build(fl_batch *plan, void *run_arena, size_t run_bytes,
                                          hipStream_t stream) {
    FL_ARG(plan && run_arena, "fl_batch_graph_build: NULL argument");
    // the legacy null stream cannot be captured: use the plan's own stream,
    // ordered after the caller's work
    if (!stream) {
        FL_HIP(hipStreamSynchronize(nullptr));
        stream = plan->capture;
    }
    if (run_bytes < plan->run_bytes) {
        fl_set_error("fl_batch_graph_build: run arena too small");
        return FL_ERR_WORKSPACE;
    }
    if (plan->exec) {
        (void)hipGraphExecDestroy(plan->exec);
        plan->exec = nullptr;
    }
    if (plan->graph) {
        (void)hipGraphDestroy(plan->graph);
        plan->graph = nullptr;
    }
    const bool prof = fl_prof_set(false);  // no event records inside the graph
    hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        fl_prof_set(prof);
        FL_HIP(e);
    }
    fl_status st = batch_run(plan, run_arena, run_bytes, stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(stream, &g);
    fl_prof_set(prof);
    if (st != FL_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    FL_HIP(e);
    plan->graph = g;
    FL_HIP(hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0));
    return FL_OK;
}

extern "C" fl_status fl_batch_graph_launch(fl_batch *plan, hipStream_t stream) {
    FL_ARG(plan && plan->exec, "fl_batch_graph_launch: no graph built");
    FL_HIP(hipGraphLaunch(plan->exec, stream));
    return FL_OK;
}

extern "C" uint64_t *fl_batch_summary(const fl_batch *plan, void *run_arena) {
    if (!plan || !run_arena) return nullptr;
    return (uint64_t *)((char *)run_arena + plan->summary_off);
}

extern "C" fl_status fl_batch_matrix_info(const fl_batch *plan, uint32_t i, void *run_arena,
                                          fl_batch_matrix *out) {
    FL_ARG(plan && run_arena && out, "fl_batch_matrix_info: NULL argument");
    FL_ARG(i < plan->count, "fl_batch_matrix_info: index out of range");
    const MatrixRun &mr = plan->mats[i];
    char *base = (char *)run_arena;
    out->status = mr.status;
    out->mode = mr.mode;
    out->npiv = mr.info.npiv;
    out->mD = mr.info.mD;
    out->nB = mr.info.nB;
    out->rank_max = (uint32_t)(mr.info.npiv + mr.maxr);
    out->nnz_cap = mr.status == FL_OK ? mr.nnz_cap : 0;
    out->row_ptr = mr.status == FL_OK ? (uint64_t *)(base + mr.off_rowptr) : nullptr;
    out->col = mr.status == FL_OK ? (uint32_t *)(base + mr.off_col) : nullptr;
    out->val = mr.status == FL_OK ? (uint16_t *)(base + mr.off_val) : nullptr;
    return FL_OK;
}

extern "C" void fl_batch_get_config(const fl_batch *plan, fl_batch_config *out) {
    if (plan && out) *out = plan->cfg;
}

extern "C" void fl_batch_free(fl_batch *plan) { batch_destroy(plan); }

extern "C" fl_status fl_batch_autotune(const fl_csr *Ms, uint32_t count, uint32_t p,
                                       void *split_arena, size_t split_bytes, void *run_arena,
                                       size_t run_bytes, fl_batch_config *best, double *best_ms,
                                       hipStream_t stream) {
    FL_ARG(Ms && count && split_arena && run_arena && best, "fl_batch_autotune: NULL argument");
    hipEvent_t e0, e1;
    FL_HIP(hipEventCreate(&e0));
    FL_HIP(hipEventCreate(&e1));
    // one full timed pass (plan + run) per candidate, after one warm-up
    auto measure = [&](const fl_batch_config &c, double *ms) -> fl_status {
        *ms = INFINITY;
        if (split_bytes < split_arena_bytes(Ms, count, c.ml_width)) return FL_OK;
        float best_t = INFINITY;
        for (int rep = 0; rep < 2; rep++) {
            fl_batch *b = nullptr;
            FL_HIP(hipEventRecord(e0, stream));
            fl_status st = batch_plan(Ms, count, p, &c, split_arena, split_bytes, &b, stream);
            if (st != FL_OK) return st;
            if (b->run_bytes > run_bytes) {
                batch_destroy(b);
                return FL_OK;
            }
            st = batch_run(b, run_arena, run_bytes, stream);
            if (st == FL_OK) {
                hipError_t he = hipEventRecord(e1, stream);
                if (he == hipSuccess) he = hipEventSynchronize(e1);
                float t = 0;
                if (he == hipSuccess) he = hipEventElapsedTime(&t, e0, e1);
                if (he != hipSuccess) {
                    batch_destroy(b);
                    FL_HIP(he);
                }
                if (rep) best_t = t;
            }
            batch_destroy(b);
            if (st != FL_OK) return st;
        }
        *ms = best_t;
        return FL_OK;
    };
    fl_batch_config cur = {2, 8, kDefaultMfmaMin};
    double cur_ms;
    fl_status st = measure(cur, &cur_ms);
    // coordinate descent: multiline width, then MFMA threshold, then branches
    const uint32_t widths[] = {1, 4};
    const uint64_t thresholds[] = {(uint64_t)1 << 18, (uint64_t)1 << 26, ~(uint64_t)0};
    const uint32_t branches[] = {4, 16};
    for (uint32_t w : widths) {
        if (st != FL_OK) break;
        fl_batch_config c = cur;
        c.ml_width = w;
        double ms;
        st = measure(c, &ms);
        if (ms < cur_ms) cur = c, cur_ms = ms;
    }
    for (uint64_t t : thresholds) {
        if (st != FL_OK) break;
        fl_batch_config c = cur;
        c.mfma_min_entries = t;
        double ms;
        st = measure(c, &ms);
        if (ms < cur_ms) cur = c, cur_ms = ms;
    }
    for (uint32_t s : branches) {
        if (st != FL_OK) break;
        fl_batch_config c = cur;
        c.streams = s;
        double ms;
        st = measure(c, &ms);
        if (ms < cur_ms) cur = c, cur_ms = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != FL_OK) return st;
    if (!isfinite(cur_ms)) {
        fl_set_error("fl_batch_autotune: no candidate fits the arenas");
        return FL_ERR_WORKSPACE;
    }
    *best = cur;
    if (best_ms) *best_ms = cur_ms;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[shape_key(Ms, count, p)] = cur;
    return FL_OK;
}
