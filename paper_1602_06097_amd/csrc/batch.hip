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
constexpr uint32_t kDefaultQueuePerCu = 2;
constexpr uint32_t kDefaultFarGroups = 128;

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
    uint64_t off_X, off_Dt, off_rank, off_piv, off_rowptr, off_col, off_val, off_ws, ws_bytes;
    uint32_t nblk, npanels;  // TRSM blocks and echelon panels
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
    fl_batch_config c = {};
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
    if (c.queue_per_cu == 0) c.queue_per_cu = kDefaultQueuePerCu;
    if (c.far_groups == 0) c.far_groups = kDefaultFarGroups;
    return c;
}

}  // namespace

struct fl_batch {
    uint32_t count = 0, p = 0;
    fl_batch_config cfg = {};
    std::vector<MatrixRun> mats;
    uint64_t summary_off = 0, run_bytes = 0;
    // device tables of the stepped loops (TRSM blocks, echelon panels)
    uint64_t off_ttask = 0, off_tids = 0, off_tpre = 0;  // 4 lists each (solves and updates by form)
    uint64_t off_etask = 0, off_eids = 0, off_epre_rows = 0, off_epre = 0;
    uint64_t off_queue = 0;  // work-queue counters of the stepped launches (4 per TRSM step)
    uint32_t n_queue = 0;
    uint32_t max_blk = 0, max_panels = 0;
    hipStream_t streams[kMaxStreams] = {};
    hipStream_t capture = nullptr;  // graph capture when the caller passes the null stream
    hipEvent_t fork = nullptr, join[kMaxStreams] = {};
    // second stream of the panel loop (its far part) and its events
    hipStream_t ech_far = nullptr;
    hipEvent_t ech_near_ev = nullptr, ech_far_ev = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

fl_status batch_init_streams(fl_batch *b) {
    FL_HIP(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
    FL_HIP(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
    FL_HIP(hipStreamCreateWithFlags(&b->ech_far, hipStreamNonBlocking));
    FL_HIP(hipEventCreateWithFlags(&b->ech_near_ev, hipEventDisableTiming));
    FL_HIP(hipEventCreateWithFlags(&b->ech_far_ev, hipEventDisableTiming));
    for (uint32_t k = 0; k < b->cfg.streams; k++) {
        FL_HIP(hipStreamCreateWithFlags(&b->streams[k], hipStreamNonBlocking));
        FL_HIP(hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming));
    }
    return FL_OK;
}

// Lays out the run arena from the split sizes and deals matrices to branches.
// Every matrix has its own workspace: the stepped loops keep the state of all
// matrices alive at once.
void batch_layout(fl_batch *b) {
    const uint32_t S = b->cfg.streams;
    std::vector<double> load(S, 0.0);
    std::vector<uint32_t> order(b->count);
    for (uint32_t i = 0; i < b->count; i++) order[i] = i;
    b->max_blk = b->max_panels = 0;
    for (auto &mr : b->mats) {
        const fl_split_info &f = mr.info;
        mr.maxr = std::min(f.mD, f.nB);
        mr.cost = (double)f.nnzA * f.nB + (double)f.nnzC * f.nB +
                  (double)f.mD * f.nB * (double)std::min<uint64_t>(mr.maxr, 4096) +
                  (double)f.npiv * f.nB * (double)mr.maxr * 0.25 + (double)f.nnz;
        const uint64_t dense = ((uint64_t)f.npiv + f.mD) * f.nB;
        mr.mode = dense >= b->cfg.mfma_min_entries ? FL_MFMA_I8 : FL_PLAIN;
        const bool ok = mr.status == FL_OK;
        mr.nblk = ok && f.npiv && f.nB ? (f.npiv + kFlTrsmBlock - 1) / kFlTrsmBlock : 0;
        mr.npanels = ok && f.mD && f.nB ? (f.nB + 63) / 64 : 0;
        b->max_blk = std::max(b->max_blk, mr.nblk);
        b->max_panels = std::max(b->max_panels, mr.npanels);
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t x, uint32_t y) { return b->mats[x].cost > b->mats[y].cost; });
    for (uint32_t i : order) {
        MatrixRun &mr = b->mats[i];
        uint32_t k = (uint32_t)(std::min_element(load.begin(), load.end()) - load.begin());
        mr.branch = k;
        load[k] += mr.cost + 2e6;  // per-matrix launch overhead, in work units
    }
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t at = o;
        o = align256(o + (bytes ? bytes : 1));
        return at;
    };
    const uint64_t n = b->count;
    b->summary_off = take(32 * n);
    b->off_ttask = take(sizeof(FlTrsmTask) * n);
    b->off_tids = take(4 * 4 * n);
    b->off_tpre = take(4 * 4 * (n + 1));
    b->off_etask = take(sizeof(FlEchTask) * n);
    b->off_eids = take(4 * 3 * n);
    b->off_epre_rows = take(4 * (n + 1));
    b->off_epre = take(4 * (3 * (uint64_t)b->max_panels + 6 * (uint64_t)((b->max_panels + 3) / 4)) * (n + 1));
    b->n_queue = 4 * b->max_blk;
    b->off_queue = take(4 * (uint64_t)(b->n_queue ? b->n_queue : 1));
    for (auto &mr : b->mats) {
        const fl_split_info &f = mr.info;
        mr.ldx = ld64(f.nB);
        mr.ldd = ld64(f.nB);
        mr.nnz_cap = ((uint64_t)f.npiv + mr.maxr) * ((uint64_t)f.nB + 1);
        if (mr.status != FL_OK) {
            mr.off_X = mr.off_Dt = mr.off_rank = mr.off_piv = mr.off_rowptr = mr.off_col = mr.off_val = 0;
            mr.off_ws = mr.ws_bytes = 0;
            continue;
        }
        const fl_split_info *fi = &mr.info;
        size_t w = fl_trsm_workspace(fi, mr.mode);
        w = std::max(w, fl_reduce_cd_workspace(fi, mr.mode));
        w = std::max(w, fl_echelon_d_workspace(fi->mD, fi->nB, mr.mode));
        w = std::max(w, fl_rref_workspace(fi, mr.mode));
        w = std::max(w, fl_rref_csr_workspace(fi));
        mr.ws_bytes = std::max<uint64_t>(w, 256);
        mr.off_ws = take(mr.ws_bytes);
        mr.off_X = take(2 * mr.ldx * std::max<uint64_t>(f.npiv, 1));
        mr.off_Dt = take(2 * mr.ldd * std::max<uint64_t>(f.mD, 1));
        mr.off_rank = take(4);
        mr.off_piv = take(4 * std::max<uint64_t>(mr.maxr, 1));
        mr.off_rowptr = take(8 * ((uint64_t)f.npiv + mr.maxr + 1));
        mr.off_col = take(4 * mr.nnz_cap);
        mr.off_val = take(2 * mr.nnz_cap);
    }
    b->run_bytes = o;
}

template <class T>
T *at(void *arena, uint64_t off) {
    return (T *)((char *)arena + off);
}

fl_status fork(fl_batch *b, hipStream_t stream) {
    FL_HIP(hipEventRecord(b->fork, stream));
    for (uint32_t k = 0; k < b->cfg.streams; k++) FL_HIP(hipStreamWaitEvent(b->streams[k], b->fork, 0));
    return FL_OK;
}

fl_status join(fl_batch *b, hipStream_t stream) {
    for (uint32_t k = 0; k < b->cfg.streams; k++) {
        FL_HIP(hipEventRecord(b->join[k], b->streams[k]));
        FL_HIP(hipStreamWaitEvent(stream, b->join[k], 0));
    }
    return FL_OK;
}

// Indices of the matrices with key(i) > 0, largest key first (stable).
template <class F>
std::vector<uint32_t> sorted_ids(const fl_batch *b, F key, int mode_filter) {
    std::vector<uint32_t> ids;
    for (uint32_t i = 0; i < b->count; i++)
        if (key(b->mats[i]) > 0 && (mode_filter < 0 || (int)b->mats[i].mode == mode_filter)) ids.push_back(i);
    std::stable_sort(ids.begin(), ids.end(), [&](uint32_t x, uint32_t y) { return key(b->mats[x]) > key(b->mats[y]); });
    return ids;
}

fl_status upload_ids(void *dst, const std::vector<uint32_t> &v, hipStream_t s) {
    if (!v.empty()) FL_HIP(fl_upload(dst, v.data(), 4 * v.size(), s));
    return FL_OK;
}

// Workgroup prefix over ids of per-matrix counts.
template <class F>
std::vector<uint32_t> prefix_of(const fl_batch *b, const std::vector<uint32_t> &ids, F count) {
    std::vector<uint32_t> pre(ids.size() + 1, 0);
    for (size_t i = 0; i < ids.size(); i++) pre[i + 1] = pre[i] + count(b->mats[ids[i]]);
    return pre;
}

// The batched TRSM: per-matrix set-up on the branches, then one launch per
// step and kind for all matrices (step s solves block nblk - 1 - s of each).
fl_status run_trsm(fl_batch *b, void *arena, hipStream_t stream) {
    const uint32_t n = b->count, w = b->cfg.ml_width;
    std::vector<FlTrsmTask> tasks(n);
    FL_CHECK_ST(fork(b, stream));
    for (uint32_t i = 0; i < n; i++) {
        MatrixRun &mr = b->mats[i];
        tasks[i] = FlTrsmTask{};
        if (mr.status != FL_OK) continue;
        FL_CHECK_ST(fl_trsm_prepare(&mr.info, &mr.out, at<uint16_t>(arena, mr.off_X), mr.ldx, mr.mode,
                                    at<char>(arena, mr.off_ws), mr.ws_bytes, b->streams[mr.branch], &tasks[i]));
    }
    FL_CHECK_ST(join(b, stream));
    if (b->max_blk == 0) return FL_OK;
    auto nblk = [](const MatrixRun &m) { return m.nblk; };
    // lists: 0 = MFMA-form solve (product with the block inverse), 1 = MFMA
    // update, 2 = VALU update, 3 = VALU-form solve (back substitution)
    const std::vector<uint32_t> ids[4] = {sorted_ids(b, nblk, FL_MFMA_I8), sorted_ids(b, nblk, FL_MFMA_I8),
                                          sorted_ids(b, nblk, FL_PLAIN), sorted_ids(b, nblk, FL_PLAIN)};
    const std::vector<uint32_t> pre[4] = {
        prefix_of(b, ids[0], [](const MatrixRun &m) { return (m.info.nB + 63) / 64; }),
        prefix_of(b, ids[1], [](const MatrixRun &m) { return (m.info.nB + 127) / 128 * kFlTrsmSuper; }),
        prefix_of(b, ids[2], [&](const MatrixRun &m) { return (m.info.nB + 255) / 256 * (kFlTrsmBlock / w / 4); }),
        prefix_of(b, ids[3], [](const MatrixRun &m) { return (m.info.nB + 63) / 64; })};
    FlTrsmTask *d_tasks = at<FlTrsmTask>(arena, b->off_ttask);
    FL_HIP(fl_upload(d_tasks, tasks.data(), sizeof(FlTrsmTask) * n, stream));
    uint32_t *d_ids[4], *d_pre[4];
    for (int k = 0; k < 4; k++) {
        d_ids[k] = at<uint32_t>(arena, b->off_tids) + (size_t)k * n;
        d_pre[k] = at<uint32_t>(arena, b->off_tpre) + (size_t)k * (n + 1);
        FL_CHECK_ST(upload_ids(d_ids[k], ids[k], stream));
        FL_CHECK_ST(upload_ids(d_pre[k], pre[k], stream));
    }
    const int kind_of[4] = {3, 1, 0, 2};
    std::vector<uint32_t> active(4);
    for (int k = 0; k < 4; k++) active[k] = (uint32_t)ids[k].size();
    // one counter per (step, kind), all cleared by one fill kernel (captured
    // with the run, so every graph replay starts from zero)
    uint32_t *queue = at<uint32_t>(arena, b->off_queue);
    const uint32_t per_cu = b->cfg.queue_per_cu == FL_BATCH_DIRECT ? 0 : b->cfg.queue_per_cu;
    FL_HIP(fl_fill_u32(queue, 0, b->n_queue, stream));
    for (uint32_t step = 0; step < b->max_blk; step++) {
        for (int k : {1, 2, 0, 3}) {  // updates of the step, then its solves
            while (active[k] && b->mats[ids[k][active[k] - 1]].nblk <= step) active[k]--;
            if (!active[k]) continue;
            FL_HIP(fl_trsm_batch_launch(kind_of[k], b->p, w, d_tasks, d_ids[k], d_pre[k], active[k],
                                        pre[k][active[k]], step, queue + 4 * step + k, per_cu, stream));
        }
    }
    return FL_OK;
}

// The batched echelon: set-up per matrix, one launch per panel and kernel for
// all matrices, then the final row placement per matrix on the branches.
fl_status run_echelon(fl_batch *b, void *arena, std::vector<FlEchTask> &tasks, hipStream_t stream) {
    const uint32_t n = b->count;
    if (b->max_panels == 0) return FL_OK;
    auto npan = [](const MatrixRun &m) { return m.npanels; };
    const std::vector<uint32_t> ids[3] = {sorted_ids(b, npan, -1), sorted_ids(b, npan, FL_MFMA_I8),
                                          sorted_ids(b, npan, FL_PLAIN)};
    const std::vector<uint32_t> pre_rows =
        prefix_of(b, ids[0], [](const MatrixRun &m) { return (m.info.mD + 31) / 32; });
    FlEchTask *d_tasks = at<FlEchTask>(arena, b->off_etask);
    FL_HIP(fl_upload(d_tasks, tasks.data(), sizeof(FlEchTask) * n, stream));
    uint32_t *d_ids[3];
    for (int k = 0; k < 3; k++) {
        d_ids[k] = at<uint32_t>(arena, b->off_eids) + (size_t)k * n;
        FL_CHECK_ST(upload_ids(d_ids[k], ids[k], stream));
    }
    uint32_t *d_pre_rows = at<uint32_t>(arena, b->off_epre_rows);
    FL_CHECK_ST(upload_ids(d_pre_rows, pre_rows, stream));
    const uint32_t Pm = b->max_panels, Bm = (Pm + 3) / 4;
    uint32_t *q = at<uint32_t>(arena, b->off_epre);
    auto take_tab = [&q, n](uint32_t count) {
        uint32_t *r = q;
        q += (size_t)count * (n + 1);
        return r;
    };
    FlEchLists L = {};
    L.ids_all = d_ids[0];
    L.ids_mfma = d_ids[1];
    L.ids_plain = d_ids[2];
    L.n_all = (uint32_t)ids[0].size();
    L.n_mfma = (uint32_t)ids[1].size();
    L.n_plain = (uint32_t)ids[2].size();
    L.pre_rows = d_pre_rows;
    L.pre_n_all = take_tab(Pm);
    L.pre_n_mfma = take_tab(Pm);
    L.pre_n_plain = take_tab(Pm);
    L.pre_bn_all = take_tab(Bm);
    L.pre_bn_mfma = take_tab(Bm);
    L.pre_bn_plain = take_tab(Bm);
    L.pre_bf_all = take_tab(Bm);
    L.pre_bf_mfma = take_tab(Bm);
    L.pre_bf_plain = take_tab(Bm);
    FL_HIP(fl_echelon_prefixes(d_tasks, L, Pm, Bm, stream));
    FlEchAux aux = {b->ech_far, b->ech_near_ev, b->ech_far_ev, false, b->cfg.far_groups};
    uint32_t active = L.n_all;
    auto active_at = [&](uint32_t P, uint32_t a) {
        while (a && b->mats[ids[0][a - 1]].npanels <= P) a--;
        return a;
    };
    for (uint32_t P = 0; P < Pm; P++) {
        active = active_at(P, active);
        if (!active) break;
        FlEchGrid g = {};
        g.n_active = active;
        g.grid_rows = pre_rows[active];
        g.n_next = active_at(P + 1, active);
        g.grid_rows_next = g.n_next ? pre_rows[g.n_next] : 0;
        for (uint32_t i : ids[1])
            if (b->mats[i].npanels > P) {
                g.n_mfma++;
                g.mfma_rows = std::max(g.mfma_rows, b->mats[i].info.mD);
            }
        for (uint32_t i : ids[2])
            if (b->mats[i].npanels > P) g.n_plain++;
        FlEchBlockGrid bg = {};
        const bool end = P % 4 == 3 || !g.n_next;
        if (end) {
            const uint64_t bend = (uint64_t)(P / 4 + 1) * kFlEchBlock;
            for (uint32_t i : ids[0]) {
                bg.bn_all += fl_ech_tiles(b->mats[i].info.nB, bend, kFlEchBlock, 64);
                bg.bf_all += fl_ech_tiles(b->mats[i].info.nB, bend + kFlEchBlock, ~0ull, 64);
            }
            for (uint32_t i : ids[1]) {
                const uint32_t cols = b->mats[i].info.nB;
                bg.bn_mfma += fl_ech_tiles(cols, bend, kFlEchBlock, 64);
                bg.bf_mfma += fl_ech_tiles(cols, bend + kFlEchBlock, ~0ull, 128);
                if (cols > bend) bg.mfma_rows = std::max(bg.mfma_rows, b->mats[i].info.mD);
            }
            for (uint32_t i : ids[2]) {
                bg.bn_plain += fl_ech_tiles(b->mats[i].info.nB, bend, kFlEchBlock, 256);
                bg.bf_plain += fl_ech_tiles(b->mats[i].info.nB, bend + kFlEchBlock, ~0ull, 256);
            }
        }
        FL_HIP(fl_echelon_batch_panel(b->p, d_tasks, L, P, g, end ? &bg : nullptr, stream, aux));
    }
    FL_HIP(fl_echelon_join(stream, aux));
    return FL_OK;
}

fl_status batch_run(fl_batch *b, void *arena, size_t bytes, hipStream_t stream) {
    FL_ARG(b && arena, "fl_batch_run: NULL argument");
    if (bytes < b->run_bytes) {
        fl_set_error("fl_batch_run: run arena too small");
        return FL_ERR_WORKSPACE;
    }
    const uint32_t n = b->count;
    // step 2: X = A^-1 B for every matrix
    FL_CHECK_ST(run_trsm(b, arena, stream));
    // step 3 and the echelon set-up, per matrix on the branches
    std::vector<FlEchTask> etasks(n);
    FL_CHECK_ST(fork(b, stream));
    for (uint32_t i = 0; i < n; i++) {
        MatrixRun &mr = b->mats[i];
        etasks[i] = FlEchTask{};
        if (mr.status != FL_OK) continue;
        const fl_split_info *f = &mr.info;
        hipStream_t s = b->streams[mr.branch];
        void *ws = at<char>(arena, mr.off_ws);
        uint16_t *X = at<uint16_t>(arena, mr.off_X), *Dt = at<uint16_t>(arena, mr.off_Dt);
        FL_CHECK_ST(fl_reduce_cd(f, &mr.out, X, mr.ldx, Dt, mr.ldd, mr.mode, ws, mr.ws_bytes, s));
        FL_CHECK_ST(fl_echelon_prepare(b->p, f->mD, f->nB, Dt, mr.ldd, at<uint32_t>(arena, mr.off_rank),
                                       at<uint32_t>(arena, mr.off_piv), mr.mode, ws, mr.ws_bytes, s, &etasks[i]));
    }
    FL_CHECK_ST(join(b, stream));
    // step 4: the panel loop for every matrix
    FL_CHECK_ST(run_echelon(b, arena, etasks, stream));
    // placement, second pass, read-off and summary, per matrix
    FL_CHECK_ST(fork(b, stream));
    for (uint32_t i = 0; i < n; i++) {
        MatrixRun &mr = b->mats[i];
        hipStream_t s = b->streams[mr.branch];
        uint64_t *sum = at<uint64_t>(arena, b->summary_off) + 4 * (size_t)i;
        if (mr.status != FL_OK) {
            hipLaunchKernelGGL(k_batch_skip, dim3(1), dim3(64), 0, s, sum, (uint64_t)mr.status);
            FL_LAUNCH_CHECK("k_batch_skip");
            continue;
        }
        const fl_split_info *f = &mr.info;
        void *ws = at<char>(arena, mr.off_ws);
        uint16_t *X = at<uint16_t>(arena, mr.off_X), *Dt = at<uint16_t>(arena, mr.off_Dt);
        uint32_t *rank = at<uint32_t>(arena, mr.off_rank), *piv = at<uint32_t>(arena, mr.off_piv);
        uint64_t *rp = at<uint64_t>(arena, mr.off_rowptr);
        FL_CHECK_ST(fl_echelon_finish(etasks[i], s));
        FL_CHECK_ST(fl_rref(f, &mr.out, X, mr.ldx, Dt, mr.ldd, rank, piv, mr.mode, ws, mr.ws_bytes, s));
        FL_CHECK_ST(fl_rref_csr_enqueue(f, &mr.out, X, mr.ldx, Dt, mr.ldd, rank, piv, rp,
                                        at<uint32_t>(arena, mr.off_col), at<uint16_t>(arena, mr.off_val), ws,
                                        mr.ws_bytes, s));
        hipLaunchKernelGGL(k_batch_summary, dim3(1), dim3(64), 0, s, sum, f->npiv, (uint32_t)mr.maxr,
                           (const uint32_t *)rank, (const uint64_t *)rp, (uint64_t)FL_OK);
        FL_LAUNCH_CHECK("k_batch_summary");
    }
    FL_CHECK_ST(join(b, stream));
    return FL_OK;
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
    if (b->ech_far) (void)hipStreamDestroy(b->ech_far);
    if (b->ech_near_ev) (void)hipEventDestroy(b->ech_near_ev);
    if (b->ech_far_ev) (void)hipEventDestroy(b->ech_far_ev);
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
    struct Events {  // destroyed on every return path
        hipEvent_t a = nullptr, b = nullptr;
        ~Events() {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } ev;
    FL_HIP(hipEventCreate(&ev.a));
    FL_HIP(hipEventCreate(&ev.b));
    hipEvent_t e0 = ev.a, e1 = ev.b;
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
    fl_batch_config cur = {2, 8, kDefaultMfmaMin, kDefaultQueuePerCu, kDefaultFarGroups};
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
    // launch geometry: work-queue width of the stepped TRSM launches (or
    // one workgroup per tile), column groups of the far echelon updates
    const uint32_t queues[] = {FL_BATCH_DIRECT, 1, 4};
    const uint32_t groups[] = {32, 512};
    for (uint32_t qw : queues) {
        if (st != FL_OK) break;
        fl_batch_config c = cur;
        c.queue_per_cu = qw;
        double ms;
        st = measure(c, &ms);
        if (ms < cur_ms) cur = c, cur_ms = ms;
    }
    for (uint32_t gsz : groups) {
        if (st != FL_OK) break;
        fl_batch_config c = cur;
        c.far_groups = gsz;
        double ms;
        st = measure(c, &ms);
        if (ms < cur_ms) cur = c, cur_ms = ms;
    }
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
