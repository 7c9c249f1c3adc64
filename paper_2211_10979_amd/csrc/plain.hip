// Host side of the single-LP solver: context lifetime, the captured pivot
// graph, and the C entry points lp_create ... lp_destroy.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "common.hpp"
#include "fused_launch.hpp"
#include "lane.hpp"
#include "plain_kernels.hpp"

using namespace lpgpu;

namespace {

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

struct UpdateConfig {
    int block;      // threads per workgroup
    int cols;       // listed columns per workgroup
    int rv;         // row pairs (double2) per thread and column
    int rowchunks;  // row chunks of block*rv pairs covering rows 0..m
    int nt;         // bit 0: non-temporal loads, bit 1: non-temporal stores
    int gs_per_cu;  // > 0: grid-stride kernel with this many workgroups per CU
    int gs_unroll;  // tiles in flight per thread in the grid-stride kernel
};

// Small m: one chunk of 64 or 128 pairs; otherwise `block` threads (256 by
// default) with `rv` pairs each. Defaults from sweeps on MI355X: for one
// pivot per pass, one column and one pair per thread for tall tableaux (the
// most independent, shortest streams: 5.5 TB/s at m = 8000) and four columns
// per workgroup below 4096 rows; with pivot fusion, kFusedCols columns (the
// group's pivot columns are then loaded once per kFusedCols columns).
constexpr int kFusedCols = 8;
constexpr int kAutoFuse = 24;  // the group size when fuse_pivots is 0 (kMaxFuseSplit where 24 has no kernels)

UpdateConfig pick_update_config(int32_t m, int cols, int rv, int block, bool fused) {
    const int64_t nvec = ((int64_t)m + 2) / 2;
    if (nvec <= 128) {
        const int b = nvec <= 64 ? 64 : 128;
        return {b, cols > 0 ? cols : 4, 1, 1, 0, 0, 0};
    }
    if (cols <= 0) cols = fused ? kFusedCols : (nvec > 2048 ? 1 : 4);
    if (rv <= 0) rv = 1;
    if (block <= 0) block = 256;
    const int64_t span = block * (int64_t)rv;
    return {block, cols, rv, (int)((nvec + span - 1) / span), 0, 0, 0};
}

// (queried once per device)
int device_cu_count(int device) {
    static std::atomic<int> cache[64];
    if (device >= 0 && device < 64) {
        const int v = cache[device].load(std::memory_order_relaxed);
        if (v > 0) return v;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0) return 256;
    if (device >= 0 && device < 64) cache[device].store(cus, std::memory_order_relaxed);
    return cus;
}

bool valid_cols(int c) { return c == 1 || c == 2 || c == 4 || c == 8 || c == 16; }
bool valid_rv(int v) { return v == 1 || v == 2 || v == 4 || v == 8; }

}  // namespace

struct lp_ctx {
    int device = 0;
    int32_t m = 0, n = 0;
    int64_t W = 0, ld = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    double *T = nullptr;
    bool own_T = false;
    unsigned char *aux = nullptr;  // owned block holding every other device buffer below (carve_aux)
    double *F = nullptr;
    ArgMin *parts = nullptr;
    DevState *st = nullptr;
    int32_t *basis = nullptr;
    int32_t *log_r = nullptr, *log_q = nullptr;
    double *out = nullptr;
    int32_t *cols = nullptr;  // rewrite list (n+2)
    int32_t *pos = nullptr;   // position of each nonbasic column in the list (n+m)
    double *Rl = nullptr;     // normalised pivot row by list position (n+2)
    DevState *host_st = nullptr;  // pinned: two slots for the pipelined status read-back, one for the end
    unsigned long long *host_cols = nullptr;  // pinned: the work counters at the end of the last solve
    double *host_out = nullptr;               // pinned: extraction output
    bool counters_cached = false;             // host_st[2] and host_cols hold the device's current values
    bool solution_cached = false;             // host_out holds the extraction of the current tableau
    double eps_d = 1e-9, eps_p = 1e-9;
    int64_t max_pivots = 0, log_cap = 0;
    int nparts = 0;
    int cus = 256;
    UpdateConfig ucfg{};
    unsigned long long *cols_done = nullptr;  // device counter of rewritten columns
    RatioPart *rparts = nullptr;              // multi-workgroup select: ratio partials
    uint32_t *ticket = nullptr;               // multi-workgroup select: arrival counter
    int select_wgs = 1;                       // workgroups of the select kernel
    int chunk = 4;                            // pivots (K = 1) or groups (K > 1) per replay
    int fuse = 1;                             // pivots per update pass (K)
    int64_t Lg = 0;                           // list slots: n + 2 (K = 1) or n + 1 + K
    GroupState *gs = nullptr;                 // K > 1: decisions of the current group
    double *D = nullptr;                      // K > 1: row-0 entry of every slot during a group
    double *dump = nullptr;                   // K > 1: zero column written for slots past the list
    double *PV = nullptr;                     // K > 1: pivot rows after the group (one-launch decisions)
    SPart *sparts = nullptr;                  // K > 1: Step 1 partials of the staging kernel
    GRatio *grparts = nullptr;                // K > 1: Step 2 partials of the select workgroups
    GridSync *gsync = nullptr;                // K > 1: barrier counters of the decision kernel
    int decide_wgs = 0;                       // K > 1: > 0 = one-launch decision kernel, its workgroups
    int decide_block = 256;                   // K > 1: its threads per workgroup
    uint32_t decide_spin = kDefaultDecideSpin;
    bool force_gate_close = false;            // decide_spin -1: close the first decision launch's gate
    int32_t stall_fallbacks = 0;              // decision launches whose gate closed (then barrier-free)
    int nsparts = 0;
    bool use_graph = true;
    bool timing = false;
    // Deferred build (lp_reload_device with the one-launch decision kernel):
    // the inputs the first update pass reads, whether that pass is still to
    // come, and whether basic columns may be unstored (slack columns are
    // written only when they leave the basis).
    bool eager_build = false;
    // The host reads the state right after each group's decisions (instead
    // of one group behind), while the group's update pass runs.
    bool early_status = false;
    int64_t dev_stop_at = 0;  // the pause point the device state holds (the last one enqueued)
    const double *pend_A = nullptr, *pend_b = nullptr, *pend_c = nullptr;
    bool pending = false;
    bool first_ran = false;  // the first group of the current build was such a group
    bool lazy = false;
    bool first_slot[2] = {false, false};  // the chunk in this slot is the first group of a deferred build
    hipEvent_t ev_first[2] = {nullptr, nullptr};
    double first_ms = 0.0;
    // Two captured chunk graphs used alternately, so that the events of one
    // can be read while the other runs.
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    hipGraph_t graph[2] = {nullptr, nullptr};
    std::vector<hipEvent_t> ev_upd[2];  // timing mode: before/after each update kernel of a chunk
    hipEvent_t ev_start = nullptr, ev_stop = nullptr, ev_slot[2] = {nullptr, nullptr};
    // status read-back 2: host memory mapped into the device, two slots of
    // kPubStride bytes, each the solver state and the work counters as the
    // decision kernel leaves them, then a sequence word (pub_seq: the last
    // one asked for)
    unsigned char *pub = nullptr;
    uint32_t pub_seq = 0;
    uint32_t *xticket = nullptr;  // the mapped extraction's count of finished workgroups (zero between launches)
    double clock_khz = 0.0;       // rate of the device clock the kernels read (wall_clock64)
    double update_ms = 0.0;
    int64_t update_launches = 0;
    double update_ms_applied = 0.0;  // part of update_ms in launches that applied pivots
    int64_t applied_launches = 0;
    int64_t pivots_host = 0;
    int32_t status_host = LP_RUNNING;
    bool ran = false;
    double last_ms = -1.0;
    // General form (lp_create_general): the caller's sizes, the tableau's row
    // order and signs, and the phase reached (1: Phase I to run, 3: done).
    bool general = false;
    int32_t m_in = 0, n_in = 0, n_le = 0;
    std::vector<int32_t> perm;
    std::vector<double> sgn;
    double feas_scale = 1.0;
    int gphase = 0;
    int32_t *gpick = nullptr;  // device: the drive-out column found
    int32_t bland_after = 0;   // anti-cycling fallback (one pivot per pass)
};

namespace {

// The mapped blocks the kernels hand the solver state and the solution over
// in: allocating one costs more than a whole solve of a small LP, so a
// context that ends leaves its block here for the next context on the same
// device (kept until the process ends).
std::mutex g_pub_mu;
std::vector<std::pair<int, unsigned char *>> g_pub_free;

unsigned char *pub_take(int device) {
    std::lock_guard<std::mutex> lock(g_pub_mu);
    for (size_t k = 0; k < g_pub_free.size(); ++k)
        if (g_pub_free[k].first == device) {
            unsigned char *p = g_pub_free[k].second;
            g_pub_free.erase(g_pub_free.begin() + (std::ptrdiff_t)k);
            return p;
        }
    return nullptr;
}

void pub_give(int device, unsigned char *p) {
    std::lock_guard<std::mutex> lock(g_pub_mu);
    g_pub_free.emplace_back(device, p);
}

void free_ctx(lp_ctx *h) {
    if (!h) return;
    DeviceGuard g(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (int k = 0; k < 2; ++k) {
        if (h->gexec[k]) (void)hipGraphExecDestroy(h->gexec[k]);
        if (h->graph[k]) (void)hipGraphDestroy(h->graph[k]);
        for (auto e : h->ev_upd[k])
            if (e) (void)hipEventDestroy(e);
    }
    for (auto e : h->ev_first)
        if (e) (void)hipEventDestroy(e);
    if (h->own_T && h->T) (void)hipFree(h->T);
    if (h->aux) (void)hipFree(h->aux);
    if (h->host_st) (void)hipHostFree(h->host_st);
    if (h->host_cols) (void)hipHostFree(h->host_cols);
    if (h->pub) pub_give(h->device, h->pub);  // (its kernels have ended: the stream was synchronized above)
    if (h->host_out) (void)hipHostFree(h->host_out);
    if (h->ev_start) (void)hipEventDestroy(h->ev_start);
    if (h->ev_stop) (void)hipEventDestroy(h->ev_stop);
    for (auto &e : h->ev_slot)
        if (e) (void)hipEventDestroy(e);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

int validate_opts(const Options &o) {
    if (!(o.eps_dual >= 0.0) || !(o.eps_pivot >= 0.0) || !std::isfinite(o.eps_dual) || !std::isfinite(o.eps_pivot))
        return set_error(LP_E_INVAL, "eps_dual and eps_pivot must be finite and >= 0");
    if (o.cols_per_block != 0 && !valid_cols(o.cols_per_block))
        return set_error(LP_E_INVAL, "cols_per_block must be 0 (auto) or one of 1, 2, 4, 8, 16");
    if (o.rows_per_thread != 0 && !valid_rv(o.rows_per_thread))
        return set_error(LP_E_INVAL, "rows_per_thread must be 0 (auto) or one of 1, 2, 4, 8");
    if (o.update_hints < 0 || o.update_hints > 3) return set_error(LP_E_INVAL, "update_hints must be in [0, 3]");
    if (o.select_workgroups < 0 || o.select_workgroups > 64)
        return set_error(LP_E_INVAL, "select_workgroups must be in [0, 64]");
    if (o.update_grid_stride < 0 || o.update_grid_stride > 32)
        return set_error(LP_E_INVAL, "update_grid_stride must be in [0, 32]");
    if (o.update_unroll != 0 && o.update_unroll != 1 && o.update_unroll != 2 && o.update_unroll != 4 &&
        o.update_unroll != 8)
        return set_error(LP_E_INVAL, "update_unroll must be 0 (auto) or one of 1, 2, 4, 8");
    if (o.update_block != 0 && o.update_block != 64 && o.update_block != 128 && o.update_block != 256 &&
        o.update_block != 512 && o.update_block != 1024)
        return set_error(LP_E_INVAL, "update_block must be 0 (auto) or one of 64, 128, 256, 512, 1024");
    if (o.chunk_pivots < 0) return set_error(LP_E_INVAL, "chunk_pivots must be >= 0");
    if (o.fuse_pivots < 0 || o.fuse_pivots > kMaxFuse) return set_error(LP_E_INVAL, "fuse_pivots must be in [0, 48]");
    if (o.decide_kernel < 0 || o.decide_kernel > 1) return set_error(LP_E_INVAL, "decide_kernel must be 0 or 1");
    if (o.decide_spin < -1) return set_error(LP_E_INVAL, "decide_spin must be >= -1");
    if (o.decide_block != 0 && o.decide_block != 256 && o.decide_block != 512)
        return set_error(LP_E_INVAL, "decide_block must be 0 (auto), 256 or 512");
    if (o.eager_build < 0 || o.eager_build > 1) return set_error(LP_E_INVAL, "eager_build must be 0 or 1");
    if (o.status_readback < 0 || o.status_readback > 2)
        return set_error(LP_E_INVAL, "status_readback must be 0 (auto), 1 or 2");
    return LP_OK;
}

// The state block: DevState, then the work counters at a 64-byte offset.
constexpr size_t kCountersAt = (sizeof(DevState) + 63) / 64 * 64;
constexpr size_t kStateBlock = kCountersAt + 4 * sizeof(unsigned long long);
// a slot of the mapped block the decision kernel publishes to: the state
// block, then the sequence word
constexpr size_t kPubStride = (kStateBlock + sizeof(uint64_t) + 127) / 128 * 128;
// after the two slots: the device clock at the start of the solve and at the
// end of its pivoting, then the sequence word of the extraction
constexpr size_t kPubMarks = 2 * kPubStride;
constexpr size_t kPubBytes = kPubMarks + 128;

// status_readback 0 reads the state right after the decisions (2) wherever
// that form runs: with the state and the solution published by the kernels
// into mapped memory it is the faster one at every size measured (a solve of
// 200 x 200: 122 against 182 us per step; 2000 x 2000: 394 against 468).

// Resolves every launch choice of a context for an m x n LP from the
// options: group size, tile shapes, decision kernel, read-back mode. Only
// host fields are set; nothing is allocated.
int configure_ctx(lp_ctx *h, int32_t m, int32_t n, const Options &o) {
    h->device = o.device;
    h->m = m;
    h->n = n;
    h->W = (int64_t)n + m + 1;
    h->ld = padded_ld(m);
    h->eps_d = o.eps_dual;
    h->eps_p = o.eps_pivot;
    h->max_pivots = o.max_pivots > 0 ? o.max_pivots : 50 * ((int64_t)m + n);
    h->log_cap = o.record_pivots ? h->max_pivots : 0;
    // Pivot fusion: the given K, or kAutoFuse unless an option asks for a
    // form that only the one-pivot kernels have.
    if (o.bland_after < 0) return set_error(LP_E_INVAL, "bland_after must be >= 0");
    if (o.bland_after > 0 && (o.fuse_pivots > 1 || o.select_workgroups > 1))
        return set_error(LP_E_INVAL, "bland_after > 0 needs one pivot per pass: fuse_pivots 0 or 1 and "
                                     "select_workgroups <= 1");
    const bool one_pivot_form = o.update_grid_stride > 0 || o.update_hints != 0 || o.select_workgroups > 1 ||
                                o.rows_per_thread > 1 || o.cols_per_block > 8 || o.update_block > 256 ||
                                o.bland_after > 0;
    // Groups above kMaxFuseSplit pivots need the one-launch decision kernel
    // (at most kMaxDecideWgs workgroups over the rows and the list).
    const int32_t dblock = o.decide_block > 0 ? o.decide_block : 256;
    // (512-thread decision workgroups hold groups of at most 16; the grid
    // barriers need every decision workgroup resident at once)
    const int cus = device_cu_count(o.device);
    auto one_launch = [&](int K) {
        const int32_t g = decide_workgroups_for(m, (int64_t)n + 1 + K, dblock);
        return o.decide_kernel == 0 && g <= kMaxDecideWgs && (dblock == 256 || K <= kMaxFuseSplit) &&
               (int64_t)decide_blocks_per_cu(dblock, fused_update_kf(K)) * cus >= g;
    };
    if (o.fuse_pivots > 0) {
        h->fuse = o.fuse_pivots;
    } else {
        h->fuse = 1;
        if (!one_pivot_form) {  // kAutoFuse, else kMaxFuseSplit, where kernels exist for this shape
            const UpdateConfig u = pick_update_config(m, o.cols_per_block, o.rows_per_thread, o.update_block, true);
            for (int K : {kAutoFuse, kMaxFuseSplit}) {
                if ((K <= kMaxFuseSplit || one_launch(K)) &&
                    fused_update_supported(u.block, u.cols, u.rv, K, one_launch(K))) {
                    h->fuse = K;
                    break;
                }
            }
        }
    }
    h->ucfg = pick_update_config(m, o.cols_per_block, o.rows_per_thread, o.update_block, h->fuse > 1);
    if (h->ucfg.block == 256) h->ucfg.nt = o.update_hints & 3;
    if (o.update_grid_stride > 0) {  // grid-stride kernel: one column, one pair per thread per tile
        h->ucfg.cols = 1;
        h->ucfg.rv = 1;
        h->ucfg.rowchunks = (int)((((int64_t)m + 2) / 2 + h->ucfg.block - 1) / h->ucfg.block);
        h->ucfg.gs_per_cu = o.update_grid_stride;
        h->ucfg.gs_unroll = o.update_unroll > 0 ? o.update_unroll : 4;
        h->ucfg.nt = 0;
    }
    if (h->ucfg.gs_per_cu > 0 && h->ucfg.block > 512)
        return set_error(LP_E_INVAL, "the grid-stride update kernel takes at most 512 threads per workgroup");
    // (the fused kernels' shapes are checked below)
    const bool big_block_ok = h->fuse > 1 || h->ucfg.block == 256 || (h->ucfg.cols <= 2 && h->ucfg.rv <= 2) ||
                              (h->ucfg.block <= 128 && h->ucfg.rv == 1 && h->ucfg.rowchunks == 1);
    if ((o.update_block > 0 && h->ucfg.block != o.update_block) || !big_block_ok)
        return set_error(LP_E_INVAL, "update_block needs m + 1 > 256, and values other than 256 need "
                                     "cols_per_block and rows_per_thread <= 2");
    if (h->fuse > kMaxFuseSplit && !one_launch(h->fuse))
        return set_error(LP_E_INVAL, "fuse_pivots above 16 needs the one-launch decision kernel (decide_kernel 0, "
                                     "decide_block 256 and at most 128 decision workgroups)");
    if (h->fuse > 1) {
        const UpdateConfig &u = h->ucfg;
        if (u.gs_per_cu > 0 || u.nt != 0 || o.select_workgroups > 1 ||
            !fused_update_supported(u.block, u.cols, u.rv, h->fuse, one_launch(h->fuse)))
            return set_error(LP_E_INVAL, "fuse_pivots > 1 needs update_block <= 256, cols_per_block <= 8, "
                                         "rows_per_thread 1, update_hints 0, update_grid_stride 0 and "
                                         "select_workgroups <= 1; above 16 pivots, update_block 256 and "
                                         "cols_per_block 2, 4 or 8");
    }
    h->Lg = h->fuse > 1 ? (int64_t)n + 1 + h->fuse : (int64_t)n + 2;
    h->nparts = (int)((h->Lg + h->ucfg.cols - 1) / h->ucfg.cols);
    h->nsparts = (int)((h->Lg + 255) / 256);
    h->cus = cus;
    if (h->fuse > 1)
        h->chunk = o.chunk_pivots > 0 ? (o.chunk_pivots + h->fuse - 1) / h->fuse : 1;
    else
        h->chunk = o.chunk_pivots > 0 ? o.chunk_pivots : 4;
    h->select_wgs = o.select_workgroups > 0 ? o.select_workgroups : 1;
    h->use_graph = o.plain_launches == 0;
    h->timing = o.time_kernels != 0;
    h->eager_build = o.eager_build != 0;
    h->bland_after = o.bland_after;
    if (o.status_readback == 2 && h->fuse <= 1)
        return set_error(LP_E_INVAL, "status_readback 2 needs pivot fusion (fuse_pivots > 1)");
    if (h->fuse > 1) {
        h->decide_block = dblock;
        const int32_t g = decide_workgroups_for(m, h->Lg, h->decide_block);
        h->decide_wgs = one_launch(h->fuse) ? g : 0;
        h->decide_spin = o.decide_spin > 0 ? (uint32_t)o.decide_spin : kDefaultDecideSpin;
        h->force_gate_close = o.decide_spin == -1 && h->decide_wgs > 0;
        const bool can_early = h->decide_wgs > 0 && h->chunk == 1;
        if (o.status_readback == 2 && !can_early)
            return set_error(LP_E_INVAL,
                             "status_readback 2 needs the one-launch decision kernel and one group per chunk");
        h->early_status = can_early && o.status_readback != 1;
    }
    return LP_OK;
}

// Lays out the context's device buffers (all but the tableau) in one block,
// in a fixed order, each on a 256-byte boundary. With base == nullptr it only
// measures; otherwise it points the context's buffers into the block. Returns
// the bytes the block needs. A new block must be zeroed before first use
// (k_zero_words): the barrier counters, the select ticket, the zero dump
// column, R's padding and the work counters start at zero and the kernels
// keep them so; everything else is written by the build.
size_t carve_aux(lp_ctx *h, unsigned char *base) {
    size_t off = 0;
    auto take = [&](auto **p, size_t bytes) {
        off = (off + 255) / 256 * 256;
        using T = std::remove_pointer_t<std::remove_reference_t<decltype(p)>>;
        *p = base ? reinterpret_cast<T>(base + off) : nullptr;
        off += bytes;
    };
    const int32_t m = h->m, n = h->n;
    // F and R hold the pivots of the update instance (fused_update_kf(K) >= K)
    const int kf = h->fuse > 1 ? fused_update_kf(h->fuse) : 1;
    take(&h->F, (size_t)kf * h->ld * sizeof(double));
    take(&h->parts, (size_t)h->nparts * sizeof(ArgMin));
    // the state block: the solver state, then the four work counters, so
    // that one copy reads both
    take(&h->st, kStateBlock);
    h->cols_done = base ? reinterpret_cast<unsigned long long *>(reinterpret_cast<unsigned char *>(h->st) + kCountersAt)
                        : nullptr;
    take(&h->basis, (size_t)m * sizeof(int32_t));
    if (h->log_cap) {
        take(&h->log_r, (size_t)h->log_cap * sizeof(int32_t));
        take(&h->log_q, (size_t)h->log_cap * sizeof(int32_t));
    } else {
        h->log_r = h->log_q = nullptr;
    }
    take(&h->out, ((size_t)n + m + 1) * sizeof(double));
    take(&h->rparts, 64 * sizeof(RatioPart));
    take(&h->ticket, sizeof(uint32_t));
    take(&h->xticket, sizeof(uint32_t));
    // the fused update reads the list and R of a whole slot group at once, so
    // both are padded past the last slot
    take(&h->cols, ((size_t)h->Lg + kMaxFuse) * sizeof(int32_t));
    take(&h->pos, ((size_t)n + m) * sizeof(int32_t));
    take(&h->Rl, ((size_t)kf * h->Lg + 64) * sizeof(double));  // (row-lane tiles read R of 64 slots past the list)
    take(&h->gpick, 4 * sizeof(int32_t));
    if (h->fuse > 1) {
        take(&h->gs, sizeof(GroupState));
        take(&h->D, (size_t)h->Lg * sizeof(double));
        const size_t nsp = std::max<size_t>((size_t)h->nsparts, (size_t)kMaxDecideWgs);
        take(&h->sparts, nsp * sizeof(SPart));
        take(&h->grparts, kMaxDecideWgs * sizeof(GRatio));
        take(&h->gsync, sizeof(GridSync));
        take(&h->dump, (size_t)h->ld * sizeof(double));
        take(&h->PV, (size_t)kf * h->Lg * sizeof(double));
    }
    return (off + 255) / 256 * 256;
}

// Zeroes a block of `bytes` (a multiple of 8) on the stream: a fill kernel,
// not hipMemsetAsync, so that the clear is an ordinary kernel node if the
// caller captures the stream.
int enqueue_zero(void *p, size_t bytes, hipStream_t stream) {
    const int64_t words = (int64_t)(bytes / sizeof(uint64_t));
    if (words <= 0) return LP_OK;
    const int64_t blocks = std::min<int64_t>((words + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)blocks), dim3(256), 0, stream, (uint64_t *)p, words);
    LP_HIP_CHECK(hipGetLastError());
    return LP_OK;
}

// Allocates everything except the inputs; the tableau is not built yet.
int alloc_ctx(lp_ctx **out, int32_t m, int32_t n, const lp_options *opt_in) {
    const Options o = resolve_options(opt_in);
    if (int rc = validate_opts(o)) return rc;
    int ndev = 0;
    LP_HIP_CHECK(hipGetDeviceCount(&ndev));
    if (o.device < 0 || o.device >= ndev) return set_error(LP_E_INVAL, "device ordinal out of range");

    lp_ctx *h = new (std::nothrow) lp_ctx;
    if (!h) return set_error(LP_E_NOMEM, "host allocation failed");
    h->device = o.device;
    DeviceGuard g(h->device);
    auto fail = [&](int rc) {
        free_ctx(h);
        return rc;
    };
    if (int rc = configure_ctx(h, m, n, o)) return fail(rc);
    auto dev_alloc = [&](void **p, size_t bytes) -> int {
        hipError_t e = hipMalloc(p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return set_error(e == hipErrorOutOfMemory ? LP_E_NOMEM : LP_E_DEVICE,
                             std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        return LP_OK;
    };

    if (o.stream) {
        h->stream = (hipStream_t)o.stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return fail(set_error(LP_E_DEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e)));
        h->own_stream = true;
    }
    const size_t tbytes = lp_tableau_bytes(m, n);
    if (o.device_buffer) {
        if (o.device_buffer_bytes < tbytes || ((uintptr_t)o.device_buffer & 255u))
            return fail(set_error(LP_E_INVAL, "device_buffer too small or not 256-byte aligned"));
        h->T = (double *)o.device_buffer;
    } else {
        if (int rc = dev_alloc((void **)&h->T, tbytes)) return fail(rc);
        h->own_T = true;
    }
    const size_t aux_bytes = carve_aux(h, nullptr);
    if (int rc = dev_alloc((void **)&h->aux, aux_bytes)) return fail(rc);
    carve_aux(h, h->aux);
    if (int rc = enqueue_zero(h->aux, aux_bytes, h->stream)) return fail(rc);
    {
        hipError_t e = hipHostMalloc((void **)&h->host_st, 3 * sizeof(DevState), hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void **)&h->host_cols, 4 * sizeof(unsigned long long), hipHostMallocDefault);
        if (e == hipSuccess)  // (mapped: the extraction after a read-back-2 solve writes it directly)
            e = hipHostMalloc((void **)&h->host_out, ((size_t)n + m + 1) * sizeof(double),
                              hipHostMallocMapped | hipHostMallocCoherent);
        if (e != hipSuccess) return fail(set_error(LP_E_NOMEM, "hipHostMalloc failed"));
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, h->device) != hipSuccess || khz <= 0)
            return fail(set_error(LP_E_DEVICE, "no device clock rate"));
        h->clock_khz = (double)khz;
    }
    if (hipEventCreate(&h->ev_start) != hipSuccess || hipEventCreate(&h->ev_stop) != hipSuccess ||
        hipEventCreateWithFlags(&h->ev_slot[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->ev_slot[1], hipEventDisableTiming) != hipSuccess)
        return fail(set_error(LP_E_DEVICE, "hipEventCreate failed"));
    if (h->timing) {
        for (int k = 0; k < 2; ++k) {
            h->ev_upd[k].assign(2 * (size_t)h->chunk, nullptr);
            for (auto &e : h->ev_upd[k])
                if (hipEventCreate(&e) != hipSuccess) return fail(set_error(LP_E_DEVICE, "hipEventCreate failed"));
            if (hipEventCreate(&h->ev_first[k]) != hipSuccess)
                return fail(set_error(LP_E_DEVICE, "hipEventCreate failed"));
        }
    }
    *out = h;
    return LP_OK;
}

// The whole tableau of Table I: structural columns, slack identity and (with
// `rhs`) the RHS column.
void enqueue_full_build(lp_ctx *h, const double *dA, const double *db, const double *dc, bool rhs = true) {
    const int32_t m = h->m, n = h->n;
    const int64_t ld = h->ld;
    dim3 gs((unsigned)((n + kBuildTile - 1) / kBuildTile), (unsigned)((ld + kBuildTile - 1) / kBuildTile));
    hipLaunchKernelGGL(k_build_struct, gs, dim3(256), 0, h->stream, h->T, ld, m, n, dA, dc);
    const int32_t ncols = rhs ? m + 1 : m;  // without the RHS, b is not read (and may be NULL)
    const int64_t nslack = (int64_t)ncols * (ld / 2);
    hipLaunchKernelGGL(k_build_slack, dim3((unsigned)((nslack + 255) / 256)), dim3(256), 0, h->stream, h->T, ld, m,
                       n, db, ncols);
}

// Initialization Step from device-resident inputs, on the context stream.
// Deferred (`defer`, with the one-launch decision kernel): only the RHS
// column and the solver state here; the first group reads the structural
// columns from A and c, and its update pass writes them.
// With dA == nullptr the tableau is built already and only the solver state
// is set up.
int enqueue_build(lp_ctx *h, const double *dA, const double *db, const double *dc, bool defer) {
    const int32_t m = h->m, n = h->n;
    const int64_t ld = h->ld;
    const bool built = dA == nullptr;
    defer = defer && !built && !h->eager_build && h->fuse > 1 && h->decide_wgs > 0;
    h->counters_cached = false;
    h->solution_cached = false;
    if (!defer && !built) enqueue_full_build(h, dA, db, dc);
    h->pending = defer;
    h->first_ran = false;
    h->lazy = defer;
    h->pend_A = defer ? dA : nullptr;
    h->pend_b = defer ? db : nullptr;
    h->pend_c = defer ? dc : nullptr;
    DevState init{};
    init.status = LP_RUNNING;
    init.go = 0;
    init.pivots = 0;
    init.stop_at = INT64_MAX;  // no budget: what lp_solve asks for
    init.max_pivots = h->max_pivots;
    init.log_cap = h->log_cap;
    init.eps_d = h->eps_d;
    init.eps_p = h->eps_p;
    init.fresh = 1;
    init.nparts = h->nparts;
    init.bar = n + m;
    init.force_r = init.force_q = -1;
    init.bland_after = h->bland_after;
    init.degen = 0;
    if (h->fuse > 1) {
        const int32_t kf = fused_update_kf(h->fuse);
        const int64_t ninit = std::max<int64_t>(std::max<int64_t>((int64_t)n + m, (int64_t)kf * ld), h->Lg + kMaxFuse);
        hipLaunchKernelGGL(k_ginit, dim3((unsigned)((ninit + 255) / 256)), dim3(256), 0, h->stream, h->st, init,
                           h->gs, h->basis, m, n, (int32_t)h->fuse, kf, h->F, ld, h->cols, h->pos, h->cols_done,
                           h->T, defer ? db : nullptr);
    } else {
        const int64_t ninit = std::max<int64_t>(std::max<int64_t>((int64_t)n + m, ld), 1);
        hipLaunchKernelGGL(k_init, dim3((unsigned)((ninit + 255) / 256)), dim3(256), 0, h->stream, h->st, init,
                           h->basis, m, n, h->F, ld, h->cols, h->pos, h->cols_done);
    }
    LP_HIP_CHECK(hipGetLastError());
    h->dev_stop_at = init.stop_at;
    h->pivots_host = 0;
    h->status_host = LP_RUNNING;
    h->ran = false;
    return LP_OK;
}

// Enqueues the update kernel; with events, the dispatch itself records them
// at its start and end (timing mode).
void launch_update(lp_ctx *h, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
    const UpdateConfig &u = h->ucfg;
    if (u.gs_per_cu > 0) {
        const dim3 ggrid((unsigned)(u.gs_per_cu * h->cus)), gblock((unsigned)u.block);
#define LP_GS(B, U)                                                                                        \
    if (u.block == B && u.gs_unroll == U) {                                                                \
        if (e0)                                                                                            \
            hipExtLaunchKernelGGL((k_update_gs<B, U>), ggrid, gblock, 0, h->stream, e0, e1, 0, h->T,       \
                                  h->ld, h->m, h->n, u.rowchunks, (const int32_t *)h->cols,                \
                                  (const double *)h->Rl, (const double *)h->F, (const DevState *)h->st,    \
                                  h->parts);                                                               \
        else                                                                                               \
            hipLaunchKernelGGL((k_update_gs<B, U>), ggrid, gblock, 0, h->stream, h->T, h->ld, h->m, h->n,  \
                               u.rowchunks, h->cols, h->Rl, h->F, h->st, h->parts);                        \
        return;                                                                                            \
    }
        LP_GS(64, 1) LP_GS(64, 2) LP_GS(64, 4) LP_GS(64, 8)
        LP_GS(128, 1) LP_GS(128, 2) LP_GS(128, 4) LP_GS(128, 8)
        LP_GS(256, 1) LP_GS(256, 2) LP_GS(256, 4) LP_GS(256, 8)
        LP_GS(512, 1) LP_GS(512, 2) LP_GS(512, 4) LP_GS(512, 8)
#undef LP_GS
        return;
    }
    const dim3 grid((unsigned)((int64_t)u.rowchunks * h->nparts)), block((unsigned)u.block);
#define LP_UPD(B, C, V, NL, NS)                                                                        \
    if (u.block == B && u.cols == C && u.rv == V && u.nt == (NL | (NS << 1))) {                        \
        if (e0)                                                                                        \
            hipExtLaunchKernelGGL((k_update<B, C, V, NL, NS>), grid, block, 0, h->stream, e0, e1, 0,   \
                                  h->T, h->ld, h->m, h->n, u.rowchunks, (const int32_t *)h->cols,      \
                                  (const double *)h->Rl, (const double *)h->F,                         \
                                  (const DevState *)h->st, h->parts);                                  \
        else                                                                                           \
            hipLaunchKernelGGL((k_update<B, C, V, NL, NS>), grid, block, 0, h->stream, h->T, h->ld,    \
                               h->m, h->n, u.rowchunks, h->cols, h->Rl, h->F, h->st, h->parts);        \
        return;                                                                                        \
    }
#define LP_UPD_V(C, V) LP_UPD(256, C, V, 0, 0) LP_UPD(256, C, V, 1, 0) LP_UPD(256, C, V, 0, 1) \
    LP_UPD(256, C, V, 1, 1)
#define LP_UPD_C(C) LP_UPD(64, C, 1, 0, 0) LP_UPD(128, C, 1, 0, 0) LP_UPD_V(C, 1) LP_UPD_V(C, 2) \
    LP_UPD_V(C, 4) LP_UPD_V(C, 8)
#define LP_UPD_B(B) LP_UPD(B, 1, 1, 0, 0) LP_UPD(B, 1, 2, 0, 0) LP_UPD(B, 2, 1, 0, 0) LP_UPD(B, 2, 2, 0, 0)
    LP_UPD_B(512)
    LP_UPD_B(1024)
    LP_UPD(64, 1, 2, 0, 0)
    LP_UPD(64, 2, 2, 0, 0)
    LP_UPD(64, 2, 1, 0, 0)
    LP_UPD(128, 1, 2, 0, 0)
    LP_UPD(128, 2, 2, 0, 0)
    LP_UPD(128, 2, 1, 0, 0)
    LP_UPD_C(1)
    LP_UPD_C(2)
    LP_UPD_C(4)
    LP_UPD_C(8)
    LP_UPD_C(16)
#undef LP_UPD_B
#undef LP_UPD_C
#undef LP_UPD_V
#undef LP_UPD
}

FusedArgs fused_args(lp_ctx *h) {
    FusedArgs a{};  // (pub NULL: the decision kernel copies nothing to the host)
    a.T = h->T;
    a.ld = h->ld;
    a.m = h->m;
    a.n = h->n;
    a.K = h->fuse;
    a.KF = fused_update_kf(h->fuse);
    a.dump = h->dump;
    a.PV = h->PV;
    a.rowchunks = (int32_t)(((int64_t)h->m + h->ucfg.block) / h->ucfg.block);  // one row per thread
    a.nsparts = h->nsparts;
    a.nparts = h->nparts;
    a.st = h->st;
    a.gs = h->gs;
    a.Fk = h->F;
    a.Rk = h->Rl;
    a.D = h->D;
    a.cols = h->cols;
    a.pos = h->pos;
    a.basis = h->basis;
    a.log_r = h->log_r;
    a.log_q = h->log_q;
    a.parts = h->parts;
    a.sparts = h->sparts;
    a.cols_done = h->cols_done;
    a.select_wgs = select_workgroups_for(h->m);
    a.rparts = h->grparts;
    a.ticket = h->ticket;
    a.decide_wgs = h->decide_wgs;
    a.decide_block = h->decide_block;
    a.gsync = h->gsync;
    a.decide_spin = h->decide_spin;
    a.gate_spin = std::max(h->decide_spin, kDefaultDecideSpin);
    return a;
}

// One group of pivot fusion: its decisions (one launch, or a select and a
// stage launch per pivot), then one update pass.
void enqueue_group(lp_ctx *h, hipEvent_t e0, hipEvent_t e1) {
    const FusedArgs a = fused_args(h);
    if (a.decide_wgs > 0) {
        launch_fused_decide(a, h->stream);
    } else {
        for (int j = 0; j < h->fuse; ++j) {
            launch_fused_select(a, j, h->stream);
            launch_fused_stage(a, j, h->stream);
        }
    }
    const UpdateConfig &u = h->ucfg;
    launch_fused_update(a, u.block, u.cols, u.rv, h->stream, e0, e1);
}

// The first group after a deferred build, launched directly (its kernels
// take the caller's A and c): the decisions, then the pass that writes the
// structural columns with the group's pivots applied.
int launch_first_group(lp_ctx *h) {
    const FusedArgs a = fused_args(h);
    launch_first_decide(a, h->pend_A, h->pend_c, h->stream);
    if (h->timing)
        launch_first_update(a, h->pend_A, h->pend_c, h->stream, h->ev_first[0], h->ev_first[1]);
    else
        launch_first_update(a, h->pend_A, h->pend_c, h->stream, nullptr, nullptr);
    LP_HIP_CHECK(hipGetLastError());
    return LP_OK;
}

// One chunk: `chunk` pivots of (select, stage, update), or `chunk` groups of
// pivot fusion, with event records around each update kernel in timing mode.
int enqueue_chunk(lp_ctx *h, int slot) {
    if (h->fuse > 1) {
        for (int k = 0; k < h->chunk; ++k) {
            if (h->timing)
                enqueue_group(h, h->ev_upd[slot][2 * k], h->ev_upd[slot][2 * k + 1]);
            else
                enqueue_group(h, nullptr, nullptr);
        }
        LP_HIP_CHECK(hipGetLastError());
        return LP_OK;
    }
    for (int k = 0; k < h->chunk; ++k) {
        if (h->select_wgs > 1)
            hipLaunchKernelGGL(k_select_mw, dim3((unsigned)h->select_wgs), dim3(1024), 0, h->stream, h->T, h->ld,
                               h->m, h->n, h->parts, h->st, h->F, h->basis, h->log_r, h->log_q, h->pos, h->rparts,
                               h->ticket);
        else
            hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, h->stream, h->T, h->ld, h->m, h->n, h->parts,
                               h->st, h->F, h->basis, h->log_r, h->log_q, h->pos);
        hipLaunchKernelGGL(k_stage, dim3((unsigned)(((int64_t)h->n + 2 + 255) / 256)), dim3(256), 0, h->stream, h->T,
                           h->ld, h->m, h->n, h->st, h->cols, h->pos, h->Rl, h->cols_done);
        if (h->timing)
            launch_update(h, h->ev_upd[slot][2 * k], h->ev_upd[slot][2 * k + 1]);
        else
            launch_update(h);
    }
    LP_HIP_CHECK(hipGetLastError());
    return LP_OK;
}

// Captures the two chunk graphs (kernel arguments are fixed per context).
// Timing mode launches directly instead: HIP cannot report elapsed time
// between events recorded by a graph.
int capture_graphs(lp_ctx *h) {
    if (!h->use_graph || h->timing) return LP_OK;
    LP_HIP_CHECK(hipStreamSynchronize(h->stream));
    for (int slot = 0; slot < 2; ++slot) {
        LP_HIP_CHECK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
        const int rc = enqueue_chunk(h, slot);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(h->stream, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return set_error(LP_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        h->graph[slot] = graph;
        LP_HIP_CHECK(hipGraphInstantiate(&h->gexec[slot], graph, nullptr, nullptr, 0));
    }
    return LP_OK;
}

int launch_chunk(lp_ctx *h, int slot) {
    if (!h->gexec[slot]) return enqueue_chunk(h, slot);
    LP_HIP_CHECK(hipGraphLaunch(h->gexec[slot], h->stream));
    return LP_OK;
}

// Adds the times of every update launch of a finished chunk: those that
// applied a pivot and the no-op ones queued after the solve ended.
int harvest_timing(lp_ctx *h, int slot, int64_t advanced) {
    if (!h->timing) return LP_OK;
    if (h->first_slot[slot]) {  // the first group of a deferred build: its own kernel, timed apart
        float ms = 0.f;
        LP_HIP_CHECK(hipEventElapsedTime(&ms, h->ev_first[0], h->ev_first[1]));
        h->first_ms += ms;
        return LP_OK;
    }
    for (int64_t k = 0; k < h->chunk; ++k) {
        float ms = 0.f;
        LP_HIP_CHECK(hipEventElapsedTime(&ms, h->ev_upd[slot][2 * k], h->ev_upd[slot][2 * k + 1]));
        h->update_ms += ms;
        h->update_launches += 1;
        // the chunk's launches run in order and only the first ones apply
        // pivots: one per pivot, or one per group of `fuse` pivots
        if (k < (advanced + h->fuse - 1) / h->fuse) {
            h->update_ms_applied += ms;
            h->applied_launches += 1;
        }
    }
    return LP_OK;
}

// Finalization into pinned host memory: x, y and the objective (k_extract_y,
// k_extract_x), copied on the stream.
int enqueue_extract(lp_ctx *h) {
    const int64_t ny = (int64_t)h->n + h->m + 1;
    hipLaunchKernelGGL(k_extract_y, dim3((unsigned)((ny + 255) / 256)), dim3(256), 0, h->stream, h->T, h->ld, h->m,
                       h->n, h->out, (int64_t)0, nullptr);
    hipLaunchKernelGGL(k_extract_x, dim3((unsigned)((h->m + 255) / 256)), dim3(256), 0, h->stream, h->T, h->ld, h->m,
                       h->n, (const int32_t *)h->basis, h->out, nullptr, nullptr, 0u);
    LP_HIP_CHECK(hipGetLastError());
    LP_HIP_CHECK(hipMemcpyAsync(h->host_out, h->out, (size_t)ny * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    return LP_OK;
}

// The pause point of the device state, written only when it changes.
void set_stop(lp_ctx *h, int64_t stop_at) {
    if (stop_at == h->dev_stop_at) return;
    hipLaunchKernelGGL(k_set_stop, dim3(1), dim3(1), 0, h->stream, h->st, stop_at);
    h->dev_stop_at = stop_at;
}

// Solver-state read-back right after each group's decisions: the next
// group is launched while the current group's update pass runs, so no group
// is queued after the solve ends.
// Waits until the decision kernel has published the state in `slot` with
// sequence `seq`: polls the mapped word for up to 20 ms, then waits for the
// stream (the kernel has then ended) and checks once more.
int wait_word(lp_ctx *h, const volatile uint32_t *w, uint32_t seq) {
    const auto t0 = std::chrono::steady_clock::now();
    for (uint32_t k = 0; *w != seq; ++k) {
        if ((k & 1023) == 1023 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(20)) {
            LP_HIP_CHECK(hipStreamSynchronize(h->stream));
            if (*w != seq) return set_error(LP_E_DEVICE, "a kernel's published result did not arrive");
            break;
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return LP_OK;
}

int wait_pub(lp_ctx *h, int slot, uint32_t seq) {
    return wait_word(h, reinterpret_cast<const volatile uint32_t *>(h->pub + slot * kPubStride + kStateBlock), seq);
}

int run_until_early(lp_ctx *h, int64_t stop_at) {
    if (!h->pub) {  // (taken on first use: one an ended context left, else a new one)
        h->pub = pub_take(h->device);
        if (!h->pub &&
            hipHostMalloc((void **)&h->pub, kPubBytes, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
            (void)hipGetLastError();
            h->pub = nullptr;
            return set_error(LP_E_NOMEM, "hipHostMalloc failed");
        }
        std::memset(h->pub, 0, kPubBytes);  // (no sequence word of an earlier context left)
    }
    // the device time of the solve is taken from the device clock, read by
    // the first decision kernel and by the extraction: events between the
    // kernels would each delay the next dispatch
    unsigned long long *marks = reinterpret_cast<unsigned long long *>(h->pub + kPubMarks);
    uint32_t *xseq_at = reinterpret_cast<uint32_t *>(h->pub + kPubMarks + 2 * sizeof(unsigned long long));
    int64_t last = h->pivots_host;  // pivots before the group being harvested
    set_stop(h, stop_at);
    int slot = 0;
    int64_t advanced = 0;  // pivots of the group in the other slot, harvested once its pass is done
    bool have_prev = false;
    for (;;) {
        // the group's decisions, which hand the state they leave to the host
        // (published to mapped memory by the kernel's last workgroup), then
        // its update pass (queued at once: the device never waits for the
        // host)
        FusedArgs a = fused_args(h);
        const uint32_t seq = ++h->pub_seq;
        unsigned char *blk = h->pub + slot * kPubStride;  // the state and the work counters
        a.pub = blk;
        a.pub_words = (int32_t)(kStateBlock / sizeof(uint64_t));
        a.pub_seq_at = reinterpret_cast<uint32_t *>(blk + kStateBlock);
        a.pub_seq = seq;
        a.t_mark = have_prev ? nullptr : marks;
        const bool first = h->pending;
        h->first_slot[slot] = first;
        if (first) {
            h->pending = false;
            h->first_ran = true;
            launch_first_decide(a, h->pend_A, h->pend_c, h->stream);
        } else {
            launch_fused_decide(a, h->stream);
        }
        if (first) {
            launch_first_update(a, h->pend_A, h->pend_c, h->stream, h->timing ? h->ev_first[0] : nullptr,
                                h->timing ? h->ev_first[1] : nullptr);
        } else {
            const UpdateConfig &u = h->ucfg;
            launch_fused_update(a, u.block, u.cols, u.rv, h->stream, h->timing ? h->ev_upd[slot][0] : nullptr,
                                h->timing ? h->ev_upd[slot][1] : nullptr);
        }
        LP_HIP_CHECK(hipGetLastError());
        if (int rc = wait_pub(h, slot, seq)) return rc;
        std::memcpy(&h->host_st[slot], blk, sizeof(DevState));
        const DevState s = h->host_st[slot];
        // the previous group's update pass ran before these decisions
        if (have_prev)
            if (int rc = harvest_timing(h, slot ^ 1, advanced)) return rc;
        advanced = s.pivots - last;
        last = s.pivots;
        have_prev = true;
        if (s.status != LP_RUNNING || s.pivots >= stop_at) break;
        slot ^= 1;
    }
    // Finalization straight into the mapped host buffer, which the host
    // reads once the extraction's last workgroup has stored the sequence
    // word. x is zeroed here, by the host, while the last update pass runs
    // (before the launches, so before any device write to it), and the
    // device writes y, the objective and the basic entries of x.
    {
        std::memset(h->host_out, 0, (size_t)h->n * sizeof(double));
        const int64_t ny = (int64_t)h->m + 1;
        const uint32_t xseq = ++h->pub_seq;
        hipLaunchKernelGGL(k_extract_y, dim3((unsigned)((ny + 255) / 256)), dim3(256), 0, h->stream, h->T, h->ld,
                           h->m, h->n, h->host_out, (int64_t)h->n, marks + 1);
        hipLaunchKernelGGL(k_extract_x, dim3((unsigned)((h->m + 255) / 256)), dim3(256), 0, h->stream, h->T, h->ld,
                           h->m, h->n, (const int32_t *)h->basis, h->host_out, h->xticket, xseq_at, xseq);
        LP_HIP_CHECK(hipGetLastError());
        if (int rc = wait_word(h, xseq_at, xseq)) return rc;
    }
    // the state and the work counters read after the last decisions are
    // final: only the decision kernels write them (not the update pass, the
    // pivot-row stores or the extraction)
    h->host_st[2] = h->host_st[slot];
    std::memcpy(h->host_cols, h->pub + slot * kPubStride + kCountersAt, 4 * sizeof(unsigned long long));
    const DevState s = h->host_st[2];
    h->counters_cached = true;
    h->solution_cached = true;
    if (int rc = harvest_timing(h, slot, advanced)) return rc;  // the last group
    h->pivots_host = s.pivots;
    h->status_host = s.status;
    const volatile unsigned long long *vm = marks;
    h->last_ms = (double)(vm[1] - vm[0]) / h->clock_khz;
    h->ran = true;
    return LP_OK;
}

// Runs pivots until the status leaves RUNNING or `stop_at` pivots are done.
// Chunks are pipelined two deep: chunk k+1 is queued before the status of
// chunk k is read back, so the device never waits for the host.
int run_until_once(lp_ctx *h, int64_t stop_at) {
    h->counters_cached = false;
    h->solution_cached = false;
    if (h->early_status) return run_until_early(h, stop_at);
    // the first chunk is the first group of a deferred build when one is pending
    auto launch = [h](int sl) -> int {
        h->first_slot[sl] = h->pending;
        if (h->pending) {
            h->pending = false;
            h->first_ran = true;
            return launch_first_group(h);
        }
        return launch_chunk(h, sl);
    };
    int64_t last = h->pivots_host;  // pivots before the chunk being harvested
    set_stop(h, stop_at);
    LP_HIP_CHECK(hipEventRecord(h->ev_start, h->stream));
    int slot = 0;
    if (int rc = launch(0)) return rc;
    LP_HIP_CHECK(hipMemcpyAsync(&h->host_st[0], h->st, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
    LP_HIP_CHECK(hipEventRecord(h->ev_slot[0], h->stream));
    for (;;) {
        const int next = slot ^ 1;
        if (int rc = launch(next)) return rc;
        LP_HIP_CHECK(hipMemcpyAsync(&h->host_st[next], h->st, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
        LP_HIP_CHECK(hipEventRecord(h->ev_slot[next], h->stream));
        LP_HIP_CHECK(hipEventSynchronize(h->ev_slot[slot]));
        const DevState s = h->host_st[slot];
        if (int rc = harvest_timing(h, slot, s.pivots - last)) return rc;
        last = s.pivots;
        if (s.status != LP_RUNNING || s.pivots >= stop_at) break;
        slot = next;
    }
    LP_HIP_CHECK(hipEventRecord(h->ev_stop, h->stream));
    // the solution, the final state and the work counters, read back with
    // the last sync
    if (int rc = enqueue_extract(h)) return rc;
    LP_HIP_CHECK(hipMemcpyAsync(&h->host_st[2], h->st, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
    LP_HIP_CHECK(hipMemcpyAsync(h->host_cols, h->cols_done, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                h->stream));
    LP_HIP_CHECK(hipStreamSynchronize(h->stream));
    const DevState s = h->host_st[2];
    h->counters_cached = true;
    h->solution_cached = true;
    if (int rc = harvest_timing(h, slot ^ 1, s.pivots - last)) return rc;  // the chunk queued last
    h->pivots_host = s.pivots;
    h->status_host = s.status;
    float ms = 0.f;
    LP_HIP_CHECK(hipEventElapsedTime(&ms, h->ev_start, h->ev_stop));
    h->last_ms = ms;
    h->ran = true;
    return LP_OK;
}

// Closes the gate of the first decision launch when the options ask for it
// (decide_spin -1, a host-forced test of the fallback below).
void maybe_close_gate(lp_ctx *h) {
    if (!h->force_gate_close || h->fuse <= 1 || h->decide_wgs <= 0) return;
    hipLaunchKernelGGL(k_gate_close, dim3(1), dim3(1), 0, h->stream, h->gsync);
    h->force_gate_close = false;
}

// The fallback after a decision launch whose check-in gate closed (its
// workgroups were not all resident at once, e.g. while other streams held
// the compute units): that launch wrote nothing and the update pass queued
// after it applied nothing, so the tableau is the one after the last whole
// group. The open group is closed, the basic columns a deferred build left
// unstored are stored (the barrier-free kernels read every column they
// select), and the solve goes on with two launches per pivot (no grid
// barrier) in groups of at most kMaxFuseSplit pivots: the same pivots and
// bits. *resumed is false (and the solve stays LP_STALLED) when the stall
// came from a wait after the gate, or when no barrier-free kernels exist for
// the context's update shape.
int recover_stall(lp_ctx *h, bool *resumed) {
    *resumed = false;
    if (h->fuse <= 1 || h->decide_wgs <= 0 || h->status_host != LP_STALLED) return LP_OK;
    int32_t how = 0;
    LP_HIP_CHECK(hipMemcpy(&how, &h->gs->stalled, sizeof(int32_t), hipMemcpyDeviceToHost));
    const int K2 = std::min(h->fuse, kMaxFuseSplit);
    const UpdateConfig &u = h->ucfg;
    if (how != kStallGate || !fused_update_supported(u.block, u.cols, u.rv, K2, false)) return LP_OK;
    if (h->lazy) {
        const int64_t nb = (int64_t)h->m * (h->ld / 2);
        hipLaunchKernelGGL(k_store_basic, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, h->stream, h->T, h->ld,
                           h->m, (const int32_t *)h->basis);
        h->lazy = false;
    }
    hipLaunchKernelGGL(k_grecover, dim3(1), dim3(1), 0, h->stream, h->st, h->gs, h->cols, h->pos, h->n);
    LP_HIP_CHECK(hipGetLastError());
    LP_HIP_CHECK(hipStreamSynchronize(h->stream));
    h->decide_wgs = 0;
    h->early_status = false;
    h->fuse = K2;
    h->Lg = (int64_t)h->n + 1 + K2;
    h->nparts = (int)((h->Lg + h->ucfg.cols - 1) / h->ucfg.cols);
    h->nsparts = (int)((h->Lg + 255) / 256);
    for (int k = 0; k < 2; ++k) {
        if (h->gexec[k]) (void)hipGraphExecDestroy(h->gexec[k]);
        if (h->graph[k]) (void)hipGraphDestroy(h->graph[k]);
        h->gexec[k] = nullptr;
        h->graph[k] = nullptr;
    }
    if (int rc = capture_graphs(h)) return rc;
    h->status_host = LP_RUNNING;
    if (h->host_st) h->host_st[2].status = LP_RUNNING;  // (the solve that allocates nothing has no pinned state)
    h->stall_fallbacks += 1;
    *resumed = true;
    return LP_OK;
}

// run_until_once, resumed on the barrier-free kernels after a closed gate.
int run_until(lp_ctx *h, int64_t stop_at) {
    DeviceGuard g(h->device);
    h->update_ms = 0.0;
    h->update_launches = 0;
    h->update_ms_applied = 0.0;
    h->applied_launches = 0;
    h->first_ms = 0.0;
    maybe_close_gate(h);
    double ms = 0.0;
    for (;;) {
        if (int rc = run_until_once(h, stop_at)) return rc;
        ms += h->last_ms;
        bool resumed = false;
        if (int rc = recover_stall(h, &resumed)) return rc;
        if (!resumed) break;
    }
    h->last_ms = ms;
    return LP_OK;
}

bool all_finite(const double *p, int64_t k) {
    for (int64_t i = 0; i < k; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// ---- the solve that allocates nothing (lp_solve_noalloc) ------------------

// Its work block: every device buffer of a context except the tableau, laid
// out by carve_aux. Each device holds its own copy for the life of the
// process. Host code never passes the symbol itself to a kernel or a copy:
// noalloc_block() looks up the device's copy with hipGetSymbolAddress, once
// per device with that device current, and every use goes through that
// address.
static __device__ __align__(256) unsigned char scratch[LP_NOALLOC_SCRATCH_BYTES];

constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
unsigned char *g_noalloc_ptr[kNoAllocDevices] = {};

int noalloc_block(int device, unsigned char **out) {
    if (device < 0 || device >= kNoAllocDevices) return set_error(LP_E_INVAL, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return set_error(LP_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_noalloc_ptr[device] = static_cast<unsigned char *>(ptr);
    }
    *out = g_noalloc_ptr[device];
    return LP_OK;
}

// The solve loop of lp_solve_noalloc: no events, no pinned memory, no
// graphs. With the one-launch decision kernel the state is read right after
// each group's decisions (the group's update pass is queued after the read),
// so nothing is queued after the end; otherwise after each chunk.
int run_noalloc(lp_ctx *h, DevState *fin) {
    DevState s{};
    maybe_close_gate(h);
    for (;;) {
        if (h->fuse > 1 && h->decide_wgs > 0) {
            const FusedArgs a = fused_args(h);
            const bool first = h->pending;
            if (first) {
                h->pending = false;
                h->first_ran = true;
                launch_first_decide(a, h->pend_A, h->pend_c, h->stream);
            } else {
                launch_fused_decide(a, h->stream);
            }
            LP_HIP_CHECK(hipGetLastError());
            LP_HIP_CHECK(hipMemcpyAsync(&s, h->st, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
            LP_HIP_CHECK(hipStreamSynchronize(h->stream));
            if (first) {
                launch_first_update(a, h->pend_A, h->pend_c, h->stream, nullptr, nullptr);
            } else {
                const UpdateConfig &u = h->ucfg;
                launch_fused_update(a, u.block, u.cols, u.rv, h->stream, nullptr, nullptr);
            }
            LP_HIP_CHECK(hipGetLastError());
        } else {
            if (int rc = enqueue_chunk(h, 0)) return rc;
            LP_HIP_CHECK(hipMemcpyAsync(&s, h->st, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
            LP_HIP_CHECK(hipStreamSynchronize(h->stream));
        }
        if (s.status == LP_STALLED) {  // a closed gate: on with the barrier-free kernels
            h->status_host = s.status;
            bool resumed = false;
            if (int rc = recover_stall(h, &resumed)) return rc;
            if (resumed) continue;
        }
        if (s.status != LP_RUNNING) break;
    }
    *fin = s;
    return LP_OK;
}

// The relative tolerance of the infeasibility test after Phase I.
constexpr double kFeasTol = 1e-9;

// Ends a general-form solve with `status` (set on the device and in the
// host's copy of the final state).
int general_finish(lp_ctx *h, int32_t status) {
    hipLaunchKernelGGL(k_set_status, dim3(1), dim3(1), 0, h->stream, h->st, status);
    LP_HIP_CHECK(hipGetLastError());
    LP_HIP_CHECK(hipStreamSynchronize(h->stream));
    h->host_st[2].status = status;
    h->status_host = status;
    h->gphase = 3;
    return LP_OK;
}

// Both phases of a general-form LP: Phase I with Steps 1-3 (columns and rows
// of the carried objective barred), the infeasibility test, the drive-out of
// the artificial variables still basic (forced pivots), then rows 0 and m
// trade places and Phase II runs with the artificial columns barred.
int run_general(lp_ctx *h) {
    if (h->gphase != 1) return LP_OK;  // solved already
    DeviceGuard g(h->device);
    const int32_t M = h->m, np = h->n, m = h->m_in;
    const int64_t ld = h->ld, W = h->W;
    if (int rc = run_until(h, INT64_MAX)) return rc;
    if (h->host_st[2].status != LP_OPTIMAL) {
        h->gphase = 3;
        return LP_OK;
    }
    double w = 0.0;
    LP_HIP_CHECK(hipMemcpy(&w, h->T + (W - 1) * ld, sizeof(double), hipMemcpyDeviceToHost));
    if (w != w) return general_finish(h, LP_NUMERICAL);
    if (w < -kFeasTol * h->feas_scale) return general_finish(h, LP_INFEASIBLE);
    // drive-out: rows 1..m in order whose basic variable is artificial
    const int32_t allowed = np + h->n_le;
    std::vector<int32_t> basis((size_t)M);
    LP_HIP_CHECK(hipMemcpy(basis.data(), h->basis, (size_t)M * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int32_t t = 1; t <= m; ++t) {
        if (basis[t - 1] < allowed) continue;
        int32_t j = -1;
        hipLaunchKernelGGL(k_find_driveout, dim3(1), dim3(256), 0, h->stream, h->T, ld, t, allowed, h->eps_p, h->gpick);
        LP_HIP_CHECK(hipGetLastError());
        LP_HIP_CHECK(hipMemcpyAsync(&j, h->gpick, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
        LP_HIP_CHECK(hipStreamSynchronize(h->stream));
        if (j < 0) continue;  // a redundant row: its artificial variable stays basic
        hipLaunchKernelGGL(k_set_force, dim3(1), dim3(1), 0, h->stream, h->st, t, j);
        hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, h->stream, h->T, ld, M, np, h->parts, h->st, h->F,
                           h->basis, h->log_r, h->log_q, h->pos);
        hipLaunchKernelGGL(k_stage, dim3((unsigned)(((int64_t)np + 2 + 255) / 256)), dim3(256), 0, h->stream, h->T,
                           ld, M, np, h->st, h->cols, h->pos, h->Rl, h->cols_done);
        launch_update(h);
        LP_HIP_CHECK(hipGetLastError());
        DevState s;
        LP_HIP_CHECK(hipMemcpyAsync(&s, h->st, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
        LP_HIP_CHECK(hipStreamSynchronize(h->stream));
        h->pivots_host = s.pivots;
        if (s.status != LP_RUNNING) {  // the cap
            h->host_st[2] = s;
            h->status_host = s.status;
            h->solution_cached = false;
            h->counters_cached = false;
            h->gphase = 3;
            return LP_OK;
        }
    }
    // Phase II: the carried objective becomes row 0
    hipLaunchKernelGGL(k_swap_rows, dim3((unsigned)((W + 255) / 256)), dim3(256), 0, h->stream, h->T, ld, W, 0, M);
    hipLaunchKernelGGL(k_set_bar, dim3(1), dim3(1), 0, h->stream, h->st, allowed);
    LP_HIP_CHECK(hipGetLastError());
    if (int rc = run_until(h, INT64_MAX)) return rc;
    h->gphase = 3;
    return LP_OK;
}

}  // namespace

extern "C" {

int lp_create_device(lp_ctx **out, int32_t m, int32_t n, const double *dA, const double *db, const double *dc,
                     const lp_options *opt) {
    if (!out) return set_error(LP_E_INVAL, "out is NULL");
    *out = nullptr;
    if (m < 1 || n < 1 || !dA || !db || !dc) return set_error(LP_E_INVAL, "m, n must be >= 1 and inputs non-NULL");
    lp_ctx *h = nullptr;
    if (int rc = alloc_ctx(&h, m, n, opt)) return rc;
    DeviceGuard g(h->device);
    if (int rc = enqueue_build(h, dA, db, dc, false)) {
        free_ctx(h);
        return rc;
    }
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        free_ctx(h);
        return set_error(LP_E_DEVICE, std::string("build: ") + hipGetErrorString(e));
    }
    if (int rc = capture_graphs(h)) {
        free_ctx(h);
        return rc;
    }
    *out = h;
    return LP_OK;
}

int lp_create(lp_ctx **out, int32_t m, int32_t n, const double *A, const double *b, const double *c,
              const lp_options *opt) {
    if (!out) return set_error(LP_E_INVAL, "out is NULL");
    *out = nullptr;
    if (m < 1 || n < 1 || !A || !b || !c) return set_error(LP_E_INVAL, "m, n must be >= 1 and inputs non-NULL");
    if (!all_finite(A, (int64_t)m * n) || !all_finite(b, m) || !all_finite(c, n))
        return set_error(LP_E_INVAL, "non-finite input");
    for (int32_t i = 0; i < m; ++i)
        if (b[i] < 0.0) return set_error(LP_E_NEG_RHS, "b has a negative entry: the slack basis is infeasible "
                                                   "(lp_create_general takes any sign of b)");
    lp_ctx *h = nullptr;
    if (int rc = alloc_ctx(&h, m, n, opt)) return rc;
    DeviceGuard g(h->device);
    double *stage = nullptr;
    const size_t na = (size_t)m * n, bytes = (na + m + n) * sizeof(double);
    hipError_t e = hipMalloc((void **)&stage, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_ctx(h);
        return set_error(LP_E_NOMEM, "hipMalloc (input staging) failed");
    }
    int rc = LP_OK;
    if (hipMemcpyAsync(stage, A, na * sizeof(double), hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(stage + na, b, (size_t)m * sizeof(double), hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(stage + na + m, c, (size_t)n * sizeof(double), hipMemcpyHostToDevice, h->stream) != hipSuccess)
        rc = set_error(LP_E_DEVICE, "input copy failed");
    if (!rc) rc = enqueue_build(h, stage, stage + na, stage + na + m, false);
    if (!rc && hipStreamSynchronize(h->stream) != hipSuccess) rc = set_error(LP_E_DEVICE, "build failed");
    (void)hipFree(stage);
    if (!rc) rc = capture_graphs(h);
    if (rc) {
        free_ctx(h);
        return rc;
    }
    *out = h;
    return LP_OK;
}

int lp_create_general(lp_ctx **out, int32_t m, int32_t n, const double *A, const double *b, const double *c,
                      const int32_t *sense, const lp_options *opt) {
    if (!out) return set_error(LP_E_INVAL, "out is NULL");
    *out = nullptr;
    if (m < 1 || n < 1 || !A || !b || !c || !sense)
        return set_error(LP_E_INVAL, "m, n must be >= 1 and inputs non-NULL");
    if (!all_finite(A, (int64_t)m * n) || !all_finite(b, m) || !all_finite(c, n))
        return set_error(LP_E_INVAL, "non-finite input");
    for (int32_t i = 0; i < m; ++i)
        if (sense[i] < LP_LE || sense[i] > LP_EQ) return set_error(LP_E_INVAL, "sense must be LP_LE, LP_GE or LP_EQ");
    const Options ro = resolve_options(opt);
    if (ro.fuse_pivots > 1 || ro.select_workgroups > 1 || ro.update_grid_stride > 0)
        return set_error(LP_E_INVAL, "the general form runs one pivot per pass: fuse_pivots must be 0 or 1, "
                                     "select_workgroups <= 1 and update_grid_stride 0");
    // normalised senses and the tableau order: <= rows, then >=, then =
    std::vector<int32_t> kind((size_t)m), perm, surplus;
    int32_t n_le = 0, n_ge = 0;
    for (int32_t i = 0; i < m; ++i) {
        int32_t k = sense[i];
        if (b[i] < 0.0 && k != LP_EQ) k = LP_LE + LP_GE - k;
        kind[i] = k;
        n_le += k == LP_LE;
        n_ge += k == LP_GE;
    }
    std::vector<double> sgn;
    for (int32_t want : {LP_LE, LP_GE, LP_EQ})
        for (int32_t i = 0; i < m; ++i)
            if (kind[i] == want) {
                perm.push_back(i);
                sgn.push_back(b[i] < 0.0 ? -1.0 : 1.0);
            }
    // the >= rows are tableau rows n_le+1 .. n_le+n_ge; their surplus columns n ..
    surplus.assign((size_t)m, -1);
    for (int32_t t = n_le; t < n_le + n_ge; ++t) surplus[t] = n + (t - n_le);
    const int32_t np = n + n_ge, M = m + 1;
    lp_options o = opt ? *opt : lp_options{};
    if (!opt) lp_options_default(&o);
    lp_tuning tun;
    if (o.tuning)
        tun = *o.tuning;
    else
        lp_tuning_default(&tun);
    tun.fuse_pivots = 1;
    o.tuning = &tun;
    lp_ctx *h = nullptr;
    if (int rc = alloc_ctx(&h, M, np, &o)) return rc;
    DeviceGuard g(h->device);
    h->general = true;
    h->m_in = m;
    h->n_in = n;
    h->n_le = n_le;
    h->perm = perm;
    h->sgn = sgn;
    h->gphase = 1;
    // inputs to the device: A, b, c, the signs; then the order and surplus maps
    const size_t nd = (size_t)m * n + m + n + m;
    void *stage = nullptr;
    hipError_t e = hipMalloc(&stage, nd * sizeof(double) + 2 * (size_t)m * sizeof(int32_t));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_ctx(h);
        return set_error(LP_E_NOMEM, "hipMalloc (input staging) failed");
    }
    double *dA = (double *)stage, *db = dA + (size_t)m * n, *dc = db + m, *dsg = dc + n;
    int32_t *dperm = (int32_t *)(dsg + m), *dsur = dperm + m;
    int rc = LP_OK;
    const int64_t ld = h->ld, W = h->W;
    if (hipMemcpyAsync(dA, A, (size_t)m * n * sizeof(double), hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(db, b, (size_t)m * sizeof(double), hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(dc, c, (size_t)n * sizeof(double), hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(dsg, sgn.data(), (size_t)m * sizeof(double), hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(dperm, perm.data(), (size_t)m * sizeof(int32_t), hipMemcpyHostToDevice, h->stream) !=
            hipSuccess ||
        hipMemcpyAsync(dsur, surplus.data(), (size_t)m * sizeof(int32_t), hipMemcpyHostToDevice, h->stream) !=
            hipSuccess)
        rc = set_error(LP_E_DEVICE, "input copy failed");
    if (!rc) {
        const int64_t total = ld * W;
        const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
        hipLaunchKernelGGL(k_build_general, dim3((unsigned)blocks), dim3(256), 0, h->stream, h->T, ld, M, np, n, dA,
                           db, dc, dperm, dsg, dsur);
        hipLaunchKernelGGL(k_phase1_row0, dim3((unsigned)((W + 255) / 256)), dim3(256), 0, h->stream, h->T, ld, W,
                           n_le + 1, m + 1, np + n_le, np + m);
        if (hipGetLastError() != hipSuccess) rc = set_error(LP_E_DEVICE, "build launch failed");
    }
    if (!rc) rc = enqueue_build(h, nullptr, nullptr, nullptr, false);  // the state for a built tableau
    if (!rc) {
        hipLaunchKernelGGL(k_set_bar, dim3(1), dim3(1), 0, h->stream, h->st, np + m);  // Phase I
        if (hipGetLastError() != hipSuccess) rc = set_error(LP_E_DEVICE, "launch failed");
    }
    double w0 = 0.0;
    if (!rc && (hipMemcpyAsync(&w0, h->T + (W - 1) * ld, sizeof(double), hipMemcpyDeviceToHost, h->stream) !=
                    hipSuccess ||
                hipStreamSynchronize(h->stream) != hipSuccess))
        rc = set_error(LP_E_DEVICE, "build failed");
    (void)hipFree(stage);
    // Phase I's objective starts at minus the artificial rows' b summed in row
    // order, so its negation is that sum exactly: the scale of the test
    h->feas_scale = std::max(1.0, -w0);
    if (!rc) rc = capture_graphs(h);
    if (rc) {
        free_ctx(h);
        return rc;
    }
    *out = h;
    return LP_OK;
}

int lp_reload_device(lp_ctx *h, const double *dA, const double *db, const double *dc) {
    if (!h || !dA || !db || !dc) return set_error(LP_E_INVAL, "NULL argument");
    if (h->general) return set_error(LP_E_INVAL, "lp_reload_device takes standard-form contexts only");
    DeviceGuard g(h->device);
    return enqueue_build(h, dA, db, dc, true);
}

int lp_solve(lp_ctx *h) {
    if (!h) return set_error(LP_E_INVAL, "NULL context");
    if (h->general) return run_general(h);
    return run_until(h, INT64_MAX);
}

int lp_step(lp_ctx *h, int64_t pivots) {
    if (!h || pivots < 0) return set_error(LP_E_INVAL, "NULL context or negative pivot budget");
    if (h->general) return set_error(LP_E_INVAL, "lp_step takes standard-form contexts only (use lp_solve)");
    DeviceGuard g(h->device);
    if (h->ran || h->pivots_host > 0) {
        DevState s;
        LP_HIP_CHECK(hipStreamSynchronize(h->stream));
        LP_HIP_CHECK(hipMemcpy(&s, h->st, sizeof(DevState), hipMemcpyDeviceToHost));
        h->pivots_host = s.pivots;
    }
    const int64_t stop = h->pivots_host > INT64_MAX - pivots ? INT64_MAX : h->pivots_host + pivots;
    return run_until(h, stop);
}

int lp_get_solution(const lp_ctx *hc, lp_result *res, double *x, double *y) {
    if (!hc) return set_error(LP_E_INVAL, "NULL context");
    if (!hc->ran) return set_error(LP_E_STATE, "no solve has run on this context");
    lp_ctx *h = const_cast<lp_ctx *>(hc);
    DeviceGuard g(h->device);
    const double *buf = h->host_out;
    DevState s;
    if (h->solution_cached) {  // extracted at the end of the last solve, nothing has run since
        s = h->host_st[2];
    } else {
        if (int rc = enqueue_extract(h)) return rc;
        LP_HIP_CHECK(hipMemcpyAsync(&h->host_st[0], h->st, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
        LP_HIP_CHECK(hipStreamSynchronize(h->stream));
        s = h->host_st[0];
    }
    if (h->general) {  // the caller's variables, and its rows' duals with their signs
        if (x) std::memcpy(x, buf, (size_t)h->n_in * sizeof(double));
        if (y)
            for (int32_t t = 0; t < h->m_in; ++t) {
                const double v = buf[(size_t)h->n + t];
                y[h->perm[t]] = h->sgn[t] == 1.0 ? v : -v;
            }
    } else {
        if (x) std::memcpy(x, buf, (size_t)h->n * sizeof(double));
        if (y) std::memcpy(y, buf + h->n, (size_t)h->m * sizeof(double));
    }
    if (res) {
        res->status = s.status;
        res->reserved = 0;
        res->pivots = s.pivots;
        res->objective = buf[(size_t)h->n + h->m];
        res->solve_ms = h->last_ms;
    }
    return LP_OK;
}

int lp_get_pivots(const lp_ctx *h, int32_t *rows, int32_t *cols, int64_t cap, int64_t *count) {
    if (!h || cap < 0 || (cap > 0 && (!rows || !cols))) return set_error(LP_E_INVAL, "bad argument");
    DeviceGuard g(h->device);
    DevState s;
    LP_HIP_CHECK(hipStreamSynchronize(h->stream));
    LP_HIP_CHECK(hipMemcpy(&s, h->st, sizeof(DevState), hipMemcpyDeviceToHost));
    if (count) *count = s.pivots;
    const int64_t k = std::min<int64_t>(std::min<int64_t>(s.pivots, h->log_cap), cap);
    if (k > 0) {
        LP_HIP_CHECK(hipMemcpy(rows, h->log_r, (size_t)k * sizeof(int32_t), hipMemcpyDeviceToHost));
        LP_HIP_CHECK(hipMemcpy(cols, h->log_q, (size_t)k * sizeof(int32_t), hipMemcpyDeviceToHost));
    }
    return LP_OK;
}

int lp_get_tableau(const lp_ctx *hc, double *out) {
    if (!hc || !out) return set_error(LP_E_INVAL, "NULL argument");
    lp_ctx *h = const_cast<lp_ctx *>(hc);
    DeviceGuard g(h->device);
    if (h->pending) {  // a deferred build nothing has run yet: build it now (b is already in the RHS)
        enqueue_full_build(h, h->pend_A, nullptr, h->pend_c, false);
        h->pending = false;
        h->lazy = false;
    } else if (h->lazy) {  // store the basic columns that were never stored
        const int64_t nb = (int64_t)h->m * (h->ld / 2);
        hipLaunchKernelGGL(k_store_basic, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, h->stream, h->T, h->ld,
                           h->m, (const int32_t *)h->basis);
        h->lazy = false;
    }
    LP_HIP_CHECK(hipGetLastError());
    LP_HIP_CHECK(hipStreamSynchronize(h->stream));
    LP_HIP_CHECK(hipMemcpy2D(out, (size_t)(h->m + 1) * sizeof(double), h->T, (size_t)h->ld * sizeof(double),
                             (size_t)(h->m + 1) * sizeof(double), (size_t)h->W, hipMemcpyDeviceToHost));
    return LP_OK;
}

int lp_get_basis(const lp_ctx *h, int32_t *basis) {
    if (!h || !basis) return set_error(LP_E_INVAL, "NULL argument");
    DeviceGuard g(h->device);
    LP_HIP_CHECK(hipStreamSynchronize(h->stream));
    LP_HIP_CHECK(hipMemcpy(basis, h->basis, (size_t)h->m * sizeof(int32_t), hipMemcpyDeviceToHost));
    return LP_OK;
}

int lp_get_info(const lp_ctx *h, lp_info *info) {
    if (!h || !info) return set_error(LP_E_INVAL, "NULL argument");
    info->m = h->m;
    info->n = h->n;
    info->width = h->W;
    info->ld = h->ld;
    info->tableau_bytes = lp_tableau_bytes(h->m, h->n);
    info->tableau = h->T;
    info->update_block = h->ucfg.block;
    info->update_cols = h->ucfg.cols;
    info->update_rows = h->ucfg.rv;
    info->update_hints = h->ucfg.nt;
    info->update_fuse = h->fuse;
    info->decide_workgroups = h->fuse > 1 ? h->decide_wgs : 0;
    info->status_readback = h->early_status ? 2 : 1;
    return LP_OK;
}

int lp_get_timing(const lp_ctx *h, lp_timing *t) {
    if (!h || !t) return set_error(LP_E_INVAL, "NULL argument");
    DeviceGuard g(h->device);
    unsigned long long cols[4] = {0, 0, 0, 0};
    DevState s;
    if (h->counters_cached) {  // nothing has run since the last solve read them back
        std::memcpy(cols, h->host_cols, sizeof(cols));
        s = h->host_st[2];
    } else {
        LP_HIP_CHECK(hipStreamSynchronize(h->stream));
        LP_HIP_CHECK(hipMemcpy(cols, h->cols_done, sizeof(cols), hipMemcpyDeviceToHost));
        LP_HIP_CHECK(hipMemcpy(&s, h->st, sizeof(DevState), hipMemcpyDeviceToHost));
    }
    t->solve_ms = h->last_ms;
    t->update_ms = h->update_ms;
    t->update_launches = h->update_launches;
    t->update_ms_applied = h->update_ms_applied;
    t->applied_launches = h->applied_launches;
    t->pivots = s.pivots;
    t->updated_columns = (int64_t)cols[0];
    t->first_pass_ms = h->first_ms;
    t->first_pass_pivots = (int64_t)cols[2];
    t->first_pass_changed = (int64_t)cols[1];
    t->first_pass_columns = h->first_ran ? (int64_t)h->n + 1 + (int64_t)cols[3] : 0;
    return LP_OK;
}

void lp_destroy(lp_ctx *h) { free_ctx(h); }

int lp_solve_noalloc(int32_t m, int32_t n, const double *dA, const double *db, const double *dc, double *tableau,
                     size_t tableau_bytes, const lp_options *opt, lp_result *res, double *x, double *y,
                     int32_t *rows, int32_t *cols, int64_t cap, int64_t *count) {
    if (m < 1 || n < 1) return set_error(LP_E_INVAL, "m, n must be >= 1");
    if (cap < 0 || (cap > 0 && (!rows || !cols))) return set_error(LP_E_INVAL, "bad pivot-log arguments");
    const Options o = resolve_options(opt);
    if (int rc = validate_opts(o)) return rc;
    if (o.time_kernels) return set_error(LP_E_INVAL, "lp_solve_noalloc does not time kernels (time_kernels must be 0)");
    int ndev = 0;
    LP_HIP_CHECK(hipGetDeviceCount(&ndev));
    if (o.device < 0 || o.device >= ndev) return set_error(LP_E_INVAL, "device ordinal out of range");
    lp_ctx h;  // host fields only; its device buffers are carved from the work block
    if (int rc = configure_ctx(&h, m, n, o)) return rc;
    h.log_cap = o.record_pivots ? std::min<int64_t>(h.max_pivots, 4 * ((int64_t)m + n) + 64) : 0;
    const size_t need = carve_aux(&h, nullptr);
    if (need > (size_t)LP_NOALLOC_SCRATCH_BYTES)
        return set_error(LP_E_INVAL, "LP too large for lp_solve_noalloc: its work block needs " +
                                         std::to_string(need) + " bytes, the limit is " +
                                         std::to_string((size_t)LP_NOALLOC_SCRATCH_BYTES));
    if (!dA || !db || !dc || !tableau) return set_error(LP_E_INVAL, "NULL input or tableau");
    if (tableau_bytes < lp_tableau_bytes(m, n) || ((uintptr_t)tableau & 255u))
        return set_error(LP_E_INVAL, "tableau buffer too small or not 256-byte aligned");
    DeviceGuard g(h.device);
    unsigned char *block = nullptr;
    if (int rc = noalloc_block(h.device, &block)) return rc;
    carve_aux(&h, block);
    h.T = tableau;
    h.stream = (hipStream_t)o.stream;
    h.use_graph = false;
    if (int rc = enqueue_zero(block, need, h.stream)) return rc;
    if (int rc = enqueue_build(&h, dA, db, dc, true)) return rc;
    const auto t0 = std::chrono::steady_clock::now();
    DevState s{};
    if (int rc = run_noalloc(&h, &s)) return rc;
    // Finalization: x, y and the objective straight into the caller's arrays
    const int64_t ny = (int64_t)n + m + 1;
    hipLaunchKernelGGL(k_extract_y, dim3((unsigned)((ny + 255) / 256)), dim3(256), 0, h.stream, h.T, h.ld, m, n,
                       h.out, (int64_t)0, nullptr);
    hipLaunchKernelGGL(k_extract_x, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, h.stream, h.T, h.ld, m, n,
                       (const int32_t *)h.basis, h.out, nullptr, nullptr, 0u);
    LP_HIP_CHECK(hipGetLastError());
    double objective = 0.0;
    if (x) LP_HIP_CHECK(hipMemcpyAsync(x, h.out, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, h.stream));
    if (y) LP_HIP_CHECK(hipMemcpyAsync(y, h.out + n, (size_t)m * sizeof(double), hipMemcpyDeviceToHost, h.stream));
    LP_HIP_CHECK(hipMemcpyAsync(&objective, h.out + n + m, sizeof(double), hipMemcpyDeviceToHost, h.stream));
    const int64_t k = std::min<int64_t>(std::min<int64_t>(s.pivots, h.log_cap), cap);
    if (k > 0) {
        LP_HIP_CHECK(hipMemcpyAsync(rows, h.log_r, (size_t)k * sizeof(int32_t), hipMemcpyDeviceToHost, h.stream));
        LP_HIP_CHECK(hipMemcpyAsync(cols, h.log_q, (size_t)k * sizeof(int32_t), hipMemcpyDeviceToHost, h.stream));
    }
    LP_HIP_CHECK(hipStreamSynchronize(h.stream));
    if (count) *count = s.pivots;
    if (res) {
        res->status = s.status;
        res->reserved = 0;
        res->pivots = s.pivots;
        res->objective = objective;
        res->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return LP_OK;
}

}  // extern "C"

// ---- the server's lane of large LPs ----------------------------------------

namespace lpgpu {

struct Lane {
    lp_ctx *h = nullptr;
    Options o{};
    int32_t max_m = 0, max_n = 0;
};

namespace {

// The lane's options: pivot fusion in groups of 16 with the per-pivot
// decision kernels (k_gselect / k_gstage, no grid barrier), plain launches.
Options lane_options(Options o, hipStream_t stream, int fuse) {
    o.decide_kernel = 1;
    o.fuse_pivots = fuse;
    o.plain_launches = 1;
    o.time_kernels = 0;
    o.status_readback = 1;
    o.chunk_pivots = 0;
    o.eager_build = 0;
    o.device_buffer = nullptr;
    o.device_buffer_bytes = 0;
    o.stream = stream;
    return o;
}

// Configures a context for an m x n LP of the lane: groups of 16, or one
// pivot per pass where the fused kernels have no instance for the shape.
int lane_configure(const Options &base, lp_ctx *h, int32_t m, int32_t n) {
    const int64_t cap = base.record_pivots ? 4 * ((int64_t)m + n) + 64 : 0;
    for (int fuse : {kMaxFuseSplit, 1}) {
        const Options o = lane_options(base, h->stream, fuse);
        if (validate_opts(o) == LP_OK && configure_ctx(h, m, n, o) == LP_OK) {
            h->log_cap = std::min<int64_t>(h->max_pivots, cap);
            h->use_graph = false;
            h->timing = false;
            return LP_OK;
        }
    }
    return set_error(LP_E_INVAL, "no lane configuration for this LP shape");
}

}  // namespace

int lane_create(Lane **out, int device, hipStream_t stream, const Options &opt, int32_t max_m, int32_t max_n) {
    *out = nullptr;
    Lane *L = new (std::nothrow) Lane;
    if (!L) return set_error(LP_E_NOMEM, "host allocation failed");
    L->h = new (std::nothrow) lp_ctx;
    if (!L->h) {
        delete L;
        return set_error(LP_E_NOMEM, "host allocation failed");
    }
    L->o = opt;
    L->max_m = max_m;
    L->max_n = max_n;
    lp_ctx *h = L->h;
    h->device = device;
    h->stream = stream;
    h->own_stream = false;
    DeviceGuard g(device);
    hipError_t e = hipHostMalloc((void **)&h->host_st, 3 * sizeof(DevState), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&h->host_cols, 4 * sizeof(unsigned long long), hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&h->host_out, ((size_t)max_n + max_m + 1) * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreate(&h->ev_start);
    if (e == hipSuccess) e = hipEventCreate(&h->ev_stop);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_slot[0], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_slot[1], hipEventDisableTiming);
    if (e != hipSuccess) {
        lane_destroy(L);
        return set_error(LP_E_NOMEM, std::string("lane resources: ") + hipGetErrorString(e));
    }
    *out = L;
    return LP_OK;
}

// (a context of its own: the lane's may be solving on another thread)
size_t lane_work_bytes(const Lane *L, int32_t m, int32_t n) {
    lp_ctx tmp;
    if (m > L->max_m || n > L->max_n || lane_configure(L->o, &tmp, m, n) != LP_OK) return 0;
    return carve_aux(&tmp, nullptr);
}

int64_t lane_log_cap(const Lane *L, int32_t m, int32_t n) {
    lp_ctx tmp;
    if (lane_configure(L->o, &tmp, m, n) != LP_OK) return 0;
    return tmp.log_cap;
}

int lane_solve(Lane *L, int32_t m, int32_t n, double *T, unsigned char *work, LaneResult *out) {
    if (m > L->max_m || n > L->max_n) return set_error(LP_E_INVAL, "LP larger than the lane");
    lp_ctx *h = L->h;
    DeviceGuard g(h->device);
    if (int rc = lane_configure(L->o, h, m, n)) return rc;
    const size_t bytes = carve_aux(h, nullptr);
    carve_aux(h, work);
    h->T = T;
    if (int rc = enqueue_zero(work, bytes, h->stream)) return rc;
    if (int rc = enqueue_build(h, nullptr, nullptr, nullptr, false)) return rc;
    if (int rc = run_until(h, INT64_MAX)) return rc;
    const DevState s = h->host_st[2];
    out->status = s.status;
    out->pivots = s.pivots;
    out->x.assign(h->host_out, h->host_out + n);
    out->y.assign(h->host_out + n, h->host_out + n + m);
    out->objective = h->host_out[(size_t)n + m];
    const int64_t k = std::min<int64_t>(s.pivots, h->log_cap);
    out->rows.resize((size_t)k);
    out->cols.resize((size_t)k);
    if (k > 0) {
        LP_HIP_CHECK(hipMemcpyAsync(out->rows.data(), h->log_r, (size_t)k * sizeof(int32_t), hipMemcpyDeviceToHost,
                                    h->stream));
        LP_HIP_CHECK(hipMemcpyAsync(out->cols.data(), h->log_q, (size_t)k * sizeof(int32_t), hipMemcpyDeviceToHost,
                                    h->stream));
        LP_HIP_CHECK(hipStreamSynchronize(h->stream));
    }
    return LP_OK;
}

void lane_destroy(Lane *L) {
    if (!L) return;
    if (L->h) {
        L->h->T = nullptr;  // the tableaux and work blocks belong to the caller
        L->h->own_T = false;
        L->h->aux = nullptr;
        free_ctx(L->h);
    }
    delete L;
}

}  // namespace lpgpu
