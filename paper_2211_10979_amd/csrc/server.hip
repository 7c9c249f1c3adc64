// lp_server_*: a request loop that keeps each admitted LP's tableau resident
// in device memory and advances all resident LPs together with the batched
// kernel (continuous batching).
//
// Threads:
//   admission  takes requests in arrival order; waits until a slot is free
//              and the LP's bytes fit the budget; carves its memory from the
//              arena, copies A, b, c to the device and builds the tableau on
//              the copy stream; then hands the LP to the scheduler (small
//              tableaux) or to the large-LP lane (the LP waits there,
//              resident, until a lane worker takes it);
//   scheduler  replays the captured graph {queue reset, persistent batched
//              kernel} over the resident slots, each LP at most `budget`
//              pivots per replay, reads back the states, harvests finished
//              LPs (solution and pivot log to the host) and frees their
//              memory and slot;
//   lane       each large-LP worker solves one resident LP at a time on its
//              own stream with the single-LP kernels (pivot fusion with the
//              per-pivot decision kernels), then frees its memory and slot.
// The graph reads LPs through the device descriptor table, so it stays valid
// while the resident set changes. Work of LPs admitted while a replay runs
// overlaps with it on the copy stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch_engine.hpp"
#include "lane.hpp"
#include "plain_kernels.hpp"

using namespace lpgpu;

namespace {

using Clock = std::chrono::steady_clock;

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

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit sub-allocator over device chunks that are allocated on demand and
// kept until the server ends (hipFree would synchronise the device).
class Arena {
  public:
    Arena(size_t chunk, size_t cap) : chunk_(chunk), cap_(cap) {}
    ~Arena() {
        for (auto &c : chunks_) (void)hipFree(c.base);
    }
    void *alloc(size_t bytes) {
        bytes = align_up(bytes);
        std::lock_guard<std::mutex> lock(mu_);
        for (auto &c : chunks_)
            if (void *p = take(c, bytes)) return p;
        const size_t sz = std::max(chunk_, bytes);
        if (total_ + sz > cap_) return nullptr;
        char *base = nullptr;
        if (hipMalloc((void **)&base, sz) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        total_ += sz;
        chunks_.push_back(Chunk{base, sz, {{0, sz}}});
        return take(chunks_.back(), bytes);
    }
    void release(void *p, size_t bytes) {
        bytes = align_up(bytes);
        std::lock_guard<std::mutex> lock(mu_);
        for (auto &c : chunks_) {
            char *q = (char *)p;
            if (q < c.base || q >= c.base + c.size) continue;
            size_t off = (size_t)(q - c.base);
            auto it = c.free.emplace(off, bytes).first;
            auto nx = std::next(it);
            if (nx != c.free.end() && it->first + it->second == nx->first) {
                it->second += nx->second;
                c.free.erase(nx);
            }
            if (it != c.free.begin()) {
                auto pv = std::prev(it);
                if (pv->first + pv->second == it->first) {
                    pv->second += it->second;
                    c.free.erase(it);
                }
            }
            return;
        }
    }
    size_t reserved() const { return total_; }

  private:
    struct Chunk {
        char *base;
        size_t size;
        std::map<size_t, size_t> free;  // offset -> length
    };
    void *take(Chunk &c, size_t bytes) {
        for (auto it = c.free.begin(); it != c.free.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, len = it->second;
            c.free.erase(it);
            if (len > bytes) c.free.emplace(off + bytes, len - bytes);
            return c.base + off;
        }
        return nullptr;
    }
    std::mutex mu_;
    std::vector<Chunk> chunks_;
    size_t chunk_, cap_, total_ = 0;
};

struct Request {
    uint64_t ticket = 0;
    int32_t m = 0, n = 0;
    bool large = false;  // solved in the large-LP lane
    std::vector<double> in;  // A (row-major), b, c
    Clock::time_point t_submit, t_done;
    bool done = false;
    int32_t status = LP_RUNNING;
    int64_t pivots = 0;
    double objective = 0.0;
    std::vector<double> x, y;
    std::vector<int32_t> rows, cols;
    // resident part
    int slot = -1;
    char *block = nullptr;
    size_t bytes = 0;
    BatchDesc desc{};
    double *out = nullptr;
};

// LPs whose tableau exceeds this go to the large-LP lane: one workgroup per
// LP would take milliseconds per pivot there, while the single-LP kernels
// spread each pivot over the whole GPU. The lane takes LPs up to the
// server's largest accepted size, 4096 x 4096.
constexpr int32_t kLaneMax = 4096;
constexpr size_t kLargeTableauBytes = (size_t)16 << 20;

// Device bytes of one resident LP: tableau, lists and logs, extraction
// output, and the global work area when F/R do not fit in LDS.
struct Layout {
    size_t tab, ints, out, scratch, staging, total;
    int64_t log_cap;
};

Layout layout_of(int32_t m, int32_t n, int64_t max_pivots, bool record, size_t lds_limit) {
    Layout L{};
    const int64_t ld = padded_ld(m), W = (int64_t)n + m + 1;
    L.log_cap = record ? std::min<int64_t>(max_pivots, 4 * ((int64_t)m + n) + 64) : 0;
    L.tab = align_up((size_t)(ld * W) * sizeof(double));
    L.ints = align_up((size_t)((int64_t)m + (n + 2) + ((int64_t)n + m) + 2 * L.log_cap) * sizeof(int32_t));
    L.out = align_up(((size_t)n + m + 1) * sizeof(double));
    L.scratch = batch_lds_bytes(m, n) <= lds_limit ? 0 : align_up(batch_lds_bytes(m, n));
    L.staging = align_up(((size_t)m * n + m + n) * sizeof(double));
    L.total = L.tab + L.ints + L.out + L.scratch;
    return L;
}

double percentile(std::vector<double> v, double p) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = p * (double)(v.size() - 1);
    const size_t lo = (size_t)std::floor(pos), hi = std::min(v.size() - 1, lo + 1);
    return v[lo] + (v[hi] - v[lo]) * (pos - (double)lo);
}

static __global__ void k_extract_one(BatchDesc d, double *out) {
    const int32_t m = d.m, n = d.n;
    const int64_t W = (int64_t)n + m + 1;
    for (int32_t j = threadIdx.x; j < n; j += blockDim.x) out[j] = 0.0;
    __syncthreads();
    for (int32_t i = 1 + threadIdx.x; i <= m; i += blockDim.x) {
        const int32_t bv = d.basis[i - 1];
        if (bv < n) out[bv] = d.T[(W - 1) * d.ld + i];
        out[n + i - 1] = d.T[((int64_t)n + i - 1) * d.ld];
    }
    if (threadIdx.x == 0) out[n + m] = d.T[(W - 1) * d.ld];
}

}  // namespace

struct lp_server {
    int device = 0;
    hipStream_t sched = nullptr;
    size_t budget = 0;
    int32_t max_slots = 0;
    Options opt{};
    BatchShape shape{};
    int grid = 0;
    size_t lds = 0;
    int64_t step_budget = 8;
    Arena *arena = nullptr;
    static constexpr int kAdmitters = 4;
    double *staging[kAdmitters] = {};  // device staging of one LP's A, b, c per admission worker
    hipStream_t copy_streams[kAdmitters] = {};
    size_t staging_bytes = 0;
    BatchDesc *desc = nullptr;
    BatchState *state = nullptr;
    int32_t *order = nullptr, *norder = nullptr, *head = nullptr;
    BatchState *st_pin = nullptr;
    int32_t *order_pin = nullptr;  // max_slots entries + count
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;

    std::mutex mu;
    std::condition_variable cv_admit, cv_ready, cv_done;
    std::deque<Request *> pending;
    std::unordered_map<uint64_t, Request *> reqs;
    std::vector<Request *> slots;
    std::vector<int> free_slots;
    std::deque<int> ready;
    uint64_t next_ticket = 1;
    size_t bytes_in_use = 0, peak = 0;
    int admitting = 0;
    bool stopping = false;
    int64_t submitted = 0, completed = 0, rejected = 0, ticks = 0;
    std::vector<double> lat_ms;
    int last_error = LP_OK;
    std::thread admit_thr[kAdmitters], sched_thr;
    // large-LP lane: resident LPs waiting for a worker, and the workers'
    // solvers (each on its own stream)
    static constexpr int kLargeWorkers = 2;
    std::deque<Request *> ready_large;
    int large_busy = 0;
    hipStream_t large_streams[kLargeWorkers] = {};
    Lane *lanes[kLargeWorkers] = {};
    std::thread large_thr[kLargeWorkers];
    int64_t large_done = 0;
};

namespace {

void server_fail(lp_server *s, int code) {
    std::lock_guard<std::mutex> lock(s->mu);
    if (!s->last_error) s->last_error = code;
}

// Device bytes of a request: the batched form's layout, or for the lane the
// tableau and the lane's work block.
size_t request_bytes(const lp_server *s, int32_t m, int32_t n, bool large) {
    const int64_t maxp = s->opt.max_pivots > 0 ? s->opt.max_pivots : 50 * ((int64_t)m + n);
    if (!large) return layout_of(m, n, maxp, s->opt.record_pivots != 0, s->lds).total;
    const size_t work = lane_work_bytes(s->lanes[0], m, n);
    if (work == 0) return 0;
    return align_up((size_t)(padded_ld(m) * ((int64_t)n + m + 1)) * sizeof(double)) + align_up(work);
}

// Fails a request that could not be admitted or built; its memory and slot
// are returned.
void fail_request(lp_server *s, Request *r) {
    if (r->block) s->arena->release(r->block, r->bytes);
    std::lock_guard<std::mutex> lock(s->mu);
    if (!s->last_error) s->last_error = LP_E_DEVICE;
    s->bytes_in_use -= r->bytes;
    s->free_slots.push_back(r->slot);
    r->slot = -1;
    r->block = nullptr;
    r->status = LP_NUMERICAL;
    r->x.assign(r->n, 0.0);
    r->y.assign(r->m, 0.0);
    r->t_done = Clock::now();
    r->done = true;
    s->completed++;
    s->admitting--;
    s->cv_done.notify_all();
    s->cv_admit.notify_all();
}

// Admission worker `w`: takes requests in arrival order (both lanes share
// one queue, so the budget admits LPs in the order they came), allocates,
// copies and builds; then hands the LP to the scheduler or to the lane. Each
// worker has its own copy stream and staging buffer, so their copies and
// builds overlap.
void admission_loop(lp_server *s, int w) {
    DeviceGuard g(s->device);
    hipStream_t copy = s->copy_streams[w];
    double *staging = s->staging[w];
    for (;;) {
        Request *r = nullptr;
        size_t need = 0;
        {
            std::unique_lock<std::mutex> lock(s->mu);
            s->cv_admit.wait(lock, [&] {
                return (s->stopping && s->pending.empty()) || (!s->pending.empty() && !s->free_slots.empty());
            });
            if (s->pending.empty()) return;  // stopping and drained
            r = s->pending.front();
            need = request_bytes(s, r->m, r->n, r->large);
            if (s->free_slots.empty() || s->bytes_in_use + need > s->budget) {
                // head of the queue waits for memory: admission stays in order
                s->cv_admit.wait_for(lock, std::chrono::milliseconds(2));
                continue;
            }
            s->pending.pop_front();
            r->slot = s->free_slots.back();
            s->free_slots.pop_back();
            s->bytes_in_use += need;
            s->peak = std::max(s->peak, s->bytes_in_use);
            s->admitting++;
        }
        char *block = (char *)s->arena->alloc(need);
        if (!block) {  // fragmentation or device full: retry after harvests
            std::lock_guard<std::mutex> lock(s->mu);
            s->bytes_in_use -= need;
            s->free_slots.push_back(r->slot);
            r->slot = -1;
            s->pending.push_front(r);
            s->admitting--;
            std::this_thread::sleep_for(std::chrono::milliseconds(1));
            continue;
        }
        r->block = block;
        r->bytes = need;
        const int32_t m = r->m, n = r->n;
        const int64_t ld = padded_ld(m);
        const double *A = staging, *bb = A + (int64_t)m * n, *c = bb + m;
        bool ok = hipMemcpyAsync(staging, r->in.data(), r->in.size() * sizeof(double), hipMemcpyHostToDevice,
                                 copy) == hipSuccess;
        dim3 gs((unsigned)((n + kBuildTile - 1) / kBuildTile), (unsigned)((ld + kBuildTile - 1) / kBuildTile));
        const int64_t nslack = (int64_t)(m + 1) * (ld / 2);
        if (r->large) {  // the tableau of Table I; the lane sets up the rest when it takes the LP
            hipLaunchKernelGGL(k_build_struct, gs, dim3(256), 0, copy, (double *)block, ld, m, n, A, c);
            hipLaunchKernelGGL(k_build_slack, dim3((unsigned)((nslack + 255) / 256)), dim3(256), 0, copy,
                               (double *)block, ld, m, n, bb, m + 1);
            ok = ok && hipGetLastError() == hipSuccess && hipStreamSynchronize(copy) == hipSuccess;
            std::vector<double>().swap(r->in);
            if (!ok) {
                fail_request(s, r);
                continue;
            }
            {
                std::lock_guard<std::mutex> lock(s->mu);
                s->admitting--;
                s->ready_large.push_back(r);
            }
            s->cv_admit.notify_all();  // the lane workers wait on this too
            continue;
        }
        const int64_t maxp = s->opt.max_pivots > 0 ? s->opt.max_pivots : 50 * ((int64_t)m + n);
        const Layout L = layout_of(m, n, maxp, s->opt.record_pivots != 0, s->lds);
        BatchDesc &d = r->desc;
        d.T = (double *)block;
        d.ld = ld;
        d.m = m;
        d.n = n;
        int32_t *ints = (int32_t *)(block + L.tab);
        d.basis = ints;
        d.cols = ints + m;
        d.pos = d.cols + n + 2;
        d.log_r = d.pos + n + m;
        d.log_q = d.log_r + L.log_cap;
        d.log_cap = L.log_cap;
        d.nvec = (m + 2) / 2;
        d.magic = nvec_magic(d.nvec);
        d.pad = 0;
        r->out = (double *)(block + L.tab + L.ints);
        d.scratch = L.scratch ? (double *)(block + L.tab + L.ints + L.out) : nullptr;
        BatchState init{};
        init.status = LP_RUNNING;
        init.max_pivots = maxp;
        init.eps_d = s->opt.eps_dual;
        init.eps_p = s->opt.eps_pivot;
        hipLaunchKernelGGL(k_build_struct, gs, dim3(256), 0, copy, d.T, d.ld, m, n, A, c);
        hipLaunchKernelGGL(k_build_slack, dim3((unsigned)((nslack + 255) / 256)), dim3(256), 0, copy, d.T, d.ld, m,
                           n, bb, m + 1);
        hipLaunchKernelGGL(k_batch_init_lp, dim3(16), dim3(256), 0, copy, d, s->state + r->slot, init);
        ok = ok && hipMemcpyAsync(s->desc + r->slot, &d, sizeof(BatchDesc), hipMemcpyHostToDevice, copy) ==
                       hipSuccess;
        ok = ok && hipGetLastError() == hipSuccess && hipStreamSynchronize(copy) == hipSuccess;
        std::vector<double>().swap(r->in);
        if (!ok) {
            fail_request(s, r);
            continue;
        }
        {
            std::lock_guard<std::mutex> lock(s->mu);
            s->admitting--;
            s->slots[r->slot] = r;
            s->ready.push_back(r->slot);
        }
        s->cv_ready.notify_one();
    }
}

// Copies finished LPs' results to the host and releases their memory.
void harvest(lp_server *s, const std::vector<int> &fin) {
    if (fin.empty()) return;
    std::vector<std::vector<double>> tmp(fin.size());
    for (size_t f = 0; f < fin.size(); ++f) {
        Request *r = s->slots[fin[f]];
        const BatchState &st = s->st_pin[fin[f]];
        hipLaunchKernelGGL(k_extract_one, dim3(1), dim3(256), 0, s->sched, r->desc, r->out);
        tmp[f].resize((size_t)r->n + r->m + 1);
        (void)hipMemcpyAsync(tmp[f].data(), r->out, tmp[f].size() * sizeof(double), hipMemcpyDeviceToHost, s->sched);
        const int64_t k = std::min<int64_t>(st.pivots, r->desc.log_cap);
        r->rows.resize((size_t)k);
        r->cols.resize((size_t)k);
        if (k > 0) {
            (void)hipMemcpyAsync(r->rows.data(), r->desc.log_r, (size_t)k * sizeof(int32_t), hipMemcpyDeviceToHost,
                                 s->sched);
            (void)hipMemcpyAsync(r->cols.data(), r->desc.log_q, (size_t)k * sizeof(int32_t), hipMemcpyDeviceToHost,
                                 s->sched);
        }
    }
    const bool ok = hipStreamSynchronize(s->sched) == hipSuccess;
    const auto now = Clock::now();
    for (size_t f = 0; f < fin.size(); ++f) {
        const int slot = fin[f];
        Request *r = s->slots[slot];
        const BatchState &st = s->st_pin[slot];
        r->x.assign(tmp[f].begin(), tmp[f].begin() + r->n);
        r->y.assign(tmp[f].begin() + r->n, tmp[f].begin() + r->n + r->m);
        r->objective = tmp[f][(size_t)r->n + r->m];
        r->status = ok ? st.status : LP_NUMERICAL;
        r->pivots = st.pivots;
        s->arena->release(r->block, r->bytes);
        std::lock_guard<std::mutex> lock(s->mu);
        if (!ok && !s->last_error) s->last_error = LP_E_DEVICE;
        r->t_done = now;
        s->bytes_in_use -= r->bytes;
        r->block = nullptr;
        s->slots[slot] = nullptr;
        s->free_slots.push_back(slot);
        r->slot = -1;
        r->done = true;
        s->completed++;
        s->lat_ms.push_back(std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count());
    }
    s->cv_admit.notify_all();
    s->cv_done.notify_all();
}


// ---- large-LP lane -------------------------------------------------------

// Lane worker `w`: takes resident large LPs in admission order and solves
// each on its own stream; harvests, frees the memory and the slot.
void large_loop(lp_server *s, int w) {
    DeviceGuard g(s->device);
    for (;;) {
        Request *r = nullptr;
        {
            std::unique_lock<std::mutex> lock(s->mu);
            s->cv_admit.wait(lock, [&] {
                return !s->ready_large.empty() || (s->stopping && s->pending.empty() && s->admitting == 0);
            });
            if (s->ready_large.empty()) return;  // stopping and drained
            r = s->ready_large.front();
            s->ready_large.pop_front();
            s->large_busy++;
        }
        const int32_t m = r->m, n = r->n;
        const size_t tab = align_up((size_t)(padded_ld(m) * ((int64_t)n + m + 1)) * sizeof(double));
        LaneResult out;
        const int rc = lane_solve(s->lanes[w], m, n, (double *)r->block, (unsigned char *)r->block + tab, &out);
        s->arena->release(r->block, r->bytes);
        const auto now = Clock::now();
        std::lock_guard<std::mutex> lock(s->mu);
        if (rc != LP_OK) {
            if (!s->last_error) s->last_error = rc;
            out.status = LP_NUMERICAL;
            out.x.assign(n, 0.0);
            out.y.assign(m, 0.0);
        }
        r->status = out.status;
        r->pivots = out.pivots;
        r->objective = out.objective;
        r->x.swap(out.x);
        r->y.swap(out.y);
        r->rows.swap(out.rows);
        r->cols.swap(out.cols);
        s->bytes_in_use -= r->bytes;
        r->block = nullptr;
        s->free_slots.push_back(r->slot);
        r->slot = -1;
        s->large_busy--;
        r->t_done = now;
        r->done = true;
        s->completed++;
        s->large_done++;
        s->lat_ms.push_back(std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count());
        s->cv_done.notify_all();
        s->cv_admit.notify_all();
    }
}

void scheduler_loop(lp_server *s) {
    DeviceGuard g(s->device);
    std::vector<int> active;
    for (;;) {
        {
            std::unique_lock<std::mutex> lock(s->mu);
            if (active.empty() && s->ready.empty())
                s->cv_ready.wait_for(lock, std::chrono::milliseconds(1), [&] {
                    return !s->ready.empty() || (s->stopping && s->pending.empty() && s->admitting == 0);
                });
            while (!s->ready.empty()) {
                const int slot = s->ready.front();
                s->ready.pop_front();
                active.push_back(slot);
            }
            if (active.empty()) {
                if (s->stopping && s->pending.empty() && s->admitting == 0 && s->ready.empty()) return;
                continue;
            }
        }
        // largest LP first
        std::sort(active.begin(), active.end(), [&](int a, int b) {
            const Request *ra = s->slots[a], *rb = s->slots[b];
            return (int64_t)ra->m * (ra->n + 2) > (int64_t)rb->m * (rb->n + 2);
        });
        const int32_t na = (int32_t)active.size();
        std::copy(active.begin(), active.end(), s->order_pin);
        s->order_pin[s->max_slots] = na;
        bool ok = hipMemcpyAsync(s->order, s->order_pin, (size_t)na * sizeof(int32_t), hipMemcpyHostToDevice,
                                 s->sched) == hipSuccess &&
                  hipMemcpyAsync(s->norder, s->order_pin + s->max_slots, sizeof(int32_t), hipMemcpyHostToDevice,
                                 s->sched) == hipSuccess &&
                  hipGraphLaunch(s->gexec, s->sched) == hipSuccess &&
                  hipMemcpyAsync(s->st_pin, s->state, (size_t)s->max_slots * sizeof(BatchState),
                                 hipMemcpyDeviceToHost, s->sched) == hipSuccess &&
                  hipStreamSynchronize(s->sched) == hipSuccess;
        if (!ok) {
            server_fail(s, LP_E_DEVICE);
            for (int slot : active) s->st_pin[slot].status = LP_NUMERICAL;
        }
        s->ticks++;
        std::vector<int> fin, keep;
        for (int slot : active) (s->st_pin[slot].status != LP_RUNNING ? fin : keep).push_back(slot);
        harvest(s, fin);
        active.swap(keep);
    }
}

void free_server(lp_server *s) {
    if (!s) return;
    DeviceGuard g(s->device);
    if (s->sched) (void)hipStreamSynchronize(s->sched);
    for (auto cs : s->copy_streams)
        if (cs) (void)hipStreamSynchronize(cs);
    if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    for (void *p : {(void *)s->desc, (void *)s->state, (void *)s->order, (void *)s->norder, (void *)s->head})
        if (p) (void)hipFree(p);
    for (auto p : s->staging)
        if (p) (void)hipFree(p);
    for (auto L : s->lanes) lane_destroy(L);
    for (auto cs : s->large_streams)
        if (cs) {
            (void)hipStreamSynchronize(cs);
            (void)hipStreamDestroy(cs);
        }
    if (s->st_pin) (void)hipHostFree(s->st_pin);
    if (s->order_pin) (void)hipHostFree(s->order_pin);
    delete s->arena;
    for (auto &kv : s->reqs) delete kv.second;
    if (s->sched) (void)hipStreamDestroy(s->sched);
    for (auto cs : s->copy_streams)
        if (cs) (void)hipStreamDestroy(cs);
    delete s;
}

}  // namespace

extern "C" {

int lp_server_create(lp_server **out, size_t hbm_budget_bytes, int32_t max_slots, const lp_options *opt_in) {
    if (!out) return set_error(LP_E_INVAL, "out is NULL");
    *out = nullptr;
    if (hbm_budget_bytes < ((size_t)1 << 20)) return set_error(LP_E_INVAL, "budget below 1 MiB");
    const Options o = resolve_options(opt_in);
    if (o.bland_after != 0) return set_error(LP_E_INVAL, "the server takes bland_after 0 only");
    if (!(o.eps_dual >= 0.0) || !(o.eps_pivot >= 0.0) || !std::isfinite(o.eps_dual) || !std::isfinite(o.eps_pivot))
        return set_error(LP_E_INVAL, "eps_dual and eps_pivot must be finite and >= 0");
    int ndev = 0;
    LP_HIP_CHECK(hipGetDeviceCount(&ndev));
    if (o.device < 0 || o.device >= ndev) return set_error(LP_E_INVAL, "device ordinal out of range");
    lp_server *s = new (std::nothrow) lp_server;
    if (!s) return set_error(LP_E_NOMEM, "host allocation failed");
    s->device = o.device;
    DeviceGuard g(s->device);
    auto fail = [&](int rc) {
        free_server(s);
        return rc;
    };
    s->opt = o;
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots > 0 ? max_slots : 4096;
    s->step_budget = o.chunk_pivots > 0 ? o.chunk_pivots : 8;
    s->lds = std::min<size_t>(device_lds_limit(o.device), 64 * 1024);
    s->arena = new Arena(std::min<size_t>((size_t)4 << 30, hbm_budget_bytes), hbm_budget_bytes + ((size_t)4 << 30));
    // staging for the largest LP the batched kernel accepts is sized lazily
    // per request below the 4096 x 4096 bound; start at 4096 x 4096
    s->staging_bytes = ((size_t)4096 * 4096 + 8192) * sizeof(double);
    auto dmalloc = [&](void **p, size_t bytes) -> int {
        if (hipMalloc(p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(LP_E_NOMEM, "hipMalloc failed");
        }
        return LP_OK;
    };
    for (auto &p : s->staging)
        if (int rc = dmalloc((void **)&p, s->staging_bytes)) return fail(rc);
    for (auto &cs : s->large_streams)
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
            return fail(set_error(LP_E_DEVICE, "hipStreamCreate failed"));
    for (int w = 0; w < lp_server::kLargeWorkers; ++w)
        if (int rc = lane_create(&s->lanes[w], s->device, s->large_streams[w], o, kLaneMax, kLaneMax))
            return fail(rc);
    if (int rc = dmalloc((void **)&s->desc, (size_t)s->max_slots * sizeof(BatchDesc))) return fail(rc);
    if (int rc = dmalloc((void **)&s->state, (size_t)s->max_slots * sizeof(BatchState))) return fail(rc);
    if (int rc = dmalloc((void **)&s->order, (size_t)s->max_slots * sizeof(int32_t))) return fail(rc);
    if (int rc = dmalloc((void **)&s->norder, sizeof(int32_t))) return fail(rc);
    if (int rc = dmalloc((void **)&s->head, sizeof(int32_t))) return fail(rc);
    if (hipHostMalloc((void **)&s->st_pin, (size_t)s->max_slots * sizeof(BatchState), hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void **)&s->order_pin, ((size_t)s->max_slots + 1) * sizeof(int32_t), hipHostMallocDefault) !=
            hipSuccess)
        return fail(set_error(LP_E_NOMEM, "hipHostMalloc failed"));
    std::memset(s->st_pin, 0, (size_t)s->max_slots * sizeof(BatchState));
    if (hipStreamCreateWithFlags(&s->sched, hipStreamNonBlocking) != hipSuccess)
        return fail(set_error(LP_E_DEVICE, "hipStreamCreate failed"));
    for (auto &cs : s->copy_streams)
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
            return fail(set_error(LP_E_DEVICE, "hipStreamCreate failed"));
    if (hipMemset(s->state, 0, (size_t)s->max_slots * sizeof(BatchState)) != hipSuccess)
        return fail(set_error(LP_E_DEVICE, "hipMemset failed"));
    if (int rc = set_batch_lds_limit(s->lds)) return fail(rc);
    s->shape = BatchShape{1024, 2, 1};
    if (o.batch_block > 0 || o.batch_unroll > 0) {
        bool found = false;
        for (int i = 0; i < kNumBatchShapes; ++i)
            if ((o.batch_block <= 0 || kBatchShapes[i].block == o.batch_block) &&
                (o.batch_unroll <= 0 || kBatchShapes[i].unroll == o.batch_unroll)) {
                s->shape = kBatchShapes[i];
                found = true;
                break;
            }
        if (!found) return fail(set_error(LP_E_INVAL, "no batch kernel shape with that block / unroll"));
    }
    s->shape.split = 1;  // the server's LPs come and go: none is split
    s->grid = std::max(1, s->shape.grid_per_cu * device_cus(o.device));
    // the captured graph: queue reset + persistent kernel over the order list
    if (hipStreamBeginCapture(s->sched, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(set_error(LP_E_DEVICE, "hipStreamBeginCapture failed"));
    int rc = launch_batch_kernel(s->shape, s->grid, s->lds, s->sched, s->desc, s->state, s->order, s->norder,
                                 s->head, s->step_budget);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(s->sched, &graph);
    if (rc) return fail(rc);
    if (e != hipSuccess) return fail(set_error(LP_E_DEVICE, "hipStreamEndCapture failed"));
    s->graph = graph;
    if (hipGraphInstantiate(&s->gexec, graph, nullptr, nullptr, 0) != hipSuccess)
        return fail(set_error(LP_E_DEVICE, "hipGraphInstantiate failed"));
    s->slots.assign((size_t)s->max_slots, nullptr);
    for (int i = s->max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
    for (int w = 0; w < lp_server::kAdmitters; ++w) s->admit_thr[w] = std::thread(admission_loop, s, w);
    for (int w = 0; w < lp_server::kLargeWorkers; ++w) s->large_thr[w] = std::thread(large_loop, s, w);
    s->sched_thr = std::thread(scheduler_loop, s);
    *out = s;
    return LP_OK;
}

int lp_server_submit(lp_server *s, int32_t m, int32_t n, const double *A, const double *b, const double *c,
                     uint64_t *ticket) {
    if (!s || !A || !b || !c || !ticket || m < 1 || n < 1) return set_error(LP_E_INVAL, "bad argument");
    if (m > 4096 || n > 4096 || !batch_fits(m, n, (size_t)1 << 40))
        return set_error(LP_E_INVAL, "the server accepts LPs up to 4096 x 4096");
    for (int64_t t = 0; t < (int64_t)m * n; ++t)
        if (!std::isfinite(A[t])) return set_error(LP_E_INVAL, "non-finite A");
    for (int32_t i = 0; i < m; ++i) {
        if (!std::isfinite(b[i])) return set_error(LP_E_INVAL, "non-finite b");
        if (b[i] < 0.0) return set_error(LP_E_NEG_RHS, "negative b");
    }
    for (int32_t j = 0; j < n; ++j)
        if (!std::isfinite(c[j])) return set_error(LP_E_INVAL, "non-finite c");
    const bool large = (size_t)(padded_ld(m) * ((int64_t)n + m + 1)) * sizeof(double) > kLargeTableauBytes;
    const size_t need = request_bytes(s, m, n, large);
    if (need == 0) return set_error(LP_E_INVAL, "no kernel configuration for this LP shape");
    if (need > s->budget) {
        std::lock_guard<std::mutex> lock(s->mu);
        s->rejected++;
        return set_error(LP_E_BUDGET, "LP larger than the server budget");
    }
    Request *r = new (std::nothrow) Request;
    if (!r) return set_error(LP_E_NOMEM, "host allocation failed");
    r->m = m;
    r->n = n;
    r->large = large;
    r->in.resize((size_t)m * n + m + n);
    std::memcpy(r->in.data(), A, (size_t)m * n * sizeof(double));
    std::memcpy(r->in.data() + (size_t)m * n, b, (size_t)m * sizeof(double));
    std::memcpy(r->in.data() + (size_t)m * n + m, c, (size_t)n * sizeof(double));
    {
        std::lock_guard<std::mutex> lock(s->mu);
        if (s->stopping) {
            delete r;
            return set_error(LP_E_STATE, "server is stopping");
        }
        r->ticket = s->next_ticket++;
        r->t_submit = Clock::now();
        s->reqs[r->ticket] = r;
        s->pending.push_back(r);
        s->submitted++;
    }
    s->cv_admit.notify_all();
    *ticket = r->ticket;
    return LP_OK;
}

static int collect(lp_server *s, Request *r, uint64_t ticket, lp_result *res, double *x, double *y) {
    if (x) std::memcpy(x, r->x.data(), (size_t)r->n * sizeof(double));
    if (y) std::memcpy(y, r->y.data(), (size_t)r->m * sizeof(double));
    if (res) {
        res->status = r->status;
        res->reserved = 0;
        res->pivots = r->pivots;
        res->objective = r->objective;
        res->solve_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    }
    s->reqs.erase(ticket);
    delete r;
    return LP_OK;
}

int lp_server_poll(lp_server *s, uint64_t ticket, lp_result *res, double *x, double *y) {
    if (!s) return set_error(LP_E_INVAL, "NULL server");
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return set_error(LP_E_INVAL, "unknown or collected ticket");
    if (!it->second->done) return LP_E_PENDING;
    return collect(s, it->second, ticket, res, x, y);
}

int lp_server_wait(lp_server *s, uint64_t ticket, lp_result *res, double *x, double *y) {
    if (!s) return set_error(LP_E_INVAL, "NULL server");
    std::unique_lock<std::mutex> lock(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return set_error(LP_E_INVAL, "unknown or collected ticket");
    Request *r = it->second;
    s->cv_done.wait(lock, [&] { return r->done; });
    return collect(s, r, ticket, res, x, y);
}

int lp_server_get_pivots(lp_server *s, uint64_t ticket, int32_t *rows, int32_t *cols, int64_t cap,
                         int64_t *count) {
    if (!s || cap < 0 || (cap > 0 && (!rows || !cols))) return set_error(LP_E_INVAL, "bad argument");
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return set_error(LP_E_INVAL, "unknown or collected ticket");
    Request *r = it->second;
    if (!r->done) return LP_E_PENDING;
    if (count) *count = r->pivots;
    const int64_t k = std::min<int64_t>((int64_t)r->rows.size(), cap);
    if (k > 0) {
        std::memcpy(rows, r->rows.data(), (size_t)k * sizeof(int32_t));
        std::memcpy(cols, r->cols.data(), (size_t)k * sizeof(int32_t));
    }
    return LP_OK;
}

int lp_server_stats(const lp_server *cs, struct lp_server_stats *st) {
    if (!cs || !st) return set_error(LP_E_INVAL, "NULL argument");
    lp_server *s = const_cast<lp_server *>(cs);  // only the lock is taken
    std::lock_guard<std::mutex> lock(s->mu);
    st->submitted = s->submitted;
    st->completed = s->completed;
    st->rejected = s->rejected;
    int64_t resident = 0;
    for (auto *r : s->slots) resident += r != nullptr;
    st->resident_now = resident + (int64_t)s->ready.size() + (int64_t)s->ready_large.size() + s->large_busy;
    st->bytes_in_use = s->bytes_in_use;
    st->peak_bytes = s->peak;
    st->ticks = s->ticks;
    st->p50_ms = percentile(s->lat_ms, 0.50);
    st->p99_ms = percentile(s->lat_ms, 0.99);
    double sum = 0.0;
    for (double v : s->lat_ms) sum += v;
    st->mean_ms = s->lat_ms.empty() ? 0.0 : sum / (double)s->lat_ms.size();
    if (s->last_error) return set_error(s->last_error, "a device operation of the server failed");
    return LP_OK;
}

int lp_server_get_stats(const lp_server *s, struct lp_server_stats *st) { return lp_server_stats(s, st); }

void lp_server_destroy(lp_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->stopping = true;
    }
    s->cv_admit.notify_all();
    s->cv_ready.notify_all();
    for (auto &t : s->admit_thr)
        if (t.joinable()) t.join();
    for (auto &t : s->large_thr)
        if (t.joinable()) t.join();
    if (s->sched_thr.joinable()) s->sched_thr.join();
    free_server(s);
}

}  // extern "C"
