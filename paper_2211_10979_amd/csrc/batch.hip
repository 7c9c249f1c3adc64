// Host side of the batched solver (lp_batch_*): one arena for every LP's
// tableau and lists, a captured graph {queue reset, persistent kernel}, and
// the autotuner that picks the persistent kernel's shape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "batch_engine.hpp"
#include "plain_kernels.hpp"

using namespace lpgpu;

namespace lpgpu {

// (the shapes that split large LPs come last: the server, which never
// splits, takes the first shape that matches its options)
const BatchShape kBatchShapes[] = {
    {256, 1, 2},     {256, 2, 2},     {256, 4, 2},     {256, 4, 4},     {256, 8, 2},     {512, 1, 1},
    {512, 2, 1},     {512, 2, 2},     {512, 4, 1},     {512, 4, 2},     {1024, 1, 1},    {1024, 2, 1},
    {1024, 4, 1},    {1024, 2, 2},    {256, 2, 2, 8},  {512, 2, 2, 4},  {512, 2, 2, 8},  {1024, 2, 1, 4},
    {1024, 2, 1, 8}, {1024, 4, 1, 4}, {1024, 4, 1, 8},
};
const int kNumBatchShapes = sizeof(kBatchShapes) / sizeof(kBatchShapes[0]);

size_t batch_lds_bytes(int32_t m, int32_t n) {
    const int64_t nvec = ((int64_t)m + 2) / 2;
    return (size_t)(16 * nvec + 12 * ((int64_t)n + 2));
}

bool batch_fits(int32_t m, int32_t n, size_t lds_limit) {
    return batch_size_ok(m, n) && batch_lds_bytes(m, n) <= lds_limit;
}

bool batch_size_ok(int32_t m, int32_t n) {
    const int64_t nvec = ((int64_t)m + 2) / 2;
    return nvec < 4096 && ((int64_t)n + 2) * nvec < (int64_t)1 << 24;
}

uint64_t nvec_magic(int32_t nvec) { return (((uint64_t)1 << 36) + (uint64_t)nvec - 1) / (uint64_t)nvec; }

int launch_batch_kernel(const BatchShape &sh, int grid, size_t lds, hipStream_t stream, const BatchDesc *desc,
                        BatchState *state, const int32_t *order, const int32_t *norder, int32_t *head,
                        int64_t budget, const int32_t *parts, uint32_t gate_spin) {
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, stream, head);
#define LP_BATCH(B, U)                                                                                          \
    if (sh.block == B && sh.unroll == U) {                                                                      \
        hipLaunchKernelGGL((k_batch<B, U>), dim3((unsigned)grid), dim3(B), lds, stream, desc, state, order,     \
                           norder, head, budget, parts, gate_spin);                                             \
        return LP_OK;                                                                                           \
    }
    LP_BATCH(256, 1)
    LP_BATCH(256, 2)
    LP_BATCH(256, 4)
    LP_BATCH(256, 8)
    LP_BATCH(512, 1)
    LP_BATCH(512, 2)
    LP_BATCH(512, 4)
    LP_BATCH(1024, 1)
    LP_BATCH(1024, 2)
    LP_BATCH(1024, 4)
#undef LP_BATCH
    return set_error(LP_E_INVAL, "unsupported batch kernel shape");
}

int batch_blocks_per_cu(const BatchShape &sh, size_t lds) {
    int blocks = 0;
#define LP_OCC(B, U)                                                                                          \
    if (sh.block == B && sh.unroll == U &&                                                                    \
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void *>(&k_batch<B, U>), B, \
                                                     lds) == hipSuccess)                                     \
        return blocks;
    LP_OCC(256, 1)
    LP_OCC(256, 2)
    LP_OCC(256, 4)
    LP_OCC(256, 8)
    LP_OCC(512, 1)
    LP_OCC(512, 2)
    LP_OCC(512, 4)
    LP_OCC(1024, 1)
    LP_OCC(1024, 2)
    LP_OCC(1024, 4)
#undef LP_OCC
    (void)hipGetLastError();
    return 0;
}

// Raises (never lowers) the dynamic-LDS limit of every batched-kernel
// instance: batches and servers of one process share these attributes.
int set_batch_lds_limit(size_t lds) {
    static std::mutex mu;
    static size_t current = 0;
    std::lock_guard<std::mutex> lock(mu);
    if (lds <= current) return LP_OK;
#define LP_ATTR(B, U)                                                                                         \
    LP_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_batch<B, U>),                         \
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    LP_ATTR(256, 1)
    LP_ATTR(256, 2)
    LP_ATTR(256, 4)
    LP_ATTR(256, 8)
    LP_ATTR(512, 1)
    LP_ATTR(512, 2)
    LP_ATTR(512, 4)
    LP_ATTR(1024, 1)
    LP_ATTR(1024, 2)
    LP_ATTR(1024, 4)
#undef LP_ATTR
    current = lds;
    return LP_OK;
}

size_t device_lds_limit(int device) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return 64 * 1024;
    return prop.sharedMemPerBlock;
}

int device_cus(int device) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return 256;
    return prop.multiProcessorCount;
}

// ---- autotune cache: one JSON object per line,
// {"key": "<bucket>", "block": B, "unroll": U, "grid_per_cu": G, "split": S, "ms": t}
// (a line without "split" means 1)
std::string batch_bucket_key(int32_t count, int32_t mmax, int32_t nmax) {
    auto up = [](int64_t x) {
        int64_t p = 1;
        while (p < x) p <<= 1;
        return p;
    };
    char buf[128];
    std::snprintf(buf, sizeof buf, "batch/count%lld/m%lld/n%lld", (long long)up(count), (long long)up(mmax),
                  (long long)up(nmax));
    return buf;
}

bool cache_lookup(const char *path, const std::string &key, BatchShape *out) {
    if (!path || !*path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        char k[256];
        int b = 0, u = 0, g = 0, sp = 1;
        const int got = std::sscanf(line, " {\"key\": \"%255[^\"]\", \"block\": %d, \"unroll\": %d, \"grid_per_cu\": %d, "
                                          "\"split\": %d", k, &b, &u, &g, &sp);
        if (got >= 4 && key == k) {
            if (got < 5) sp = 1;
            for (int i = 0; i < kNumBatchShapes; ++i)
                if (kBatchShapes[i].block == b && kBatchShapes[i].unroll == u && kBatchShapes[i].grid_per_cu == g &&
                    kBatchShapes[i].split == sp) {
                    *out = kBatchShapes[i];
                    found = true;  // the last matching line wins
                }
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const char *path, const std::string &key, const BatchShape &sh, double ms) {
    if (!path || !*path) return;
    static std::mutex mu;
    std::lock_guard<std::mutex> lock(mu);
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "{\"key\": \"%s\", \"block\": %d, \"unroll\": %d, \"grid_per_cu\": %d, \"split\": %d, \"ms\": %.6f}\n",
                 key.c_str(), sh.block, sh.unroll, sh.grid_per_cu, sh.split, ms);
    std::fclose(f);
}

}  // namespace lpgpu

namespace {

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

}  // namespace

struct lp_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int32_t count = 0;
    std::vector<int32_t> m, n;
    std::vector<int64_t> ld, out_off, in_off;
    std::vector<BatchDesc> desc_host;
    double *tab = nullptr;       // tableaux
    int32_t *ints = nullptr;     // basis, lists, logs
    double *inputs = nullptr;    // A, b, c of every LP, kept for rebuilds
    double *out = nullptr;       // x, y, objective of every LP
    double *scratch = nullptr;   // global work areas of LPs whose F/R exceed the LDS limit
    int64_t *out_off_dev = nullptr;
    BatchDesc *desc = nullptr;
    BatchState *state = nullptr;
    int32_t *order = nullptr;    // the queue: LP indices, largest first (a split LP once per part)
    int32_t *parts = nullptr;    // per queue entry: (parts << 8) | part of a split LP, else 0
    int32_t *norder = nullptr;   // number of entries of `order`
    int32_t *head = nullptr;     // queue head
    BatchSync *sync = nullptr;   // meeting areas, one per LP (used by split LPs)
    int32_t entries = 0;         // queue entries of the current plan
    uint32_t gate_spin = kPartGateSpin;  // polls of a split LP's check-in gate (0: closes at once)
    int32_t split_lps = 0;       // LPs the current plan splits
    int32_t *tile_lp = nullptr;  // build tile -> LP
    int64_t *tile_first = nullptr, *in_off_dev = nullptr;
    int64_t ntiles = 0;
    std::vector<BatchState> st_init;  // initial state of every LP
    BatchState init{};
    size_t lds = 0;
    BatchShape shape{};
    int cus = 256;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double last_ms = -1.0;
    bool solved = false;
    std::vector<BatchState> st_host;
    std::vector<double> out_host;
};

namespace {

void free_batch(lp_batch *b) {
    if (!b) return;
    DeviceGuard g(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (void *p : {(void *)b->tab, (void *)b->ints, (void *)b->inputs, (void *)b->out, (void *)b->scratch,
                    (void *)b->out_off_dev,
                    (void *)b->desc, (void *)b->state, (void *)b->order, (void *)b->parts, (void *)b->norder,
                    (void *)b->head, (void *)b->sync,
                    (void *)b->tile_lp, (void *)b->tile_first, (void *)b->in_off_dev})
        if (p) (void)hipFree(p);
    if (b->e0) (void)hipEventDestroy(b->e0);
    if (b->e1) (void)hipEventDestroy(b->e1);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

// The queue for the current shape: LPs in decreasing order of estimated work
// ((m+1)(n+2) entries times min(m, n), a stand-in for the pivot count); with
// a shape that splits, an LP whose estimate exceeds twice the work per
// workgroup of the grid gets ceil(estimate / that) parts, at most
// shape.split, and only while the parts of the split LPs fill at most half
// of the grid (they come first, so their parts start together) and every
// workgroup of the grid is resident at once. LPs whose work area lives in
// global memory are never split.
int plan_queue(lp_batch *b) {
    const int32_t count = b->count;
    std::vector<double> work(count);
    double total = 0.0;
    for (int32_t k = 0; k < count; ++k) {
        work[k] = (double)(b->m[k] + 1) * (b->n[k] + 2) * std::min(b->m[k], b->n[k]);
        total += work[k];
    }
    std::vector<int32_t> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) { return work[a] > work[c]; });
    const int slots = std::max(1, b->shape.grid_per_cu * b->cus);
    int wmax = std::min(b->shape.split, kMaxBatchParts);
    if (wmax > 1 && batch_blocks_per_cu(b->shape, b->lds) < b->shape.grid_per_cu) wmax = 1;
    const double share = total / slots;
    std::vector<int32_t> q, qp;
    int used = 0;
    b->split_lps = 0;
    for (int32_t k : order) {
        int w = 1;
        if (wmax > 1 && !b->desc_host[k].scratch && work[k] > 2.0 * share) {
            w = std::min<int>(wmax, (int)std::ceil(work[k] / share));
            if (used + w > slots / 2) w = 1;
        }
        b->desc_host[k].sync = w > 1 ? b->sync + k : nullptr;
        if (w > 1) {
            used += w;
            ++b->split_lps;
        }
        for (int p = 0; p < w; ++p) {
            q.push_back(k);
            qp.push_back(w > 1 ? (w << 8) | p : 0);
        }
    }
    b->entries = (int32_t)q.size();
    LP_HIP_CHECK(hipMemcpy(b->desc, b->desc_host.data(), count * sizeof(BatchDesc), hipMemcpyHostToDevice));
    LP_HIP_CHECK(hipMemcpy(b->order, q.data(), q.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    LP_HIP_CHECK(hipMemcpy(b->parts, qp.data(), qp.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    LP_HIP_CHECK(hipMemcpy(b->norder, &b->entries, sizeof(int32_t), hipMemcpyHostToDevice));
    return LP_OK;
}

int capture_batch_graph(lp_batch *b) {
    LP_HIP_CHECK(hipStreamSynchronize(b->stream));  // (nothing in flight reads the queue being replaced)
    if (int rc = plan_queue(b)) return rc;
    if (b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    const int grid = std::max(1, std::min<int>(b->entries, b->shape.grid_per_cu * b->cus));
    LP_HIP_CHECK(hipStreamSynchronize(b->stream));
    LP_HIP_CHECK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    int rc = launch_batch_kernel(b->shape, grid, b->lds, b->stream, b->desc, b->state, b->order, b->norder, b->head,
                                 INT64_MAX, b->parts, b->gate_spin);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return set_error(LP_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    b->graph = graph;
    LP_HIP_CHECK(hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0));
    return LP_OK;
}

// Initialization Step for every LP, from the stored inputs: one build launch
// over all tiles, one launch for the lists, one copy of the states.
int rebuild_all(lp_batch *b) {
    hipLaunchKernelGGL(k_batch_build, dim3((unsigned)b->ntiles), dim3(256), 0, b->stream, b->desc, b->inputs,
                       b->in_off_dev, b->tile_lp, b->tile_first);
    hipLaunchKernelGGL(k_batch_init_all, dim3((unsigned)b->count), dim3(256), 0, b->stream, b->desc);
    hipLaunchKernelGGL(k_batch_sync_reset, dim3((unsigned)((b->count + 255) / 256)), dim3(256), 0, b->stream, b->sync,
                       b->count);
    LP_HIP_CHECK(hipGetLastError());
    LP_HIP_CHECK(hipMemcpyAsync(b->state, b->st_init.data(), b->st_init.size() * sizeof(BatchState),
                                hipMemcpyHostToDevice, b->stream));
    b->solved = false;
    return LP_OK;
}

int run_batch(lp_batch *b) {
    DeviceGuard g(b->device);
    LP_HIP_CHECK(hipEventRecord(b->e0, b->stream));
    LP_HIP_CHECK(hipGraphLaunch(b->gexec, b->stream));
    LP_HIP_CHECK(hipEventRecord(b->e1, b->stream));
    hipLaunchKernelGGL(k_batch_extract, dim3((unsigned)b->count), dim3(256), 0, b->stream, b->desc,
                       b->out_off_dev, b->out);
    LP_HIP_CHECK(hipGetLastError());
    LP_HIP_CHECK(hipMemcpyAsync(b->st_host.data(), b->state, b->st_host.size() * sizeof(BatchState),
                                hipMemcpyDeviceToHost, b->stream));
    LP_HIP_CHECK(hipMemcpyAsync(b->out_host.data(), b->out, b->out_host.size() * sizeof(double),
                                hipMemcpyDeviceToHost, b->stream));
    LP_HIP_CHECK(hipStreamSynchronize(b->stream));
    float ms = 0.f;
    LP_HIP_CHECK(hipEventElapsedTime(&ms, b->e0, b->e1));
    b->last_ms = ms;
    b->solved = true;
    return LP_OK;
}

}  // namespace

extern "C" {

int lp_batch_create(lp_batch **out, int32_t count, const int32_t *m, const int32_t *n, const double *const *A,
                    const double *const *bv, const double *const *cv, const lp_options *opt_in) {
    if (!out) return set_error(LP_E_INVAL, "out is NULL");
    *out = nullptr;
    if (count < 1 || !m || !n || !A || !bv || !cv) return set_error(LP_E_INVAL, "bad batch arguments");
    const Options o = resolve_options(opt_in);
    if (o.bland_after != 0) return set_error(LP_E_INVAL, "the batched form takes bland_after 0 only");
    if (!(o.eps_dual >= 0.0) || !(o.eps_pivot >= 0.0) || !std::isfinite(o.eps_dual) || !std::isfinite(o.eps_pivot))
        return set_error(LP_E_INVAL, "eps_dual and eps_pivot must be finite and >= 0");
    int ndev = 0;
    LP_HIP_CHECK(hipGetDeviceCount(&ndev));
    if (o.device < 0 || o.device >= ndev) return set_error(LP_E_INVAL, "device ordinal out of range");
    const size_t lds_limit = std::min<size_t>(device_lds_limit(o.device), 64 * 1024);
    for (int32_t k = 0; k < count; ++k) {
        if (m[k] < 1 || n[k] < 1 || !A[k] || !bv[k] || !cv[k])
            return set_error(LP_E_INVAL, "LP " + std::to_string(k) + ": bad size or NULL input");
        if (!batch_size_ok(m[k], n[k]))
            return set_error(LP_E_INVAL, "LP " + std::to_string(k) + " is too large for the batched kernel");
        for (int64_t t = 0; t < (int64_t)m[k] * n[k]; ++t)
            if (!std::isfinite(A[k][t])) return set_error(LP_E_INVAL, "LP " + std::to_string(k) + ": non-finite A");
        for (int32_t i = 0; i < m[k]; ++i) {
            if (!std::isfinite(bv[k][i])) return set_error(LP_E_INVAL, "LP " + std::to_string(k) + ": non-finite b");
            if (bv[k][i] < 0.0) return set_error(LP_E_NEG_RHS, "LP " + std::to_string(k) + ": negative b");
        }
        for (int32_t j = 0; j < n[k]; ++j)
            if (!std::isfinite(cv[k][j])) return set_error(LP_E_INVAL, "LP " + std::to_string(k) + ": non-finite c");
    }

    lp_batch *b = new (std::nothrow) lp_batch;
    if (!b) return set_error(LP_E_NOMEM, "host allocation failed");
    b->device = o.device;
    DeviceGuard g(b->device);
    auto fail = [&](int rc) {
        free_batch(b);
        return rc;
    };
    b->count = count;
    b->gate_spin = o.decide_spin == -1 ? 0u : kPartGateSpin;
    b->m.assign(m, m + count);
    b->n.assign(n, n + count);
    b->cus = device_cus(o.device);
    if (o.stream) {
        b->stream = (hipStream_t)o.stream;
    } else {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess)
            return fail(set_error(LP_E_DEVICE, "hipStreamCreate failed"));
        b->own_stream = true;
    }
    if (hipEventCreate(&b->e0) != hipSuccess || hipEventCreate(&b->e1) != hipSuccess)
        return fail(set_error(LP_E_DEVICE, "hipEventCreate failed"));

    // layout
    int64_t tab_total = 0, int_total = 0, in_total = 0, out_total = 0, scr_total = 0;
    std::vector<int64_t> tab_off(count), int_off(count), logcap(count), scr_off(count, -1);
    b->ld.resize(count);
    b->out_off.resize(count);
    b->in_off.resize(count);
    int32_t mmax = 0, nmax = 0;
    for (int32_t k = 0; k < count; ++k) {
        const int64_t ld = padded_ld(m[k]), W = (int64_t)n[k] + m[k] + 1;
        b->ld[k] = ld;
        tab_off[k] = tab_total;
        tab_total += ld * W;
        const int64_t maxp = o.max_pivots > 0 ? o.max_pivots : 50 * ((int64_t)m[k] + n[k]);
        logcap[k] = o.record_pivots ? std::min<int64_t>(maxp, 4 * ((int64_t)m[k] + n[k]) + 64) : 0;
        int_off[k] = int_total;
        int_total += (int64_t)m[k] + (n[k] + 2) + ((int64_t)n[k] + m[k]) + 2 * logcap[k];
        int_total = (int_total + 3) / 4 * 4;
        b->in_off[k] = in_total;
        in_total += (int64_t)m[k] * n[k] + m[k] + n[k];
        b->out_off[k] = out_total;
        out_total += (int64_t)n[k] + m[k] + 1;
        if (batch_lds_bytes(m[k], n[k]) <= lds_limit) {
            b->lds = std::max(b->lds, batch_lds_bytes(m[k], n[k]));
        } else {
            scr_off[k] = scr_total;
            scr_total += ((int64_t)batch_lds_bytes(m[k], n[k]) + 255) / 256 * 32;  // in doubles, 256-byte aligned
        }
        mmax = std::max(mmax, m[k]);
        nmax = std::max(nmax, n[k]);
    }
    auto dmalloc = [&](void **p, size_t bytes) -> int {
        if (hipMalloc(p, std::max<size_t>(bytes, 16)) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(LP_E_NOMEM, "hipMalloc failed (" + std::to_string(bytes) + " bytes)");
        }
        return LP_OK;
    };
    if (int rc = dmalloc((void **)&b->tab, tab_total * sizeof(double))) return fail(rc);
    if (int rc = dmalloc((void **)&b->ints, int_total * sizeof(int32_t))) return fail(rc);
    if (int rc = dmalloc((void **)&b->inputs, in_total * sizeof(double))) return fail(rc);
    if (int rc = dmalloc((void **)&b->out, out_total * sizeof(double))) return fail(rc);
    if (scr_total)
        if (int rc = dmalloc((void **)&b->scratch, scr_total * sizeof(double))) return fail(rc);
    if (int rc = dmalloc((void **)&b->out_off_dev, count * sizeof(int64_t))) return fail(rc);
    if (int rc = dmalloc((void **)&b->desc, count * sizeof(BatchDesc))) return fail(rc);
    if (int rc = dmalloc((void **)&b->state, count * sizeof(BatchState))) return fail(rc);
    if (int rc = dmalloc((void **)&b->order, (size_t)count * kMaxBatchParts * sizeof(int32_t))) return fail(rc);
    if (int rc = dmalloc((void **)&b->parts, (size_t)count * kMaxBatchParts * sizeof(int32_t))) return fail(rc);
    if (int rc = dmalloc((void **)&b->sync, (size_t)count * sizeof(BatchSync))) return fail(rc);
    if (hipMemset(b->sync, 0, (size_t)count * sizeof(BatchSync)) != hipSuccess)
        return fail(set_error(LP_E_DEVICE, "hipMemset failed"));
    if (int rc = dmalloc((void **)&b->norder, sizeof(int32_t))) return fail(rc);
    if (int rc = dmalloc((void **)&b->head, sizeof(int32_t))) return fail(rc);

    b->desc_host.resize(count);
    for (int32_t k = 0; k < count; ++k) {
        BatchDesc &d = b->desc_host[k];
        d.T = b->tab + tab_off[k];
        d.ld = b->ld[k];
        d.m = m[k];
        d.n = n[k];
        int32_t *base = b->ints + int_off[k];
        d.basis = base;
        d.cols = base + m[k];
        d.pos = d.cols + n[k] + 2;
        d.log_r = d.pos + n[k] + m[k];
        d.log_q = d.log_r + logcap[k];
        d.log_cap = logcap[k];
        d.nvec = (m[k] + 2) / 2;
        d.magic = nvec_magic(d.nvec);
        d.pad = 0;
        d.scratch = scr_off[k] >= 0 ? b->scratch + scr_off[k] : nullptr;
        d.sync = nullptr;
    }
    // inputs, staged through one host buffer
    {
        std::vector<double> host((size_t)in_total);
        for (int32_t k = 0; k < count; ++k) {
            double *dst = host.data() + b->in_off[k];
            std::memcpy(dst, A[k], (size_t)m[k] * n[k] * sizeof(double));
            std::memcpy(dst + (int64_t)m[k] * n[k], bv[k], (size_t)m[k] * sizeof(double));
            std::memcpy(dst + (int64_t)m[k] * n[k] + m[k], cv[k], (size_t)n[k] * sizeof(double));
        }
        if (hipMemcpy(b->inputs, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
            return fail(set_error(LP_E_DEVICE, "input copy failed"));
    }
    // (the queue, and the descriptors again with their meeting areas, are
    // uploaded with the plan of the kernel shape)
    if (hipMemcpy(b->desc, b->desc_host.data(), count * sizeof(BatchDesc), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->out_off_dev, b->out_off.data(), count * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess)
        return fail(set_error(LP_E_DEVICE, "descriptor copy failed"));

    b->init = BatchState{};
    b->init.status = LP_RUNNING;
    b->init.eps_d = o.eps_dual;
    b->init.eps_p = o.eps_pivot;
    b->st_init.resize(count);
    for (int32_t k = 0; k < count; ++k) {
        b->st_init[k] = b->init;
        b->st_init[k].max_pivots = o.max_pivots > 0 ? o.max_pivots : 50 * ((int64_t)m[k] + n[k]);
    }
    b->st_host = b->st_init;
    b->out_host.resize((size_t)out_total);
    {
        std::vector<int64_t> first(count + 1, 0);
        for (int32_t k = 0; k < count; ++k) {
            const int64_t rt = (b->ld[k] + 63) / 64;
            first[k + 1] = first[k] + (int64_t)((n[k] + 63) / 64) * rt + (int64_t)((m[k] + 1 + 63) / 64) * rt;
        }
        b->ntiles = first[count];
        std::vector<int32_t> tl((size_t)b->ntiles);
        for (int32_t k = 0; k < count; ++k)
            for (int64_t t = first[k]; t < first[k + 1]; ++t) tl[(size_t)t] = k;
        if (int rc = dmalloc((void **)&b->tile_lp, tl.size() * sizeof(int32_t))) return fail(rc);
        if (int rc = dmalloc((void **)&b->tile_first, first.size() * sizeof(int64_t))) return fail(rc);
        if (int rc = dmalloc((void **)&b->in_off_dev, count * sizeof(int64_t))) return fail(rc);
        if (hipMemcpy(b->tile_lp, tl.data(), tl.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(b->tile_first, first.data(), first.size() * sizeof(int64_t), hipMemcpyHostToDevice) !=
                hipSuccess ||
            hipMemcpy(b->in_off_dev, b->in_off.data(), count * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess)
            return fail(set_error(LP_E_DEVICE, "tile table copy failed"));
    }
    if (int rc = rebuild_all(b)) return fail(rc);
    if (hipStreamSynchronize(b->stream) != hipSuccess) return fail(set_error(LP_E_DEVICE, "build failed"));
    if (int rc = set_batch_lds_limit(b->lds)) return fail(rc);

    // kernel shape: explicit option, else the autotune cache, else a default
    b->shape = kBatchShapes[2];
    const char *cache = std::getenv("LP_AUTOTUNE_CACHE");
    BatchShape cached{};
    if (o.batch_block > 0 || o.batch_unroll > 0) {
        bool ok = false;
        for (int i = 0; i < kNumBatchShapes; ++i)
            if ((o.batch_block <= 0 || kBatchShapes[i].block == o.batch_block) &&
                (o.batch_unroll <= 0 || kBatchShapes[i].unroll == o.batch_unroll)) {
                b->shape = kBatchShapes[i];
                ok = true;
                break;
            }
        if (!ok) return fail(set_error(LP_E_INVAL, "no batch kernel shape with that block / unroll"));
    } else if (cache_lookup(cache, batch_bucket_key(count, mmax, nmax), &cached)) {
        b->shape = cached;
    }
    if (int rc = capture_batch_graph(b)) return fail(rc);
    *out = b;
    return LP_OK;
}

int lp_batch_solve(lp_batch *b) {
    if (!b) return set_error(LP_E_INVAL, "NULL batch");
    return run_batch(b);
}

int lp_batch_reset(lp_batch *b) {
    if (!b) return set_error(LP_E_INVAL, "NULL batch");
    DeviceGuard g(b->device);
    if (int rc = rebuild_all(b)) return rc;
    LP_HIP_CHECK(hipStreamSynchronize(b->stream));
    return LP_OK;
}

int lp_batch_get_solution(const lp_batch *b, int32_t k, lp_result *res, double *x, double *y) {
    if (!b || k < 0 || k >= b->count) return set_error(LP_E_INVAL, "bad batch or index");
    if (!b->solved) return set_error(LP_E_STATE, "batch not solved yet");
    const double *o = b->out_host.data() + b->out_off[k];
    const int32_t m = b->m[k], n = b->n[k];
    if (x) std::memcpy(x, o, (size_t)n * sizeof(double));
    if (y) std::memcpy(y, o + n, (size_t)m * sizeof(double));
    if (res) {
        res->status = b->st_host[k].status;
        res->reserved = 0;
        res->pivots = b->st_host[k].pivots;
        res->objective = o[n + m];
        res->solve_ms = b->last_ms;
    }
    return LP_OK;
}

int lp_batch_get_pivots(const lp_batch *b, int32_t k, int32_t *rows, int32_t *cols, int64_t cap, int64_t *count) {
    if (!b || k < 0 || k >= b->count || cap < 0 || (cap > 0 && (!rows || !cols)))
        return set_error(LP_E_INVAL, "bad argument");
    DeviceGuard g(b->device);
    LP_HIP_CHECK(hipStreamSynchronize(b->stream));
    BatchState s;
    LP_HIP_CHECK(hipMemcpy(&s, b->state + k, sizeof(s), hipMemcpyDeviceToHost));
    const BatchDesc &d = b->desc_host[k];
    if (count) *count = s.pivots;
    const int64_t c = std::min<int64_t>(std::min<int64_t>(s.pivots, d.log_cap), cap);
    if (c > 0) {
        LP_HIP_CHECK(hipMemcpy(rows, d.log_r, (size_t)c * sizeof(int32_t), hipMemcpyDeviceToHost));
        LP_HIP_CHECK(hipMemcpy(cols, d.log_q, (size_t)c * sizeof(int32_t), hipMemcpyDeviceToHost));
    }
    return LP_OK;
}

double lp_batch_solve_ms(const lp_batch *b) { return b ? b->last_ms : -1.0; }

int lp_batch_get_shape(const lp_batch *b, int32_t *block, int32_t *unroll, int32_t *grid_per_cu) {
    if (!b) return set_error(LP_E_INVAL, "NULL batch");
    if (block) *block = b->shape.block;
    if (unroll) *unroll = b->shape.unroll;
    if (grid_per_cu) *grid_per_cu = b->shape.grid_per_cu;
    return LP_OK;
}

int lp_batch_get_split(const lp_batch *b, int32_t *max_parts, int32_t *split_lps, int32_t *queue_entries) {
    if (!b) return set_error(LP_E_INVAL, "NULL batch");
    if (max_parts) *max_parts = b->shape.split;
    if (split_lps) *split_lps = b->split_lps;
    if (queue_entries) *queue_entries = b->entries;
    return LP_OK;
}

int lp_batch_set_shape(lp_batch *b, int32_t block, int32_t unroll, int32_t grid_per_cu, int32_t split) {
    if (!b) return set_error(LP_E_INVAL, "NULL batch");
    for (int i = 0; i < kNumBatchShapes; ++i) {
        const BatchShape &sh = kBatchShapes[i];
        if (sh.block == block && sh.unroll == unroll && sh.grid_per_cu == grid_per_cu && sh.split == split) {
            DeviceGuard g(b->device);
            b->shape = sh;
            return capture_batch_graph(b);
        }
    }
    return set_error(LP_E_INVAL, "no batch kernel shape with that block, unroll, grid_per_cu and split");
}

int lp_batch_autotune(lp_batch *b, const char *cache_path, int32_t trials, double *best_ms) {
    if (!b) return set_error(LP_E_INVAL, "NULL batch");
    if (trials < 1) trials = 1;
    DeviceGuard g(b->device);
    const BatchShape keep = b->shape;
    double best = 1e300;
    BatchShape best_shape = keep;
    for (int i = 0; i < kNumBatchShapes; ++i) {
        b->shape = kBatchShapes[i];
        if (int rc = capture_batch_graph(b)) return rc;
        double t = 1e300;
        for (int r = 0; r < trials; ++r) {
            if (int rc = lp_batch_reset(b)) return rc;
            if (int rc = run_batch(b)) return rc;
            t = std::min(t, b->last_ms);
        }
        if (t < best) {
            best = t;
            best_shape = b->shape;
        }
    }
    b->shape = best_shape;
    if (int rc = capture_batch_graph(b)) return rc;
    if (int rc = lp_batch_reset(b)) return rc;
    int32_t mmax = 0, nmax = 0;
    for (int32_t k = 0; k < b->count; ++k) {
        mmax = std::max(mmax, b->m[k]);
        nmax = std::max(nmax, b->n[k]);
    }
    cache_store(cache_path, batch_bucket_key(b->count, mmax, nmax), best_shape, best);
    if (best_ms) *best_ms = best;
    return LP_OK;
}

void lp_batch_destroy(lp_batch *b) { free_batch(b); }

}  // extern "C"
