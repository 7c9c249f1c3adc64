// lp_hybrid_*: the paper's CPU + GPU column split (Section IV), on one GPU
// and the host's cores. The GPU holds a share theta of the tableau's columns
// (the paper's theta) and the host the rest: the first round(theta n) of the
// n structural columns and the first round(theta m) of the m slack columns
// go to the GPU, the others to the host, so that each side holds its share
// of the columns that are nonbasic at the start. Each side numbers its
// columns in increasing order of the global column index (local indices), so
// that a side's (value, local index) argmin agrees with the (value, global
// index) order. The right-hand side is kept on both sides (as the paper
// replicates it), and both update their copy with the same operations, so the
// copies stay equal. Per pivot (Steps 1-3 in the paper's order):
//   Step 1  each side reduces the row-0 entries of its columns; the host
//           combines the two (value, column) pairs in the (value, index)
//           order (a NaN wins, ties go to the lower column);
//   Step 2  the side that owns the entering column q runs the ratio test on
//           it (and the non-finite checks over every row) and hands the
//           pivot column F to the other side (one copy over PCIe);
//   Step 3  each side normalises the pivot-row entries of its own columns
//           (R_j = T[r][j] / p) and updates them, T[i][j] = fma(-F_i, R_j,
//           T[i][j]) for i != r, T[r][j] = R_j: the GPU with the one-pivot
//           update kernel, the host's share at the same time on a pool of
//           threads (std::fma).
// As in the single-GPU solver, each side rewrites only a list of its
// columns: the nonbasic ones, the leaving column, and the RHS (a column that
// is basic is the unit vector of its row, which no pivot changes until it
// leaves). The entering column is rewritten at its pivot (into that unit
// vector, exactly) and then dropped from its side's list; the leaving column
// joins its side's list at its pivot. The host keeps both lists; the device
// keeps a copy of its own and of the basis, so that when the entering column
// is on the device, the device appends the leaving column itself and starts
// Step 3 without waiting for the host. The arithmetic is that of the
// single-GPU solver: the same pivots and, up to the sign of zeros, the same
// values.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <limits>
#include <new>
#include <thread>
#include <vector>

#include "plain_kernels.hpp"

using namespace lpgpu;

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

// The device's share of Table I: its J columns (local index d holds global
// column dglob[d]), then the RHS as device column J and a zero column J+1 (the list slot that takes a
// leaving column of the host's side: rewriting it changes nothing); one
// thread per entry, column-major.
__global__ __launch_bounds__(256) void k_hyb_build(double *__restrict__ T, int64_t ld, int32_t m, int32_t n,
                                                   int32_t J, const int32_t *__restrict__ dglob,
                                                   const double *__restrict__ A, const double *__restrict__ b,
                                                   const double *__restrict__ c) {
    const int64_t total = ld * ((int64_t)J + 2);
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = idx / ld;
        const int32_t i = (int32_t)(idx - j * ld);
        double v = 0.0;
        if (j == J + 1) {
            v = 0.0;
        } else if (j == J) {
            if (i >= 1 && i <= m) v = b[i - 1];
        } else {
            const int32_t g = dglob[j];  // the global column
            if (g < n) {
                if (i == 0)
                    v = -c[g];
                else if (i <= m)
                    v = A[(int64_t)(i - 1) * n + g];
            } else {
                v = i == g - n + 1 ? 1.0 : 0.0;
            }
        }
        T[idx] = v;
    }
}

// Step 1 on the device's columns: the final argmin of the update's partials,
// or (fresh) a scan of row 0 over columns [0, J), stored in host memory. One
// workgroup of 1024.
// The kernels hand their results to the host by storing them in pinned host
// memory themselves (no copy commands); the host polls a sequence word that
// the kernel stores last: every thread's stores to host memory are made
// visible system-wide first. Every thread of the block calls it.
__device__ __forceinline__ void hyb_signal(uint32_t *seq, uint32_t value) {
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(seq, value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ __launch_bounds__(1024) void k_hyb_price(const double *__restrict__ T, int64_t ld, int32_t J,
                                                    const ArgMin *__restrict__ parts, int32_t nparts, int32_t fresh,
                                                    ArgMin *__restrict__ out, uint32_t *seq, uint32_t seqv) {
    __shared__ double sv[16];
    __shared__ int32_t si[16];
    double v = __builtin_inf();
    int32_t q = kNoIndex;
    if (fresh) {
        for (int32_t j = threadIdx.x; j < J; j += blockDim.x) {
            const double t = T[(int64_t)j * ld];
            if (lex_less(t, j, v, q)) {
                v = t;
                q = j;
            }
        }
    } else {
        for (int32_t k = threadIdx.x; k < nparts; k += blockDim.x) {
            const ArgMin a = parts[k];
            if (lex_less(a.v, a.i, v, q)) {
                v = a.v;
                q = a.i;
            }
        }
    }
    block_argmin(v, q, sv, si);
    if (threadIdx.x == 0) *out = ArgMin{v, q};
    hyb_signal(seq, seqv);
}

// Step 2 on device column q (global column qg): F = column q (rows 0..m, to
// device and host memory), the smallest ratio over rows 1..m with F_i > eps_p (lowest row on
// ties), and the non-finite check of every row. Also arms the device's Step 3 (go, r, p in the state)
// when the pivot is taken (apply: the iteration cap allows it), so that the
// update follows without a host round trip. One workgroup of 1024.
struct HybPivot {
    double v;
    int32_t r;
    int32_t bad;
};

__global__ __launch_bounds__(1024) void k_hyb_ratio(const double *__restrict__ T, int64_t ld, int32_t m, int32_t q,
                                                    int32_t rhs_col, double eps_p, int32_t apply,
                                                    double *__restrict__ F, double *__restrict__ F_host,
                                                    HybPivot *__restrict__ out, DevState *__restrict__ st,
                                                    int32_t *__restrict__ cols, int32_t *__restrict__ basis,
                                                    const int32_t *__restrict__ dloc, int32_t qg, int32_t rem_s,
                                                    int32_t rem_v, int32_t L, uint32_t *seq, uint32_t seqv) {
    __shared__ double sv[16];
    __shared__ int32_t si[16];
    const double *colq = T + (int64_t)q * ld;
    const double *rhs = T + (int64_t)rhs_col * ld;
    double rv = __builtin_inf();
    int32_t r = kNoIndex;
    int bad = 0;
    if (threadIdx.x == 0) {
        F[0] = colq[0];
        F_host[0] = colq[0];
        if (rem_s >= 0) cols[rem_s] = rem_v;  // the previous entering column leaves the list
    }
    for (int32_t i = 1 + threadIdx.x; i <= m; i += blockDim.x) {
        const double a = colq[i], bb = rhs[i];
        F[i] = a;
        F_host[i] = a;
        if (step2_bad(a, bb)) {
            bad = 1;
        } else if (a > eps_p) {
            const double ratio = bb / a;
            if (lex_less(ratio, i, rv, r)) {
                rv = ratio;
                r = i;
            }
        }
    }
    bad = __syncthreads_or(bad);
    block_argmin(rv, r, sv, si);
    if (threadIdx.x == 0) {
        *out = HybPivot{rv, r, bad};
        const bool go = apply && !bad && r != kNoIndex;
        st->go = go;
        int32_t slot = rhs_col + 1;  // (the zero column)
        if (go) {
            st->r = r;
            st->p = colq[r];
            const int32_t leave = dloc[basis[r - 1]];  // (its local index, or -1 on the host's side)
            if (leave >= 0) slot = leave;           // a device column joins the list
            basis[r - 1] = qg;
        }
        cols[L] = slot;
    }
    hyb_signal(seq, seqv);
}

// The device's list and basis when the entering column is on the host's
// side: the previous entering column leaves the list, slot L takes the
// leaving column (or the zero column), and row r's basic column becomes q
// (global indices in the basis).
__global__ void k_hyb_relist(int32_t *__restrict__ cols, int32_t *__restrict__ basis, int32_t rem_s, int32_t rem_v,
                             int32_t L, int32_t slot, int32_t row, int32_t q) {
    if (rem_s >= 0) cols[rem_s] = rem_v;
    cols[L] = slot;
    basis[row - 1] = q;
}

// Step 3 inputs on the device: R of every list slot, from the state's (r, p).
__global__ __launch_bounds__(256) void k_hyb_stage(const double *__restrict__ T, int64_t ld, int32_t ncols,
                                                   const int32_t *__restrict__ cols, const DevState *__restrict__ st,
                                                   double *__restrict__ Rl) {
    if (!st->go) return;
    const int32_t t = (int32_t)(blockIdx.x * 256 + threadIdx.x);
    if (t < ncols) Rl[t] = T[(int64_t)cols[t] * ld + st->r] / st->p;
}

// A pool of host threads that wait for tasks by spinning with a yield (a
// pivot's host share takes tens to hundreds of microseconds; waking sleeping
// threads would cost as much, and the yield leaves the cores to other
// runnable threads). Task k of a run goes to thread k; the caller runs
// task 0.
class SpinPool {
  public:
    explicit SpinPool(int threads) : n_(std::max(1, threads)) {
        for (int k = 1; k < n_; ++k) th_.emplace_back([this, k] { loop(k); });
    }
    ~SpinPool() {
        stop_.store(true, std::memory_order_release);
        gen_.fetch_add(1, std::memory_order_acq_rel);
        for (auto &t : th_) t.join();
    }
    int size() const { return n_; }
    template <class F>
    void run(F &&f) {
        task_ = [&f](int k) { f(k); };
        done_.store(0, std::memory_order_relaxed);
        gen_.fetch_add(1, std::memory_order_acq_rel);
        f(0);
        while (done_.load(std::memory_order_acquire) != n_ - 1) std::this_thread::yield();
    }

  private:
    void loop(int k) {
        uint64_t seen = 0;
        for (;;) {
            uint64_t g;
            // spin, yielding the core to other runnable threads (the HIP
            // runtime's among them) while the GPU works
            while ((g = gen_.load(std::memory_order_acquire)) == seen) std::this_thread::yield();
            seen = g;
            if (stop_.load(std::memory_order_acquire)) return;
            task_(k);
            done_.fetch_add(1, std::memory_order_acq_rel);
        }
    }
    int n_;
    std::vector<std::thread> th_;
    std::function<void(int)> task_;
    std::atomic<uint64_t> gen_{0};
    std::atomic<int> done_{0};
    std::atomic<bool> stop_{false};
};

// The kernels' (value, index) order and non-finite checks, on the host: a NaN
// first, then smaller values, then lower indices; Step 1 stops on a NaN or
// -inf minimum, Step 2 on a non-finite entering entry or a NaN right-hand side.
bool host_lex_less(double av, int32_t ai, double bv, int32_t bi) {
    const bool an = av != av, bn = bv != bv;
    if (an || bn) return an && (!bn || ai < bi);
    return av < bv || (av == bv && ai < bi);
}
bool host_step1_bad(double v) { return v != v || v == -std::numeric_limits<double>::infinity(); }
bool host_step2_bad(double a, double rhs) { return !std::isfinite(a) || rhs != rhs; }

}  // namespace

struct lp_hybrid {
    int device = 0;
    hipStream_t stream = nullptr;
    int32_t m = 0, n = 0, J = 0, nh = 0;  // device columns [0, J), host columns [J, n+m) (nh of them)
    int64_t ld = 0;
    double theta = 0.0;
    int threads = 1;
    // device
    double *dT = nullptr, *dF = nullptr, *dR = nullptr;
    ArgMin *dparts = nullptr;
    DevState *dst = nullptr;
    int32_t *dcols = nullptr, *dbasis = nullptr;  // the device's list and its copy of the basis
    int nparts = 0, block = 256, cols = 4, rowchunks = 1;  // the update kernel's shape (nparts: the most)
    uint32_t *seq = nullptr;  // pinned: [0] the Step 2 result and F stored, [1] the Step 1 partial stored
    uint32_t seq_next = 0;
    // host
    std::vector<double> hT;  // nh + 1 columns of ld (the last the RHS)
    std::vector<int32_t> basis, log_r, log_q;
    // the lists: device columns (slot 0 the RHS) and host columns (offsets
    // from J; the host RHS is rewritten apart), the slot of each column or -1
    std::vector<int32_t> dl, dpos, hl, hpos;
    // global column of each local one, and of each global column its local
    // index on the device (>= 0) or -(1 + its local index on the host)
    std::vector<int32_t> dglob, hglob, loc;
    int32_t *ddloc = nullptr;  // device: the local index of each global column on the device, or -1
    int32_t rem_s = -1, rem_v = 0;  // a device-list removal not yet written to the device
    double *F = nullptr;  // the pivot column, rows 0..m (pinned, ld entries)
    ArgMin *pin_min = nullptr;
    HybPivot *pin_piv = nullptr;
    DevState *pin_st = nullptr;
    double eps_d = 1e-9, eps_p = 1e-9;
    int64_t max_pivots = 0, log_cap = 0, pivots = 0;
    int32_t status = LP_RUNNING;
    bool ran = false;
    double solve_ms = 0.0, host_ms = 0.0;
};

namespace {

void free_hybrid(lp_hybrid *h) {
    if (!h) return;
    DeviceGuard g(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (void *p : {(void *)h->dT, (void *)h->dF, (void *)h->dR, (void *)h->dparts, (void *)h->dst,
                    (void *)h->dcols, (void *)h->dbasis, (void *)h->ddloc})
        if (p) (void)hipFree(p);
    for (void *p : {(void *)h->F, (void *)h->pin_min, (void *)h->pin_piv, (void *)h->pin_st, (void *)h->seq})
        if (p) (void)hipHostFree(p);
    if (h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

#define LP_HYB_UPD(B, C)                                                                                      \
    hipLaunchKernelGGL((k_update<B, C, 1, 0, 0>), dim3((unsigned)((int64_t)h->rowchunks * np)), dim3(B), 0,   \
                       h->stream, h->dT, h->ld, h->m, ns - 2, h->rowchunks, (const int32_t *)h->dcols,         \
                       (const double *)h->dR, (const double *)h->dF, (const DevState *)h->dst, h->dparts)

// Partials of the update over ns list slots.
int32_t device_parts(const lp_hybrid *h, int32_t ns) { return (ns + h->cols - 1) / h->cols; }

// k_update over the first ns slots of the device's list, in the single-GPU
// solver's shape for this m: 64 or 128 threads and 4 columns per workgroup
// for short columns, else 256 threads and 1 column (4 up to 4096 rows)
void launch_device_update(lp_hybrid *h, int32_t ns) {
    const int32_t np = device_parts(h, ns);
    if (h->block == 64)
        LP_HYB_UPD(64, 4);
    else if (h->block == 128)
        LP_HYB_UPD(128, 4);
    else if (h->cols == 1)
        LP_HYB_UPD(256, 1);
    else
        LP_HYB_UPD(256, 4);
}
#undef LP_HYB_UPD

// The host's share of Steps 1 and 3 for pivot (r, p) with pivot column F:
// the host's list and its RHS updated, then the argmin of the new row-0
// entries of the listed columns.
ArgMin host_pivot(lp_hybrid *h, SpinPool &pool, int32_t r, double p) {
    const int64_t ld = h->ld;
    const int32_t m = h->m, nl = (int32_t)h->hl.size(), ncols = nl + 1;  // the list, then the RHS
    const int nt = pool.size();
    std::vector<ArgMin> best((size_t)nt, ArgMin{__builtin_inf(), kNoIndex});
    const double *F = h->F;
    double *T = h->hT.data();
    pool.run([&](int k) {
        const int32_t c0 = (int32_t)((int64_t)ncols * k / nt), c1 = (int32_t)((int64_t)ncols * (k + 1) / nt);
        ArgMin b{__builtin_inf(), kNoIndex};
        for (int32_t e = c0; e < c1; ++e) {
            const int32_t c = e < nl ? h->hl[(size_t)e] : h->nh;
            double *col = T + (int64_t)c * ld;
            const double R = col[r] / p;
            for (int32_t i = 0; i <= m; ++i) col[i] = std::fma(-F[i], R, col[i]);
            col[r] = R;  // (the pivot row takes R; its fma above is overwritten)
            const int32_t g = e < nl ? h->hglob[(size_t)c] : 0;
            if (e < nl && host_lex_less(col[0], g, b.v, b.i)) b = ArgMin{col[0], g};
        }
        best[(size_t)k] = b;
    });
    ArgMin b{__builtin_inf(), kNoIndex};
    for (const ArgMin &a : best)
        if (host_lex_less(a.v, a.i, b.v, b.i)) b = a;
    return b;
}

ArgMin host_scan(const lp_hybrid *h) {
    ArgMin b{__builtin_inf(), kNoIndex};
    for (int32_t c = 0; c < h->nh; ++c) {
        const double v = h->hT[(size_t)c * h->ld];
        if (host_lex_less(v, h->hglob[(size_t)c], b.v, b.i)) b = ArgMin{v, h->hglob[(size_t)c]};
    }
    return b;
}

// Waits until the device has stored `value` in the sequence word (the kernel
// that writes it stores its results first): a spin of up to about 20 ms
// (a pivot's device share takes well under that), then a stream
// synchronisation, which also reports a failed kernel.
int wait_seq(lp_hybrid *h, int which, uint32_t value) {
    const volatile uint32_t *w = h->seq + which;
    const auto t0 = std::chrono::steady_clock::now();
    for (uint32_t k = 0; *w != value; ++k) {
        if ((k & 1023) == 1023 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(20)) {
            LP_HIP_CHECK(hipStreamSynchronize(h->stream));
            if (*w != value) return set_error(LP_E_DEVICE, "hybrid: a device result did not arrive");
            break;
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return LP_OK;
}

int hybrid_solve(lp_hybrid *h) {
    DeviceGuard g(h->device);
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t ld = h->ld;
    const int32_t m = h->m, J = h->J, zero_col = J + 1;
    SpinPool pool(h->threads);
    double host_ms = 0.0;
    // Step 1 partials of both sides
    uint32_t sv = ++h->seq_next;
    hipLaunchKernelGGL(k_hyb_price, dim3(1), dim3(1024), 0, h->stream, h->dT, ld, J, h->dparts, h->nparts, 1,
                       h->pin_min, h->seq + 1, sv);
    LP_HIP_CHECK(hipGetLastError());
    ArgMin hmin = host_scan(h);
    if (int rc = wait_seq(h, 1, sv)) return rc;
    h->status = LP_RUNNING;
    for (;;) {
        // Step 1: the two sides' minima combined (in global indices)
        ArgMin qb = *h->pin_min;
        if (qb.i != kNoIndex) qb.i = h->dglob[(size_t)qb.i];
        if (host_lex_less(hmin.v, hmin.i, qb.v, qb.i)) qb = hmin;
        if (host_step1_bad(qb.v)) {
            h->status = LP_NUMERICAL;
            break;
        }
        if (qb.v >= -h->eps_d) {
            h->status = LP_OPTIMAL;
            break;
        }
        const int32_t q = qb.i;                        // global
        const int32_t ql = h->loc[(size_t)q];          // local: >= 0 on the device
        const bool on_dev = ql >= 0;
        const bool apply = h->pivots < h->max_pivots;
        // the device list's slots before this pivot; slot L takes the leaving
        // column if it is a device column (else the zero column)
        const int32_t L = (int32_t)h->dl.size(), ns = L + 1;
        const unsigned sgrid = (unsigned)((ns + 255) / 256);
        auto queue_device_step3 = [&]() -> int {
            hipLaunchKernelGGL(k_hyb_stage, dim3(sgrid), dim3(256), 0, h->stream, h->dT, ld, ns,
                               (const int32_t *)h->dcols, (const DevState *)h->dst, h->dR);
            launch_device_update(h, ns);
            hipLaunchKernelGGL(k_hyb_price, dim3(1), dim3(1024), 0, h->stream, h->dT, ld, J, h->dparts,
                               device_parts(h, ns), 0, h->pin_min, h->seq + 1, sv);
            LP_HIP_CHECK(hipGetLastError());
            return LP_OK;
        };
        // Step 2 on the side that owns column q; F to the other side
        int32_t r = kNoIndex;
        int bad = 0;
        if (on_dev) {
            // the device arms its own Step 3 (and appends the leaving column
            // to its list) and queues it at once; the host waits only for F
            // and the pivot
            sv = ++h->seq_next;
            hipLaunchKernelGGL(k_hyb_ratio, dim3(1), dim3(1024), 0, h->stream, h->dT, ld, m, ql, J, h->eps_p,
                               (int32_t)apply, h->dF, h->F, h->pin_piv, h->dst, h->dcols, h->dbasis,
                               (const int32_t *)h->ddloc, q, h->rem_s, h->rem_v, L, h->seq, sv);
            LP_HIP_CHECK(hipGetLastError());
            h->rem_s = -1;
            if (int rc = queue_device_step3()) return rc;
            if (int rc = wait_seq(h, 0, sv)) return rc;
            r = h->pin_piv->r;
            bad = h->pin_piv->bad;
        } else {
            const double *colq = h->hT.data() + (int64_t)(-1 - ql) * ld;
            const double *rhs = h->hT.data() + (int64_t)h->nh * ld;
            double rv = __builtin_inf();
            h->F[0] = colq[0];
            for (int32_t i = 1; i <= m; ++i) {
                const double a = colq[i], bb = rhs[i];
                h->F[i] = a;
                if (host_step2_bad(a, bb)) {
                    bad = 1;
                } else if (a > h->eps_p) {
                    const double ratio = bb / a;
                    if (host_lex_less(ratio, i, rv, r)) {
                        rv = ratio;
                        r = i;
                    }
                }
            }
            if (!bad && r != kNoIndex && apply) {
                const int32_t lloc = h->loc[(size_t)h->basis[(size_t)r - 1]];
                h->pin_st->go = 1;
                h->pin_st->r = r;
                h->pin_st->p = h->F[r];
                LP_HIP_CHECK(hipMemcpyAsync(h->dF, h->F, ((size_t)m + 1) * sizeof(double), hipMemcpyHostToDevice,
                                            h->stream));
                LP_HIP_CHECK(hipMemcpyAsync(h->dst, h->pin_st, sizeof(DevState), hipMemcpyHostToDevice, h->stream));
                hipLaunchKernelGGL(k_hyb_relist, dim3(1), dim3(1), 0, h->stream, h->dcols, h->dbasis, h->rem_s,
                                   h->rem_v, L, lloc >= 0 ? lloc : zero_col, r, q);
                h->rem_s = -1;
                sv = ++h->seq_next;
                if (int rc = queue_device_step3()) return rc;
            }
        }
        if (bad) {
            h->status = LP_NUMERICAL;
            break;
        }
        if (r == kNoIndex) {
            h->status = LP_UNBOUNDED;
            break;
        }
        if (!apply) {
            h->status = LP_ITER_LIMIT;
            break;
        }
        const double p = h->F[r];
        const int32_t leave = h->basis[(size_t)r - 1];
        h->basis[(size_t)r - 1] = q;
        if (h->pivots < h->log_cap) {
            h->log_r[(size_t)h->pivots] = r;
            h->log_q[(size_t)h->pivots] = q;
        }
        h->pivots++;
        // the leaving column joins its side's list for this pivot's Step 3
        const int32_t lloc = h->loc[(size_t)leave];
        if (lloc >= 0) {
            h->dpos[(size_t)lloc] = L;
            h->dl.push_back(lloc);
        } else {
            h->hpos[(size_t)(-1 - lloc)] = (int32_t)h->hl.size();
            h->hl.push_back(-1 - lloc);
        }
        // Step 3 on the host's side while the device runs its own
        const auto th = std::chrono::steady_clock::now();
        hmin = host_pivot(h, pool, r, p);
        host_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - th).count();
        // the entering column leaves its side's list (on the device: written
        // before the next pivot's Step 3)
        auto drop = [](std::vector<int32_t> &list, std::vector<int32_t> &pos, int32_t c) {
            const int32_t s = pos[(size_t)c], last = list.back();
            list[(size_t)s] = last;
            pos[(size_t)last] = s;
            list.pop_back();
            pos[(size_t)c] = -1;
            return s < (int32_t)list.size() ? std::make_pair(s, last) : std::make_pair(-1, 0);
        };
        if (on_dev) {
            const auto w = drop(h->dl, h->dpos, ql);
            h->rem_s = w.first;
            h->rem_v = w.second;
        } else {
            (void)drop(h->hl, h->hpos, -1 - ql);
        }
        if (int rc = wait_seq(h, 1, sv)) return rc;
    }
    LP_HIP_CHECK(hipStreamSynchronize(h->stream));
    h->ran = true;
    h->host_ms = host_ms;
    h->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return LP_OK;
}

}  // namespace

extern "C" {

int lp_hybrid_create(lp_hybrid **out, int32_t m, int32_t n, const double *A, const double *b, const double *c,
                     double theta, int32_t host_threads, const lp_options *opt_in) {
    if (!out) return set_error(LP_E_INVAL, "out is NULL");
    *out = nullptr;
    if (m < 1 || n < 1 || !A || !b || !c) return set_error(LP_E_INVAL, "m, n must be >= 1 and inputs non-NULL");
    if (!(theta >= 0.0 && theta <= 1.0)) return set_error(LP_E_INVAL, "theta must be in [0, 1]");
    for (int64_t k = 0; k < (int64_t)m * n; ++k)
        if (!std::isfinite(A[k])) return set_error(LP_E_INVAL, "non-finite input");
    for (int32_t i = 0; i < m; ++i) {
        if (!std::isfinite(b[i])) return set_error(LP_E_INVAL, "non-finite input");
        if (b[i] < 0.0) return set_error(LP_E_NEG_RHS, "b has a negative entry: the slack basis is infeasible");
    }
    for (int32_t j = 0; j < n; ++j)
        if (!std::isfinite(c[j])) return set_error(LP_E_INVAL, "non-finite input");
    const Options o = resolve_options(opt_in);
    if (!(o.eps_dual >= 0.0) || !(o.eps_pivot >= 0.0) || !std::isfinite(o.eps_dual) || !std::isfinite(o.eps_pivot))
        return set_error(LP_E_INVAL, "eps_dual and eps_pivot must be finite and >= 0");
    if (o.bland_after != 0) return set_error(LP_E_INVAL, "the hybrid takes bland_after 0 only");
    int ndev = 0;
    LP_HIP_CHECK(hipGetDeviceCount(&ndev));
    if (o.device < 0 || o.device >= ndev) return set_error(LP_E_INVAL, "device ordinal out of range");
    lp_hybrid *h = new (std::nothrow) lp_hybrid;
    if (!h) return set_error(LP_E_NOMEM, "host allocation failed");
    h->device = o.device;
    DeviceGuard g(h->device);
    auto fail = [&](int rc) {
        free_hybrid(h);
        return rc;
    };
    const int64_t NM = (int64_t)n + m;
    h->m = m;
    h->n = n;
    h->ld = padded_ld(m);
    h->theta = theta;
    // the split: the first round(theta n) structural and round(theta m) slack
    // columns on the device (halves round up)
    const int32_t Jn = (int32_t)std::floor(theta * (double)n + 0.5), Jm = (int32_t)std::floor(theta * (double)m + 0.5);
    h->J = Jn + Jm;
    h->nh = (int32_t)(NM - h->J);
    try {
        h->loc.assign((size_t)NM, 0);
        for (int32_t g = 0; g < (int32_t)NM; ++g) {
            const bool dev = g < n ? g < Jn : g - n < Jm;
            if (dev) {
                h->loc[(size_t)g] = (int32_t)h->dglob.size();
                h->dglob.push_back(g);
            } else {
                h->loc[(size_t)g] = -1 - (int32_t)h->hglob.size();
                h->hglob.push_back(g);
            }
        }
    } catch (...) {
        return fail(set_error(LP_E_NOMEM, "host allocation failed"));
    }
    const unsigned hc = std::thread::hardware_concurrency();
    h->threads = host_threads > 0 ? host_threads : (int)std::min<unsigned>(hc ? hc : 1, 16);
    h->eps_d = o.eps_dual;
    h->eps_p = o.eps_pivot;
    h->max_pivots = o.max_pivots > 0 ? o.max_pivots : 50 * NM;
    h->log_cap = o.record_pivots ? h->max_pivots : 0;
    const int64_t nvec = ((int64_t)m + 2) / 2;
    h->block = nvec <= 64 ? 64 : (nvec <= 128 ? 128 : 256);
    h->cols = (h->block == 256 && nvec > 2048) ? 1 : 4;
    h->rowchunks = (int)((nvec + h->block - 1) / h->block);
    h->nparts = (int)(((int64_t)h->J + 2 + h->cols - 1) / h->cols);  // (the longest list: every column)
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess)
        return fail(set_error(LP_E_DEVICE, "hipStreamCreate failed"));

    auto dmalloc = [&](void **p, size_t bytes) -> int {
        if (hipMalloc(p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(LP_E_NOMEM, "hipMalloc failed");
        }
        return LP_OK;
    };
    const int64_t ld = h->ld, J = h->J;
    if (int rc = dmalloc((void **)&h->dT, (size_t)(ld * (J + 2)) * sizeof(double))) return fail(rc);
    if (int rc = dmalloc((void **)&h->dF, (size_t)ld * sizeof(double))) return fail(rc);
    if (int rc = dmalloc((void **)&h->dR, ((size_t)J + 2 + 4) * sizeof(double))) return fail(rc);
    if (int rc = dmalloc((void **)&h->dparts, ((size_t)h->nparts + 1) * sizeof(ArgMin))) return fail(rc);
    if (int rc = dmalloc((void **)&h->dst, sizeof(DevState))) return fail(rc);
    if (int rc = dmalloc((void **)&h->dcols, ((size_t)J + 2 + 4) * sizeof(int32_t))) return fail(rc);
    if (int rc = dmalloc((void **)&h->dbasis, (size_t)m * sizeof(int32_t))) return fail(rc);
    if (int rc = dmalloc((void **)&h->ddloc, (size_t)NM * sizeof(int32_t))) return fail(rc);
    // (mapped and coherent: the kernels store F, the Step 1 and 2 results and
    // the sequence words directly; the host reads them as they arrive)
    const unsigned hflags = hipHostMallocMapped | hipHostMallocCoherent;
    if (hipHostMalloc((void **)&h->F, (size_t)ld * sizeof(double), hflags) != hipSuccess ||
        hipHostMalloc((void **)&h->pin_min, sizeof(ArgMin), hflags) != hipSuccess ||
        hipHostMalloc((void **)&h->pin_piv, sizeof(HybPivot), hflags) != hipSuccess ||
        hipHostMalloc((void **)&h->seq, 2 * sizeof(uint32_t), hflags) != hipSuccess ||
        hipHostMalloc((void **)&h->pin_st, sizeof(DevState), hipHostMallocDefault) != hipSuccess)
        return fail(set_error(LP_E_NOMEM, "hipHostMalloc failed"));
    h->seq[0] = h->seq[1] = 0;
    std::memset(h->pin_st, 0, sizeof(DevState));
    h->pin_st->bar = (int32_t)J;  // the RHS (device column J) is no Step 1 candidate
    std::memset(h->F, 0, (size_t)ld * sizeof(double));
    // the lists at the slack basis: the RHS (device column J), then the
    // structural columns of each side
    try {
        h->dpos.assign((size_t)J, -1);
        h->hpos.assign((size_t)h->nh, -1);
        h->dl.push_back((int32_t)J);
        for (int32_t d = 0; d < (int32_t)J; ++d)
            if (h->dglob[(size_t)d] < n) {
                h->dpos[(size_t)d] = (int32_t)h->dl.size();
                h->dl.push_back(d);
            }
        for (int32_t k = 0; k < h->nh; ++k)
            if (h->hglob[(size_t)k] < n) {
                h->hpos[(size_t)k] = (int32_t)h->hl.size();
                h->hl.push_back(k);
            }
    } catch (...) {
        return fail(set_error(LP_E_NOMEM, "host allocation failed"));
    }
    std::vector<int32_t> cols((size_t)J + 2 + 4, 0);
    std::copy(h->dl.begin(), h->dl.end(), cols.begin());
    std::vector<int32_t> basis0((size_t)m), dloc0((size_t)NM);
    for (int32_t i = 0; i < m; ++i) basis0[(size_t)i] = n + i;
    for (int64_t g = 0; g < NM; ++g) dloc0[(size_t)g] = h->loc[(size_t)g] >= 0 ? h->loc[(size_t)g] : -1;
    // the host's share of Table I
    try {
        h->hT.assign((size_t)(ld * ((int64_t)h->nh + 1)), 0.0);
        h->basis.resize((size_t)m);
        h->log_r.resize((size_t)h->log_cap);
        h->log_q.resize((size_t)h->log_cap);
    } catch (...) {
        return fail(set_error(LP_E_NOMEM, "host allocation failed"));
    }
    for (int32_t k = 0; k < h->nh; ++k) {
        const int64_t j = h->hglob[(size_t)k];
        double *col = h->hT.data() + (int64_t)k * ld;
        if (j < n) {
            col[0] = -c[j];
            for (int32_t i = 1; i <= m; ++i) col[i] = A[(int64_t)(i - 1) * n + j];
        } else {
            col[j - n + 1] = 1.0;
        }
    }
    double *rhs = h->hT.data() + (int64_t)h->nh * ld;
    for (int32_t i = 1; i <= m; ++i) rhs[i] = b[i - 1];
    for (int32_t i = 0; i < m; ++i) h->basis[(size_t)i] = n + i;
    // the device's share, built from A, b, c on the device
    double *stage = nullptr;
    const size_t na = (size_t)m * n;
    const size_t nd = na + m + n;  // doubles, then the device's global column indices
    if (hipMalloc((void **)&stage, nd * sizeof(double) + ((size_t)J + 1) * sizeof(int32_t)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(set_error(LP_E_NOMEM, "hipMalloc (input staging) failed"));
    }
    int32_t *sglob = reinterpret_cast<int32_t *>(stage + nd);
    int rc = LP_OK;
    if (hipMemcpyAsync(stage, A, na * sizeof(double), hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        (J > 0 && hipMemcpyAsync(sglob, h->dglob.data(), (size_t)J * sizeof(int32_t), hipMemcpyHostToDevice,
                                 h->stream) != hipSuccess) ||
        hipMemcpyAsync(stage + na, b, (size_t)m * sizeof(double), hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(stage + na + m, c, (size_t)n * sizeof(double), hipMemcpyHostToDevice, h->stream) !=
            hipSuccess ||
        hipMemcpyAsync(h->dcols, cols.data(), cols.size() * sizeof(int32_t), hipMemcpyHostToDevice, h->stream) !=
            hipSuccess ||
        hipMemcpyAsync(h->dst, h->pin_st, sizeof(DevState), hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(h->dbasis, basis0.data(), (size_t)m * sizeof(int32_t), hipMemcpyHostToDevice, h->stream) !=
            hipSuccess ||
        hipMemcpyAsync(h->ddloc, dloc0.data(), (size_t)NM * sizeof(int32_t), hipMemcpyHostToDevice, h->stream) !=
            hipSuccess ||
        hipMemsetAsync(h->dF, 0, (size_t)ld * sizeof(double), h->stream) != hipSuccess ||
        hipMemsetAsync(h->dR, 0, ((size_t)J + 2 + 4) * sizeof(double), h->stream) != hipSuccess)
        rc = set_error(LP_E_DEVICE, "input copy failed");
    if (!rc) {
        const int64_t total = ld * (J + 2);
        hipLaunchKernelGGL(k_hyb_build, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 65536)), dim3(256), 0,
                           h->stream, h->dT, ld, m, n, (int32_t)J, (const int32_t *)sglob, stage, stage + na,
                           stage + na + m);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess)
            rc = set_error(LP_E_DEVICE, "build failed");
    }
    (void)hipFree(stage);
    if (rc) return fail(rc);
    *out = h;
    return LP_OK;
}

int lp_hybrid_solve(lp_hybrid *h) {
    if (!h) return set_error(LP_E_INVAL, "NULL handle");
    if (h->ran) return LP_OK;  // solved already
    return hybrid_solve(h);
}

int lp_hybrid_get_solution(const lp_hybrid *h, lp_result *res, double *x, double *y) {
    if (!h) return set_error(LP_E_INVAL, "NULL handle");
    if (!h->ran) return set_error(LP_E_STATE, "no solve has run on this handle");
    DeviceGuard g(h->device);
    const int64_t ld = h->ld;
    const int32_t m = h->m, n = h->n, J = h->J;
    const double *rhs = h->hT.data() + (int64_t)h->nh * ld;  // equal to the device's copy
    if (x) {
        for (int32_t j = 0; j < n; ++j) x[j] = 0.0;
        for (int32_t i = 1; i <= m; ++i)
            if (h->basis[(size_t)i - 1] < n) x[h->basis[(size_t)i - 1]] = rhs[i];
    }
    if (y) {
        // y_i = row 0 of slack column n+i-1, from the side that holds it
        std::vector<double> row0((size_t)J);
        if (J > 0)
            LP_HIP_CHECK(hipMemcpy2D(row0.data(), sizeof(double), h->dT, (size_t)ld * sizeof(double), sizeof(double),
                                     (size_t)J, hipMemcpyDeviceToHost));
        for (int32_t i = 1; i <= m; ++i) {
            const int32_t l = h->loc[(size_t)n + i - 1];
            y[i - 1] = l >= 0 ? row0[(size_t)l] : h->hT[(size_t)(-1 - l) * ld];
        }
    }
    if (res) {
        res->status = h->status;
        res->reserved = 0;
        res->pivots = h->pivots;
        res->objective = rhs[0];
        res->solve_ms = h->solve_ms;
    }
    return LP_OK;
}

int lp_hybrid_get_pivots(const lp_hybrid *h, int32_t *rows, int32_t *cols, int64_t cap, int64_t *count) {
    if (!h || cap < 0 || (cap > 0 && (!rows || !cols))) return set_error(LP_E_INVAL, "bad argument");
    if (count) *count = h->pivots;
    const int64_t k = std::min<int64_t>(std::min<int64_t>(h->pivots, h->log_cap), cap);
    if (k > 0) {
        std::memcpy(rows, h->log_r.data(), (size_t)k * sizeof(int32_t));
        std::memcpy(cols, h->log_q.data(), (size_t)k * sizeof(int32_t));
    }
    return LP_OK;
}

int lp_hybrid_get_tableau(const lp_hybrid *h, double *out) {
    if (!h || !out) return set_error(LP_E_INVAL, "NULL argument");
    DeviceGuard g(h->device);
    const int64_t ld = h->ld, rows = (int64_t)h->m + 1, NM = (int64_t)h->n + h->m;
    const int32_t J = h->J;
    // the device's columns and its copy of the RHS (its column J), then
    // every column to its global place
    std::vector<double> dev((size_t)(rows * ((int64_t)J + 1)));
    LP_HIP_CHECK(hipMemcpy2D(dev.data(), (size_t)rows * sizeof(double), h->dT, (size_t)ld * sizeof(double),
                             (size_t)rows * sizeof(double), (size_t)J + 1, hipMemcpyDeviceToHost));
    for (int64_t gcol = 0; gcol < NM; ++gcol) {
        const int32_t l = h->loc[(size_t)gcol];
        const double *src = l >= 0 ? dev.data() + (int64_t)l * rows : h->hT.data() + (int64_t)(-1 - l) * ld;
        std::memcpy(out + gcol * rows, src, (size_t)rows * sizeof(double));
    }
    std::memcpy(out + NM * rows, dev.data() + (int64_t)J * rows, (size_t)rows * sizeof(double));
    return LP_OK;
}

int lp_hybrid_info(const lp_hybrid *h, int32_t *device_columns, int32_t *host_columns, int32_t *host_threads,
                   double *host_ms) {
    if (!h) return set_error(LP_E_INVAL, "NULL handle");
    if (device_columns) *device_columns = h->J;
    if (host_columns) *host_columns = h->nh;
    if (host_threads) *host_threads = h->threads;
    if (host_ms) *host_ms = h->host_ms;
    return LP_OK;
}

void lp_hybrid_destroy(lp_hybrid *h) { free_hybrid(h); }

}  // extern "C"
