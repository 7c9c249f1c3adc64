// Kernels of the batched solver: many independent LPs, each advanced pivot
// by pivot (Steps 1-3 of Section III) by one workgroup of a persistent kernel.
//
// Workgroups take LPs off a device queue (an atomic counter over an order
// array, largest LP first). A workgroup runs its LP for at most `budget`
// pivots, then takes the next one, so a launch always ends; an LP left
// RUNNING continues in the next launch. Nothing waits on another workgroup,
// except the parts of a split LP (below), which wait only for each other.
//
// Within a workgroup one pivot is:
//   Step 1  argmin over the nonbasic columns' row-0 entries (reduced while
//           the previous pivot's update wrote them, or by a scan on entry);
//   Step 2  ratio test over column q (block argmin);
//   Step 3  F = column q and R = normalised pivot row (by rewrite-list
//           position) staged in LDS, then the rewrite of every listed column.
// The rewrite list (nonbasic columns, the entering column, the RHS) and its
// maintenance are the same as the single-LP solver's; the arithmetic of every
// entry is identical, so each LP follows the single-LP pivot sequence.
#pragma once

#include "common.hpp"

namespace lpgpu {

struct BatchSync;

struct BatchDesc {
    double *T;          // column-major tableau, T[i][j] = T[j*ld + i]
    int64_t ld;         // padded rows (multiple of 16)
    int32_t m, n;
    int32_t *basis;     // m
    int32_t *cols;      // n+2: nonbasic columns, entering column, RHS
    int32_t *pos;       // n+m: position in cols[0..n) or -1
    int32_t *log_r;     // log_cap
    int32_t *log_q;
    int64_t log_cap;
    uint64_t magic;     // ceil(2^36 / nvec): item -> (column, row pair) split
    int32_t nvec;       // (m+2)/2 row pairs per column
    int32_t pad;
    double *scratch;    // NULL: F, R and the list live in LDS; else in this global area
    BatchSync *sync;    // the parts' meeting area of a split LP (else NULL)
};

// A split LP: its W parts (W <= kMaxBatchParts queue entries, taken by W
// workgroups at once) share its rewrite list, part p rewriting the slots
// p*S .. p*S+S-1 (S = ceil((n+2)/W)). Per pivot they meet twice: after the
// Step 1 partials of their slots (exchanged with the meeting, each part then
// reduces all W) and after every part has read what the pivot's other parts
// rewrite (column q, the RHS, the list, the basis). Step 2 and the Step 3
// inputs run in every part (the same values, so the same pivot). A meeting
// carries its data like the decision kernel's grid barrier: per part one
// 128-byte record line of 64-bit words, 32 data bits and a flag (the LP's
// meeting count) each. A turn starts with a check-in gate, as the decision
// kernel's: if the W parts are not all running within the gate's limit,
// the workgroup that closes the gate runs the LP alone (the other parts
// leave), so no part ever waits for a workgroup that is not running.
constexpr int kMaxBatchParts = 8;
constexpr uint32_t kPartGateClosed = 0x80000000u;
struct BatchSync {
    uint32_t gate;   // parts arrived this turn, kPartGateClosed once closed
    uint32_t exits;  // parts that left this turn
    uint32_t seq;    // meetings of this LP so far (every turn)
    uint32_t pad[29];
    uint64_t rec[2][kMaxBatchParts][16];  // [Step 1 partials | reads done][part][word]
};

struct BatchState {
    int32_t status;
    int32_t pad;
    int64_t pivots;
    int64_t max_pivots;
    int64_t cols_done;  // rewritten columns (nonzero R), summed over pivots
    double eps_d, eps_p;
};

// Quotient by nvec of item < 2^24 with nvec < 2^12: exact, since
// item * nvec < 2^36 (Granlund-Montgomery with a rounded-up reciprocal).
__device__ __forceinline__ uint32_t div_nvec(uint32_t item, uint64_t magic) {
    return (uint32_t)(((uint64_t)item * magic) >> 36);
}

template <int BT>
__device__ __forceinline__ void batch_block_argmin(double &v, int32_t &i, double *sv, int32_t *si) {
    wave_argmin(v, i);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int nw = BT / 64;
    __syncthreads();
    if (lane == 0) {
        sv[wave] = v;
        si[wave] = i;
    }
    __syncthreads();
    v = lane < nw ? sv[lane] : __builtin_inf();
    i = lane < nw ? si[lane] : kNoIndex;
    wave_argmin(v, i);
}

// One LP, at most `budget` pivots. `work` holds F (2*nvec doubles), R (n+2
// doubles) and the rewrite list (n+2 int32): the workgroup's LDS, or the
// LP's global scratch area when they do not fit in LDS.
template <int BT, int U>
__device__ __forceinline__ void batch_solve_one(const BatchDesc &d, BatchState *__restrict__ stp, double *work,
                                                double *sv, int32_t *si, int32_t *sint, int64_t budget) {
    const int tid = threadIdx.x;
    BatchState s = *stp;
    if (s.status != LP_RUNNING) return;
    const int32_t m = d.m, n = d.n;
    const int64_t ld = d.ld;
    const int64_t W = (int64_t)n + m + 1;
    const int32_t nvec = d.nvec;
    double *T = d.T;
    double *F = work;                                        // 2*nvec
    double *R = work + 2 * (int64_t)nvec;                    // n+2
    int32_t *L = reinterpret_cast<int32_t *>(R + n + 2);     // n+2

    // Step 1 on entry: scan the nonbasic columns' row-0 entries.
    double v = __builtin_inf();
    int32_t q = kNoIndex;
    for (int32_t t = tid; t < n; t += BT) {
        const int32_t j = d.cols[t];
        const double x = T[(int64_t)j * ld];
        if (lex_less(x, j, v, q)) {
            v = x;
            q = j;
        }
    }
    batch_block_argmin<BT>(v, q, sv, si);

    int64_t done = 0;
    int32_t status = LP_RUNNING;
    int64_t cols_done = 0;
    for (;;) {
        if (step1_bad(v)) {
            status = LP_NUMERICAL;
            break;
        }
        if (v >= -s.eps_d) {
            status = LP_OPTIMAL;
            break;
        }
        if (done >= budget) break;

        // Step 2.
        const double *colq = T + (int64_t)q * ld;
        const double *rhs = T + (W - 1) * ld;
        double rv = __builtin_inf();
        int32_t r = kNoIndex;
        int bad = 0;
        for (int32_t i = 1 + tid; i <= m; i += BT) {
            const double a = colq[i], bb = rhs[i];
            if (step2_bad(a, bb)) {
                bad = 1;
            } else if (a > s.eps_p) {
                const double ratio = bb / a;
                if (lex_less(ratio, i, rv, r)) {
                    rv = ratio;
                    r = i;
                }
            }
        }
        bad = __syncthreads_or(bad);
        batch_block_argmin<BT>(rv, r, sv, si);
        if (bad) {
            status = LP_NUMERICAL;
            break;
        }
        if (r == kNoIndex) {
            status = LP_UNBOUNDED;
            break;
        }
        if (s.pivots >= s.max_pivots) {
            status = LP_ITER_LIMIT;
            break;
        }

        // Step 3 inputs in LDS.
        const double p = colq[r];
        const int32_t leave = d.basis[r - 1];
        const int32_t pq = d.pos[q];
        for (int32_t i = tid; i < 2 * nvec; i += BT) F[i] = i <= m ? colq[i] : 0.0;
        int32_t nz = 0;
        for (int32_t t = tid; t < n + 2; t += BT) {
            const int32_t j = t == pq ? leave : (t == n ? q : d.cols[t]);
            const double Rt = T[(int64_t)j * ld + r] / p;
            R[t] = Rt;
            L[t] = j;
            nz += Rt != 0.0;
        }
        nz = wave_sum_i32(nz);
        if ((tid & 63) == 0) sint[tid >> 6] = nz;
        __syncthreads();  // F, R, L ready; every read of cols/pos/basis done
        if (tid == 0) {
            int32_t tot = 0;
            for (int w = 0; w < BT / 64; ++w) tot += sint[w];
            cols_done += tot;
            d.cols[pq] = leave;
            d.pos[leave] = pq;
            d.pos[q] = -1;
            d.cols[n] = q;
            d.basis[r - 1] = q;
            if (s.pivots < d.log_cap) {
                d.log_r[s.pivots] = r;
                d.log_q[s.pivots] = q;
            }
        }
        s.pivots += 1;
        done += 1;

        // Step 3: rewrite every listed column; items are (column, row pair),
        // row pairs fastest so that a wave reads contiguous memory.
        const uint32_t items = (uint32_t)(n + 2) * (uint32_t)nvec;
        const double2 *F2 = reinterpret_cast<const double2 *>(F);
        double bestv = __builtin_inf();
        int32_t bestj = kNoIndex;
        const int32_t rhs_col = (int32_t)(W - 1);
        auto rewrite = [&](uint32_t c, uint32_t vr, double2 *a, const double2 xx) {
            const double Rt = R[c];
            const double2 f = F2[vr];
            const int32_t row = 2 * (int32_t)vr;
            double2 y;
            y.x = (row == r) ? Rt : fma(-f.x, Rt, xx.x);
            y.y = (row + 1 == r) ? Rt : fma(-f.y, Rt, xx.y);
            *a = y;
            if (vr == 0) {  // row 0: candidate of the next Step 1
                const int32_t j = L[c];
                if (j != rhs_col && lex_less(y.x, j, bestv, bestj)) {
                    bestv = y.x;
                    bestj = j;
                }
            }
        };
        uint32_t base = tid;
        // full rounds: U items per thread, all loads issued before any store
        for (; base + (uint32_t)(U - 1) * BT < items; base += (uint32_t)BT * U) {
            double2 x[U];
            double2 *addr[U];
            uint32_t vv[U], cc[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t it = base + (uint32_t)u * BT;
                cc[u] = div_nvec(it, d.magic);
                vv[u] = it - cc[u] * (uint32_t)nvec;
                addr[u] = reinterpret_cast<double2 *>(T + (int64_t)L[cc[u]] * ld) + vv[u];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) x[u] = *addr[u];
#pragma unroll
            for (int u = 0; u < U; ++u) rewrite(cc[u], vv[u], addr[u], x[u]);
        }
        // tail: fewer than U items left for this thread
        for (; base < items; base += (uint32_t)BT) {
            const uint32_t c = div_nvec(base, d.magic);
            const uint32_t vr = base - c * (uint32_t)nvec;
            double2 *a = reinterpret_cast<double2 *>(T + (int64_t)L[c] * ld) + vr;
            rewrite(c, vr, a, *a);
        }
        // next Step 1 from the new row-0 entries; the barriers inside also
        // order this pivot's writes before the next pivot's reads
        batch_block_argmin<BT>(bestv, bestj, sv, si);
        v = bestv;
        q = bestj;
    }
    if (tid == 0) {
        stp->status = status;
        stp->pivots = s.pivots;
        stp->cols_done = s.cols_done + cols_done;
    }
    __syncthreads();
}

constexpr uint32_t kPartGateSpin = 1u << 16;  // gate polls before closing (about 0.1 s)
constexpr uint32_t kPartMeetSpin = 1u << 22;  // meeting polls before the LP is given up as stalled (seconds)

enum PartMode : int32_t { kPartSkip = 0, kPartSplit = 1, kPartSolo = 2 };

// The check-in gate of a split LP's turn: every part adds one and waits for
// W; one that polls past the limit (gate_spin, kPartGateSpin by default; 0
// closes every gate at once, a test of the fallback) closes the gate with a compare-and-swap
// of the count it last read (which fails if a part arrived meanwhile), and
// runs the LP alone; parts that find the gate closed leave. Nothing is
// written before the gate.
__device__ __forceinline__ int32_t part_gate(BatchSync *sy, int W, uint32_t gate_spin, int32_t *s_mode) {
    if (threadIdx.x == 0) {
        uint32_t v = atomicAdd(&sy->gate, 1u) + 1u, it = 0;
        int32_t mode;
        for (;;) {
            if (v & kPartGateClosed) {
                mode = kPartSkip;
                break;
            }
            if (v == (uint32_t)W) {
                mode = kPartSplit;
                break;
            }
            if (++it > gate_spin) {
                const uint32_t old = atomicCAS(&sy->gate, v, v | kPartGateClosed);
                if (old == v) {
                    mode = kPartSolo;
                    break;
                }
                v = old;
                continue;
            }
            __builtin_amdgcn_s_sleep(2);
            v = __hip_atomic_load(&sy->gate, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_mode = mode;
    }
    __syncthreads();
    return *s_mode;
}

// Every part that took a queue entry of the LP leaves through here (W per
// turn); the last one reopens the gate for the next turn.
__device__ __forceinline__ void part_leave(BatchSync *sy, int W) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&sy->exits, 1u) == (uint32_t)W - 1u) {
            sy->exits = 0;
            sy->gate = 0;
            __threadfence();
        }
    }
}

// A meeting of the W parts: thread 0 publishes this part's N words (after
// the workgroup barrier that ends the work they follow), wave 0 polls the W
// records until each word carries the flag and copies the data to xs.
// Returns false if the wait ran out (the LP is then marked LP_STALLED).
template <int N>
__device__ __forceinline__ bool part_meet(BatchSync *sy, int b, int part, int W, uint32_t flag, const uint32_t *d,
                                          uint32_t (*xs)[N], int32_t *s_ok) {
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
#pragma unroll
        for (int k = 0; k < N; ++k)
            __hip_atomic_store(&sy->rec[b][part][k], ((uint64_t)flag << 32) | d[k], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        uint64_t a[N];
        uint32_t it = 0;
        bool ok = false;
        for (;;) {
            bool mine = true;
            if (lane < W) {
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    a[k] = __hip_atomic_load(&sy->rec[b][lane][k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    mine &= (uint32_t)(a[k] >> 32) == flag;
                }
            }
            if (__ballot(!mine) == 0) {
                ok = true;
                break;
            }
            if (++it > kPartMeetSpin) break;
            __builtin_amdgcn_s_sleep(1);
        }
        if (ok) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if (lane < W) {
#pragma unroll
                for (int k = 0; k < N; ++k) xs[lane][k] = (uint32_t)a[k];
            }
        }
        if (lane == 0) *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

// The winner of the W parts' Step 1 partials (xs[p] = value bits, column).
__device__ __forceinline__ void part_step1(const uint32_t (*xs)[3], int W, double &v, int32_t &q) {
    v = __builtin_inf();
    q = kNoIndex;
    for (int p = 0; p < W; ++p) {
        const double pv = __hiloint2double((int32_t)xs[p][1], (int32_t)xs[p][0]);
        const int32_t pj = (int32_t)xs[p][2];
        if (lex_less(pv, pj, v, q)) {
            v = pv;
            q = pj;
        }
    }
}

// Part `part` of W of one LP, at most `budget` pivots: the same Steps as
// batch_solve_one with the rewrite (and the Step 1 partials) over the
// part's slots t0 .. t1-1 only. `work` holds F (2*nvec doubles), then R and
// the slots' columns for the part's S slots.
template <int BT, int U>
__device__ __forceinline__ void batch_solve_part(const BatchDesc &d, BatchState *__restrict__ stp, double *work,
                                                 double *sv, int32_t *si, int32_t *sint, int64_t budget, int part,
                                                 int W) {
    __shared__ uint32_t xs1[kMaxBatchParts][3];
    __shared__ uint32_t xs2[kMaxBatchParts][1];
    __shared__ int32_t s_ok;
    BatchSync *sy = d.sync;
    const int tid = threadIdx.x;
    BatchState s = *stp;
    if (s.status != LP_RUNNING) return;
    const int32_t m = d.m, n = d.n;
    const int64_t ld = d.ld;
    const int64_t Wc = (int64_t)n + m + 1;
    const int32_t nvec = d.nvec;
    const int32_t S = (n + 2 + W - 1) / W;
    const int32_t t0 = part * S, t1 = min(n + 2, t0 + S), ns = max(0, t1 - t0);
    double *T = d.T;
    double *F = work;                                    // 2*nvec
    double *R = work + 2 * (int64_t)nvec;                // S
    int32_t *L = reinterpret_cast<int32_t *>(R + S);     // S
    uint32_t seq = sy->seq;

    // Step 1 on entry over the part's nonbasic slots
    double v = __builtin_inf();
    int32_t q = kNoIndex;
    for (int32_t t = t0 + tid; t < min(t1, n); t += BT) {
        const int32_t j = d.cols[t];
        const double x = T[(int64_t)j * ld];
        if (lex_less(x, j, v, q)) {
            v = x;
            q = j;
        }
    }
    batch_block_argmin<BT>(v, q, sv, si);
    bool alive = true;
    {
        const uint32_t dd[3] = {(uint32_t)__double2loint(v), (uint32_t)__double2hiint(v), (uint32_t)q};
        alive = part_meet<3>(sy, 0, part, W, ++seq, dd, xs1, &s_ok);
        if (alive) part_step1(xs1, W, v, q);
    }

    int64_t done = 0;
    int32_t status = alive ? LP_RUNNING : LP_STALLED;
    int64_t cols_done = 0;
    while (alive) {
        if (step1_bad(v)) {
            status = LP_NUMERICAL;
            break;
        }
        if (v >= -s.eps_d) {
            status = LP_OPTIMAL;
            break;
        }
        if (done >= budget) break;

        // Step 2, in every part over all rows.
        const double *colq = T + (int64_t)q * ld;
        const double *rhs = T + (Wc - 1) * ld;
        double rv = __builtin_inf();
        int32_t r = kNoIndex;
        int bad = 0;
        for (int32_t i = 1 + tid; i <= m; i += BT) {
            const double a = colq[i], bb = rhs[i];
            if (step2_bad(a, bb)) {
                bad = 1;
            } else if (a > s.eps_p) {
                const double ratio = bb / a;
                if (lex_less(ratio, i, rv, r)) {
                    rv = ratio;
                    r = i;
                }
            }
        }
        bad = __syncthreads_or(bad);
        batch_block_argmin<BT>(rv, r, sv, si);
        if (bad) {
            status = LP_NUMERICAL;
            break;
        }
        if (r == kNoIndex) {
            status = LP_UNBOUNDED;
            break;
        }
        if (s.pivots >= s.max_pivots) {
            status = LP_ITER_LIMIT;
            break;
        }

        // Step 3 inputs: F whole, R and the columns of the part's slots.
        const double p = colq[r];
        const int32_t leave = d.basis[r - 1];
        const int32_t pq = d.pos[q];
        for (int32_t i = tid; i < 2 * nvec; i += BT) F[i] = i <= m ? colq[i] : 0.0;
        int32_t nz = 0;
        for (int32_t c = tid; c < ns; c += BT) {
            const int32_t t = t0 + c;
            const int32_t j = t == pq ? leave : (t == n ? q : d.cols[t]);
            const double Rt = T[(int64_t)j * ld + r] / p;
            R[c] = Rt;
            L[c] = j;
            nz += Rt != 0.0;
        }
        nz = wave_sum_i32(nz);
        if ((tid & 63) == 0) sint[tid >> 6] = nz;
        __syncthreads();  // F, R, L ready; this part's reads of the shared columns and lists done
        if (tid == 0) {
            int32_t tot = 0;
            for (int w = 0; w < BT / 64; ++w) tot += sint[w];
            cols_done += tot;
        }
        // every part has read column q, the RHS, the list and the basis
        // before any part rewrites them
        {
            const uint32_t dd[1] = {0u};
            if (!part_meet<1>(sy, 1, part, W, ++seq, dd, xs2, &s_ok)) {
                status = LP_STALLED;
                break;
            }
        }
        if (part == 0 && tid == 0) {
            d.cols[pq] = leave;
            d.pos[leave] = pq;
            d.pos[q] = -1;
            d.cols[n] = q;
            d.basis[r - 1] = q;
            if (s.pivots < d.log_cap) {
                d.log_r[s.pivots] = r;
                d.log_q[s.pivots] = q;
            }
        }
        s.pivots += 1;
        done += 1;

        // Step 3 over the part's slots (items: (slot, row pair), row pairs
        // fastest)
        const uint32_t items = (uint32_t)ns * (uint32_t)nvec;
        const double2 *F2 = reinterpret_cast<const double2 *>(F);
        double bestv = __builtin_inf();
        int32_t bestj = kNoIndex;
        const int32_t rhs_col = (int32_t)(Wc - 1);
        auto rewrite = [&](uint32_t c, uint32_t vr, double2 *a, const double2 xx) {
            const double Rt = R[c];
            const double2 f = F2[vr];
            const int32_t row = 2 * (int32_t)vr;
            double2 y;
            y.x = (row == r) ? Rt : fma(-f.x, Rt, xx.x);
            y.y = (row + 1 == r) ? Rt : fma(-f.y, Rt, xx.y);
            *a = y;
            if (vr == 0) {
                const int32_t j = L[c];
                if (j != rhs_col && lex_less(y.x, j, bestv, bestj)) {
                    bestv = y.x;
                    bestj = j;
                }
            }
        };
        uint32_t base = tid;
        for (; base + (uint32_t)(U - 1) * BT < items; base += (uint32_t)BT * U) {
            double2 x[U];
            double2 *addr[U];
            uint32_t vv[U], cc[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t it = base + (uint32_t)u * BT;
                cc[u] = div_nvec(it, d.magic);
                vv[u] = it - cc[u] * (uint32_t)nvec;
                addr[u] = reinterpret_cast<double2 *>(T + (int64_t)L[cc[u]] * ld) + vv[u];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) x[u] = *addr[u];
#pragma unroll
            for (int u = 0; u < U; ++u) rewrite(cc[u], vv[u], addr[u], x[u]);
        }
        for (; base < items; base += (uint32_t)BT) {
            const uint32_t c = div_nvec(base, d.magic);
            const uint32_t vr = base - c * (uint32_t)nvec;
            double2 *a = reinterpret_cast<double2 *>(T + (int64_t)L[c] * ld) + vr;
            rewrite(c, vr, a, *a);
        }
        // the next Step 1: this part's partial (its barriers order the
        // rewrite before the meeting), then all W
        batch_block_argmin<BT>(bestv, bestj, sv, si);
        const uint32_t dd[3] = {(uint32_t)__double2loint(bestv), (uint32_t)__double2hiint(bestv), (uint32_t)bestj};
        if (!part_meet<3>(sy, 0, part, W, ++seq, dd, xs1, &s_ok)) {
            status = LP_STALLED;
            break;
        }
        part_step1(xs1, W, v, q);
    }
    __syncthreads();
    if (tid == 0) {
        if (part == 0) {
            stp->status = status;
            stp->pivots = s.pivots;
            sy->seq = seq;
        } else if (status == LP_STALLED) {
            atomicExch(&stp->status, (int32_t)LP_STALLED);
        }
        atomicAdd(reinterpret_cast<unsigned long long *>(&stp->cols_done), (unsigned long long)cols_done);
    }
    __syncthreads();
}

// Opens every split LP's gate (a solve abandoned in a turn can leave it
// closed); the meeting counts carry on.
static __global__ void k_batch_sync_reset(BatchSync *sync, int32_t count) {
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) {
        sync[k].gate = 0;
        sync[k].exits = 0;
    }
}

// Resets the queue head; launched before every k_batch in the graph.
static __global__ void k_batch_reset(int32_t *head) { *head = 0; }

// The queue: entry idx names LP order[idx]; with `parts` (else NULL: every
// LP whole), parts[idx] = (W << 8) | p names part p of W of a split LP.
template <int BT, int U>
__global__ __launch_bounds__(BT) void k_batch(const BatchDesc *__restrict__ desc, BatchState *__restrict__ state,
                                              const int32_t *__restrict__ order, const int32_t *__restrict__ norder,
                                              int32_t *__restrict__ head, int64_t budget,
                                              const int32_t *__restrict__ parts, uint32_t gate_spin) {
    extern __shared__ double lds[];
    __shared__ double sv[BT / 64];
    __shared__ int32_t si[BT / 64];
    __shared__ int32_t sint[BT / 64];
    __shared__ int32_t s_idx, s_mode;
    const int32_t count = *norder;
    for (;;) {
        if (threadIdx.x == 0) s_idx = atomicAdd(head, 1);
        __syncthreads();
        const int32_t idx = s_idx;
        __syncthreads();
        if (idx >= count) return;
        const int32_t k = order[idx];
        const BatchDesc d = desc[k];
        const int32_t pw = parts ? parts[idx] : 0;
        const int W = pw >> 8;
        if (W > 1) {  // a part of a split LP (its work area always in LDS)
            if (!d.sync) {  // (no meeting area: its first part runs it whole)
                if ((pw & 0xff) == 0) batch_solve_one<BT, U>(d, state + k, lds, sv, si, sint, budget);
                continue;
            }
            const int32_t mode = part_gate(d.sync, W, gate_spin, &s_mode);
            if (mode == kPartSplit)
                batch_solve_part<BT, U>(d, state + k, lds, sv, si, sint, budget, pw & 0xff, W);
            else if (mode == kPartSolo)
                batch_solve_one<BT, U>(d, state + k, lds, sv, si, sint, budget);
            part_leave(d.sync, W);
        } else if (d.scratch) {
            batch_solve_one<BT, U>(d, state + k, d.scratch, sv, si, sint, budget);
        } else {
            batch_solve_one<BT, U>(d, state + k, lds, sv, si, sint, budget);
        }
    }
}

// Initialization Step of every LP of a batch in one launch. The tiles of all
// tableaux are numbered consecutively: LP k owns tiles [first[k], first[k+1]);
// its first ceil(n/64)*rt tiles transpose 64x64 blocks of its row-major A
// (with -c in row 0) through LDS, the next ceil((m+1)/64)*rt fill the slack
// identity and the RHS; rt = ceil(ld/64) row tiles per column.
static __global__ __launch_bounds__(256) void k_batch_build(const BatchDesc *__restrict__ desc,
                                                            const double *__restrict__ inputs,
                                                            const int64_t *__restrict__ in_off,
                                                            const int32_t *__restrict__ tile_lp,
                                                            const int64_t *__restrict__ first) {
    __shared__ double tile[64][65];
    const int32_t k = tile_lp[blockIdx.x];
    const BatchDesc d = desc[k];
    const int64_t local = (int64_t)blockIdx.x - first[k];
    const int32_t m = d.m, n = d.n;
    const int64_t ld = d.ld;
    const int64_t rt = (ld + 63) / 64;
    const int64_t ns = (int64_t)((n + 63) / 64) * rt;
    const double *A = inputs + in_off[k];
    const double *b = A + (int64_t)m * n;
    const double *c = b + m;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    if (local < ns) {
        const int64_t j0 = (local / rt) * 64, i0 = (local % rt) * 64;
        for (int q = 0; q < 16; ++q) {
            const int64_t i = i0 + ty + 4 * q, j = j0 + tx;
            double v = 0.0;
            if (j < n) {
                if (i == 0)
                    v = -c[j];
                else if (i <= m)
                    v = A[(i - 1) * n + j];
            }
            tile[ty + 4 * q][tx] = v;
        }
        __syncthreads();
        for (int q = 0; q < 16; ++q) {
            const int64_t j = j0 + ty + 4 * q, i = i0 + tx;
            if (j < n && i < ld) d.T[j * ld + i] = tile[tx][ty + 4 * q];
        }
    } else {
        const int64_t l2 = local - ns;
        const int64_t s0 = (l2 / rt) * 64, i0 = (l2 % rt) * 64;
        for (int q = 0; q < 16; ++q) {
            const int64_t s = s0 + ty + 4 * q, i = i0 + tx;  // column n+s, row i
            if (s > m || i >= ld) continue;
            double v;
            if (s < m)
                v = (i == s + 1) ? 1.0 : 0.0;
            else
                v = (i >= 1 && i <= m) ? b[i - 1] : 0.0;
            d.T[(n + s) * ld + i] = v;
        }
    }
}

// Rewrite lists, positions and bases of every LP: workgroup k takes LP k.
static __global__ __launch_bounds__(256) void k_batch_init_all(const BatchDesc *__restrict__ desc) {
    const BatchDesc d = desc[blockIdx.x];
    const int32_t m = d.m, n = d.n;
    if (threadIdx.x == 0) {
        d.cols[n] = 0;
        d.cols[n + 1] = n + m;
    }
    for (int32_t t = threadIdx.x; t < n + m; t += blockDim.x) {
        if (t < m) d.basis[t] = n + t;
        if (t < n) d.cols[t] = t;
        d.pos[t] = t < n ? t : -1;
    }
}

// Initial rewrite list, positions, basis and state of one LP (grid-stride).
static __global__ void k_batch_init_lp(BatchDesc d, BatchState *st, BatchState init) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t m = d.m, n = d.n;
    if (t0 == 0) {
        *st = init;
        d.cols[n] = 0;
        d.cols[n + 1] = n + m;
    }
    for (int64_t t = t0; t < (int64_t)n + m; t += stride) {
        if (t < m) d.basis[t] = n + (int32_t)t;
        if (t < n) d.cols[t] = (int32_t)t;
        d.pos[t] = t < n ? (int32_t)t : -1;
    }
}

// Finalization for every LP: out + off[k] receives x (n), y (m), objective.
static __global__ __launch_bounds__(256) void k_batch_extract(const BatchDesc *__restrict__ desc,
                                                       const int64_t *__restrict__ off, double *__restrict__ out) {
    const BatchDesc d = desc[blockIdx.x];
    double *o = out + off[blockIdx.x];
    const int32_t m = d.m, n = d.n;
    const int64_t W = (int64_t)n + m + 1;
    for (int32_t j = threadIdx.x; j < n; j += blockDim.x) o[j] = 0.0;
    __syncthreads();
    for (int32_t i = 1 + threadIdx.x; i <= m; i += blockDim.x) {
        const int32_t bv = d.basis[i - 1];
        if (bv < n) o[bv] = d.T[(W - 1) * d.ld + i];
        o[n + i - 1] = d.T[((int64_t)n + i - 1) * d.ld];
    }
    if (threadIdx.x == 0) o[n + m] = d.T[(W - 1) * d.ld];
}

}  // namespace lpgpu
