// Kernels of the single-LP solver with pivot fusion: a group of up to K
// consecutive pivots is decided first and then applied to the tableau in ONE
// streaming pass, so each entry is read and written once per group instead
// of once per pivot.
//
// Why the decisions do not need the intermediate tableaux: Steps 1 and 2 of
// pivot j (0-based inside the group) read only row 0, column q_j and the RHS
// column of T^(j) (the tableau after the first j pivots of the group), and
// Step 3 of pivot j reads only its pivot row r_j and its pivot column. Every
// one of those vectors is obtained from T^(0) by replaying the j earlier
// rank-1 updates on that vector alone:
//     x <- R_k[t]                         if the row is r_k,
//     x <- fma(-F_k[i], R_k[t], x)        otherwise,            k = 0 .. j-1,
// which are exactly the operations, in the same order, that the sequential
// method performs on those entries. The pass that finally rewrites a column
// applies the same chain to every entry, so the tableau after the group is
// bit-identical to the one the sequential method produces, and so is every
// decision.
//
// The list of the group. Slots 0..n-1 hold the nonbasic columns at the start
// of the group (any order), slot n the RHS column, slots n+1 .. n+K the
// columns that leave the basis during the group (appended when they leave,
// -1 when unused). pos[c] is the slot of column c, or -1. Columns that are
// basic during the whole group are exact unit vectors that no pivot of the
// group changes (their pivot-row entry is 0), so they are left out; a basic
// column is stored only once it has left the basis (after a deferred build
// the slack columns are not written until then). A
// column's slot t indexes R_k[t] (the normalised pivot-row entry of pivot k)
// and D[t] (its row-0 entry after the pivots staged so far).
//
// Launches per group, on one stream. The default path (at most
// kMaxDecideWgs decision workgroups):
//   k_gdecide        all the group's decisions in one launch (grid barriers),
//                    the close of the previous group, and the pivot rows after
//                    the group (PV);
//   k_gupdate_pure   applies the group's pivots to every list column, the
//                    chain without the pivot-row select;
//   k_gfix           stores the pivot rows from PV.
// The first group after a deferred build runs k_gdecide<.., true, ..> (reading
// A and c) and k_gfirst (the build of the structural columns with the group
// applied) plus a pure pass over the tail slots, then k_gfix. Otherwise, two
// launches per pivot:
//   k_gselect<j>, k_gstage<j>   for j = 0 .. K-1
//   k_gupdate                   applies the kdone pivots the group decided.
// k_gselect<0> and k_gdecide also close the previous group: the columns that
// entered and stay basic give up their slots to the appended columns that
// stay nonbasic.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace lpgpu {

constexpr int kMaxFuse = 48;       // pivots per group with the one-launch decision kernel
constexpr int kMaxFuseSplit = 16;  // with the two launches per pivot (k_gselect, k_gstage)
// How a launch of the one-launch decision kernel gave up (GroupState::stalled):
// a grid-barrier wait after the check-in ran out of polls (the group's state
// may be half written: the solve ends with LP_STALLED), or the check-in gate
// closed before every workgroup was resident (the launch wrote nothing: the
// host goes on with the barrier-free kernels).
constexpr int32_t kStallBarrier = 1;
constexpr int32_t kStallGate = 2;

// 16-byte loads and stores with the non-temporal hint, for the passes that
// stream the tableau (and A) once: they leave the L2 to the group's F and R,
// which every tile reads again (without them the first pass fetched 1.6
// times its bytes).
typedef double v2nt __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 nt_load2(const void *p) {
    const v2nt v = __builtin_nontemporal_load(reinterpret_cast<const v2nt *>(p));
    return double2{v.x, v.y};
}
__device__ __forceinline__ void nt_store2(void *p, const double2 &x) {
    const v2nt v = {x.x, x.y};
    __builtin_nontemporal_store(v, reinterpret_cast<v2nt *>(p));
}

// Decisions of the current group, resident in device memory.
struct GroupState {
    int32_t kdone;  // pivots decided in this group
    int32_t napp;   // leaving columns appended to the list (slots n+1 ..)
    int32_t stalled;  // kStallBarrier or kStallGate: the decision kernel gave up on its
                      // launch; the update passes then apply nothing (the group's inputs are
                      // incomplete)
    int32_t pad_;
    int32_t r[kMaxFuse];
    int32_t q[kMaxFuse];
    int32_t l[kMaxFuse];  // leaving column of pivot k
    double p[kMaxFuse];
};

// State, slack basis, list and zeroed pivot-column buffers for a new solve.
static __global__ void k_ginit(DevState *st, DevState init, GroupState *gs, int32_t *__restrict__ basis, int32_t m,
                               int32_t n, int32_t K, int32_t KF, double *__restrict__ Fk, int64_t ld,
                               int32_t *__restrict__ cols, int32_t *__restrict__ pos,
                               unsigned long long *__restrict__ cols_done, double *__restrict__ T,
                               const double *__restrict__ b) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t Lg = (int64_t)n + 1 + K;
    if (idx == 0) {
        *st = init;
        gs->kdone = 0;
        gs->napp = 0;
        gs->stalled = 0;
        cols_done[0] = 0;
        cols_done[1] = 0;
        cols_done[2] = 0;
        cols_done[3] = 0;
    }
    // with a deferred build, the right-hand side column (b in rows 1..m) and
    // row 0 of the slack columns (0: they are basic)
    if (b && idx < ld) T[(int64_t)(n + m) * ld + idx] = (idx >= 1 && idx <= m) ? b[idx - 1] : 0.0;
    if (b && idx < m) T[(int64_t)(n + idx) * ld] = 0.0;
    if (idx < m) basis[idx] = n + (int32_t)idx;
    if (idx < (int64_t)KF * ld) Fk[idx] = 0.0;
    if (idx < Lg + kMaxFuse) cols[idx] = idx < n ? (int32_t)idx : (idx == n ? n + m : -1);  // list + padding
    if (idx < (int64_t)n + m) pos[idx] = idx < n ? (int32_t)idx : -1;
}

// Closes the finished group (one thread). Entered columns that are still
// basic give their slots below n to the appended columns that are nonbasic
// at the end; the two counts are equal, since the group started with n
// nonbasic columns in slots 0..n-1 and ends with n nonbasic columns, each of
// which is either one that stayed in its slot or an appended one. All reads
// (the group, its appended slots, the slots of its entered columns) are
// issued in one batch and the pairing is done in registers (fully unrolled
// loops, no local arrays indexed at run time), so the close costs about two
// memory round trips.
template <int N>
__device__ void close_group_n(GroupState *gs, int32_t *__restrict__ cols, int32_t *__restrict__ pos, int32_t n) {
    const int kd = gs->kdone;
    if (kd == 0) return;
    const int na = gs->napp;
    // loads without per-entry conditions (every index is in bounds: the
    // group record and the list's padding slots have at least N entries),
    // then the entries past the group masked out, so that no load waits for
    // another
    int32_t qk[N], lk[N], app[N], pq[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        qk[k] = gs->q[k];
        lk[k] = gs->l[k];
        app[k] = cols[n + 1 + k];
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const bool in = k < kd && qk[k] >= 0;
        pq[k] = pos[in ? qk[k] : 0];
        if (!in) {
            qk[k] = -1;
            lk[k] = -1;
            pq[k] = -1;
        }
        if (k >= na) app[k] = -1;
    }
    // the last event of the group decides: entered -> basic, left -> nonbasic
    bool qb[N], ab[N];  // entered column k / appended column s basic at the end
#pragma unroll
    for (int k = 0; k < N; ++k) {
        bool bq = false, ba = false;
#pragma unroll
        for (int e = 0; e < N; ++e) {
            if (qk[e] == qk[k]) bq = true;
            if (lk[e] == qk[k]) bq = false;
            if (qk[e] == app[k]) ba = true;
            if (lk[e] == app[k]) ba = false;
        }
        qb[k] = bq;
        ab[k] = ba;
    }
    bool free_k[N];  // entered column k still basic and holding a slot below n
#pragma unroll
    for (int k = 0; k < N; ++k) {
        bool first = true;  // a column entered twice holds its slot once
#pragma unroll
        for (int e = 0; e < k; ++e) first &= qk[e] != qk[k];
        free_k[k] = k < kd && first && pq[k] >= 0 && pq[k] < n && qb[k];
    }
#pragma unroll
    for (int k = 0; k < N; ++k)
        if (k < kd && qb[k] && pq[k] >= 0) pos[qk[k]] = -1;
#pragma unroll
    for (int s = 0; s < N; ++s) {
        if (s < na) {
            const int32_t c = app[s];
            if (ab[s]) {
                pos[c] = -1;  // left and entered again within the group
            } else {
                int32_t t = -1;
#pragma unroll
                for (int k = 0; k < N; ++k)
                    if (t < 0 && free_k[k]) {
                        t = pq[k];
                        free_k[k] = false;
                    }
                if (t >= 0) {
                    cols[t] = c;
                    pos[c] = t;
                }
            }
            cols[n + 1 + s] = -1;
        }
    }
    gs->kdone = 0;
    gs->napp = 0;
}
// groups of the two-launch path (at most kMaxFuseSplit pivots)
static __device__ __forceinline__ void close_group(GroupState *gs, int32_t *__restrict__ cols,
                                                   int32_t *__restrict__ pos, int32_t n) {
    close_group_n<kMaxFuseSplit>(gs, cols, pos, n);
}

// Step 1 partial of the staging kernel: the best (row-0 value, column) of a
// workgroup's slots, and the slot itself.
struct SPart {
    double v;
    int32_t i;
    int32_t t;
};

// Step 2 partial of one select workgroup: its best (ratio, row), a NaN flag,
// and, read by the thread that owns that row, the pivot value (the row's
// entry of column q after the earlier pivots), the column basic in that row
// and that column's slot (-1 when it has none).
struct GRatio {
    double v;
    int32_t r;
    int32_t bad;
    double p;
    int32_t leave;
    int32_t lpos;
    double rb;  // k_gdecide: the RHS entry of row r after the earlier pivots of the group
};

// Lexicographic argmin that carries an int payload along with the winner:
// the steps of wave_argmin (every lane active).
__device__ __forceinline__ void wave_argmin_t(double &v, int32_t &i, int32_t &t) {
    auto take = [&](double ov, int32_t oi, int32_t ot) {
        const bool tk = lex_less(ov, oi, v, i);
        v = tk ? ov : v;
        i = tk ? oi : i;
        t = tk ? ot : t;
    };
    take(dpp_f64<0xB1>(v), dpp_i32<0xB1>(i), dpp_i32<0xB1>(t));
    take(dpp_f64<0x4E>(v), dpp_i32<0x4E>(i), dpp_i32<0x4E>(t));
    take(dpp_f64<0x141>(v), dpp_i32<0x141>(i), dpp_i32<0x141>(t));
    take(dpp_f64<0x140>(v), dpp_i32<0x140>(i), dpp_i32<0x140>(t));
    take(swap_f64<16>(v), swap_i32<16>(i), swap_i32<16>(t));
    take(swap_f64<32>(v), swap_i32<32>(i), swap_i32<32>(t));
}

__device__ __forceinline__ void block_argmin_t(double &v, int32_t &i, int32_t &t, double *sv, int32_t *si,
                                               int32_t *sl) {
    wave_argmin_t(v, i, t);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0) {
        sv[wave] = v;
        si[wave] = i;
        sl[wave] = t;
    }
    __syncthreads();
    v = lane < nw ? sv[lane] : __builtin_inf();
    i = lane < nw ? si[lane] : kNoIndex;
    t = lane < nw ? sl[lane] : -1;
    wave_argmin_t(v, i, t);
}

// Step 1 partials reduced in batches of 8 loads, so that a thread's loads
// are in flight together; `slot` gives the winner's slot (-1 for partials
// that carry none).
template <typename P>
__device__ __forceinline__ void reduce_parts(const P *__restrict__ pp, int32_t np, int tid, int nt, double &v,
                                             int32_t &q, int32_t &slot) {
    for (int32_t k0 = tid; k0 < np; k0 += 8 * nt) {
        P a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int32_t k = k0 + u * nt;
            if (k < np) a[u] = pp[k];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int32_t k = k0 + u * nt;
            if (k < np && lex_less(a[u].v, a[u].i, v, q)) {
                v = a[u].v;
                q = a[u].i;
                if constexpr (std::is_same_v<P, SPart>) slot = a[u].t;
            }
        }
    }
}

// Row 0 of columns [0, ncols) reduced in batches of 8 strided loads (the
// first Step 1 of a solve, before any partials exist).
__device__ __forceinline__ void scan_row0(const double *__restrict__ T, int64_t ld, int32_t ncols, int tid, int nt,
                                          double &v, int32_t &q) {
    for (int32_t c0 = tid; c0 < ncols; c0 += 8 * nt) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int32_t c = c0 + u * nt;
            t[u] = c < ncols ? T[(int64_t)c * ld] : __builtin_inf();
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int32_t c = c0 + u * nt;
            if (c < ncols && lex_less(t[u], c, v, q)) {
                v = t[u];
                q = c;
            }
        }
    }
}

// Steps 1 and 2 of pivot J of the group (J is a template argument so that
// the chain's coefficients load without a wait per pivot):
//   Step 1  J = 0: final stage of the argmin over the update's partials (a
//           scan of row 0 before the first pivot); J > 0: over the staging
//           kernel's partials of row 0 after pivot J-1, which also name the
//           entering column's slot;
//   Step 2  column q and the RHS column after the J earlier pivots, rebuilt
//           from the tableau by the chain above; column q is kept as F_J.
// Then the decision (r, q, p, leaving column), the basis, the log and, if the
// leaving column is not in the list yet, its appended slot.
//
// G workgroups of 256 threads, each taking rows [w*span, (w+1)*span) of
// Step 2 (about one row per thread). A thread's first row is requested
// before Step 1 finishes (its RHS and pivot-column entries, the column basic
// in it and that column's slot), so that after Step 1 only column q remains
// to load. Every workgroup runs Step 1 itself (the same reduction in the
// same order, so all agree on q), writes one partial and takes a ticket; the
// last to arrive (device-scope fences around the ticket) reduces the
// partials and records the decision. Nothing waits for another workgroup, so
// the launch cannot deadlock. For J = 0 the previous group is closed by that
// last workgroup before it reads the list, or by workgroup 0 when no pivot
// follows; no other workgroup reads the list, the slot map or the group's
// count then (the slots read ahead by J = 0 are not used).
template <int J>
__global__ __launch_bounds__(256) void k_gselect(const double *__restrict__ T, int64_t ld, int32_t m, int32_t n,
                                                 int32_t K, const ArgMin *__restrict__ parts,
                                                 const SPart *__restrict__ sparts, int32_t nsparts,
                                                 DevState *__restrict__ st, GroupState *__restrict__ gs,
                                                 double *__restrict__ Fk, double *__restrict__ Rk,
                                                 double *__restrict__ D, int32_t *__restrict__ cols,
                                                 int32_t *__restrict__ pos, int32_t *__restrict__ basis,
                                                 int32_t *__restrict__ log_r, int32_t *__restrict__ log_q,
                                                 GRatio *__restrict__ rparts, uint32_t *__restrict__ ticket) {
    __shared__ double sv[4];
    __shared__ int32_t si[4], sl[4];
    __shared__ uint32_t s_last;
    __shared__ double s_p;
    __shared__ int32_t s_leave, s_lpos;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int G = gridDim.x, w = blockIdx.x;
    const int64_t Lg = (int64_t)n + 1 + K;
    const int64_t W = (int64_t)n + m + 1;
    const double *rhs = T + (W - 1) * ld;

    // read ahead: this thread's first row
    const int32_t span = (m + 1 + G - 1) / G;
    const int32_t i0 = w * span, i1 = min(m + 1, i0 + span);
    const int32_t ia = i0 + tid;
    const bool has_a = ia < i1;
    double bb_a = 0.0;
    double f_a[J > 0 ? J : 1];
    int32_t leave_a = -1, lpos_a = -1;
    if (has_a) {
        bb_a = rhs[ia];
#pragma unroll
        for (int k = 0; k < J; ++k) f_a[k] = Fk[(int64_t)k * ld + ia];
        if (ia >= 1) {
            leave_a = basis[ia - 1];
            lpos_a = pos[leave_a];
        }
    }
    int32_t rk[J > 0 ? J : 1];
    double Rb[J > 0 ? J : 1];
#pragma unroll
    for (int k = 0; k < J; ++k) {
        rk[k] = gs->r[k];
        Rb[k] = Rk[(int64_t)k * Lg + n];
    }

    const DevState s = *st;
    if (s.status != LP_RUNNING || s.pivots >= s.stop_at || (J > 0 && gs->kdone != J)) {
        if (J == 0 && w == 0 && tid == 0) close_group(gs, cols, pos, n);
        return;
    }

    // Step 1
    double v = __builtin_inf();
    int32_t q = kNoIndex, tq = -1;
    if (J == 0 && s.fresh)
        scan_row0(T, ld, n + m, tid, nt, v, q);
    else if (J == 0)
        reduce_parts(parts, s.nparts, tid, nt, v, q, tq);
    else
        reduce_parts(sparts, nsparts, tid, nt, v, q, tq);
    block_argmin_t(v, q, tq, sv, si, sl);
    if (step1_bad(v) || v >= -s.eps_d) {
        if (w == 0 && tid == 0) {
            st->status = step1_bad(v) ? LP_NUMERICAL : LP_OPTIMAL;
            if (J == 0) close_group(gs, cols, pos, n);
        }
        return;
    }
    // every nonbasic column has a slot; a missing one (a broken list) ends
    // the solve below instead of reading outside R
    const int32_t tq_safe = tq < 0 ? 0 : tq;
    double Rq[J > 0 ? J : 1];
#pragma unroll
    for (int k = 0; k < J; ++k) Rq[k] = Rk[(int64_t)k * Lg + tq_safe];

    // Step 2 on this workgroup's rows of column q and the RHS after the J
    // earlier pivots
    const double *colq = T + (int64_t)q * ld;
    double *Fj = Fk + (int64_t)J * ld;
    double rv = __builtin_inf();
    int32_t r = kNoIndex;
    int bad = 0;
    double p_best = 0.0;
    int32_t leave_best = -1, lpos_best = -1;
    for (int32_t i = ia; i < i1; i += nt) {
        double a = colq[i], bb;
        double f[J > 0 ? J : 1];
        int32_t leave_i = -1, lpos_i = -1;
        if (i == ia) {
            bb = bb_a;
#pragma unroll
            for (int k = 0; k < J; ++k) f[k] = f_a[k];
            leave_i = leave_a;
            lpos_i = lpos_a;
        } else {
            bb = rhs[i];
#pragma unroll
            for (int k = 0; k < J; ++k) f[k] = Fk[(int64_t)k * ld + i];
            leave_i = basis[i - 1];
            lpos_i = pos[leave_i];
        }
#pragma unroll
        for (int k = 0; k < J; ++k) {
            if (i == rk[k]) {
                a = Rq[k];
                bb = Rb[k];
            } else {
                a = fma(-f[k], Rq[k], a);
                bb = fma(-f[k], Rb[k], bb);
            }
        }
        Fj[i] = a;
        if (i == 0) continue;
        if (step2_bad(a, bb)) {
            bad = 1;
        } else if (a > s.eps_p) {
            const double ratio = bb / a;
            if (lex_less(ratio, i, rv, r)) {
                rv = ratio;
                r = i;
                p_best = a;
                leave_best = leave_i;
                lpos_best = lpos_i;
            }
        }
    }
    const int32_t r_mine = r;
    bad = __syncthreads_or(bad);
    block_argmin(rv, r, sv, si);
    if (r != kNoIndex && r_mine == r) {  // the one thread that owns row r
        s_p = p_best;
        s_leave = leave_best;
        s_lpos = lpos_best;
    }
    __syncthreads();
    if (tid == 0) {
        rparts[w] = r == kNoIndex ? GRatio{rv, r, bad, 0.0, -1, -1} : GRatio{rv, r, bad, s_p, s_leave, s_lpos};
        __threadfence();
        s_last = atomicAdd(ticket, 1u) == (uint32_t)(G - 1);
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();

    // last workgroup: the decision (G <= 256: one partial per thread)
    GRatio pr{__builtin_inf(), kNoIndex, 0, 0.0, -1, -1};
    if (tid < G) pr = rparts[tid];
    rv = pr.v;
    r = pr.r;
    int32_t wk = tid;
    bad = __syncthreads_or(pr.bad);
    block_argmin_t(rv, r, wk, sv, si, sl);
    if (r != kNoIndex && wk == tid) {
        s_p = pr.p;
        s_leave = pr.leave;
        s_lpos = pr.lpos;
    }
    if (J == 0) {
        if (tid == 0) close_group(gs, cols, pos, n);
        // appended slots start with R = 0 and a row-0 entry of 0: the exact
        // values for a column that is basic (a unit vector) before it leaves
        if (tid < K * K) Rk[(int64_t)(tid / K) * Lg + n + 1 + tid % K] = 0.0;
        if (tid < K) D[n + 1 + tid] = 0.0;
    }
    __syncthreads();
    if (tid != 0) return;
    *ticket = 0;  // ready for the next launch (ordered by the kernel boundary)
    if (J > 0 && tq < 0) {
        st->status = LP_NUMERICAL;
        return;
    }
    if (bad || r == kNoIndex || s.pivots >= s.max_pivots) {
        st->status = bad ? LP_NUMERICAL : (r == kNoIndex ? LP_UNBOUNDED : LP_ITER_LIMIT);
        return;
    }
    const int32_t leave = s_leave;
    const int32_t lpos = J == 0 ? pos[leave] : s_lpos;  // J = 0: the slot map after closing
    const int32_t na = gs->napp;
    gs->r[J] = r;
    gs->q[J] = q;
    gs->l[J] = leave;
    gs->p[J] = s_p;
    if (lpos < 0) {
        cols[n + 1 + na] = leave;
        pos[leave] = n + 1 + na;
        gs->napp = na + 1;
    }
    gs->kdone = J + 1;
    basis[r - 1] = q;
    if (s.pivots < s.log_cap) {
        log_r[s.pivots] = r;
        log_q[s.pivots] = q;
    }
    st->pivots = s.pivots + 1;
    st->fresh = 0;
}

// Step 3 inputs of pivot J, one list slot per thread: the pivot-row entry
// after the J earlier pivots (chain from the tableau), R_J[t] = that / p_J,
// and the slot's row-0 entry after pivot J, D[t] = fma(-F_J[0], R_J[t], D[t])
// (row 0 is never a pivot row). Each workgroup then reduces its slots'
// (D, column) pairs to one Step 1 partial for pivot J+1, with the slot.
template <int J>
__global__ __launch_bounds__(256) void k_gstage(const double *__restrict__ T, int64_t ld, int32_t m, int32_t n,
                                                int32_t K, const GroupState *__restrict__ gs,
                                                const double *__restrict__ Fk, double *__restrict__ Rk,
                                                double *__restrict__ D, const int32_t *__restrict__ cols,
                                                SPart *__restrict__ sparts) {
    __shared__ double sv[4];
    __shared__ int32_t si[4], sl[4];
    if (gs->kdone <= J) return;
    const int64_t Lg = (int64_t)n + 1 + K;
    const int32_t r = gs->r[J];
    const double p = gs->p[J];
    int32_t rk[J > 0 ? J : 1];
    double fr[J > 0 ? J : 1];
#pragma unroll
    for (int k = 0; k < J; ++k) {
        rk[k] = gs->r[k];
        fr[k] = Fk[(int64_t)k * ld + r];
    }
    const double f0 = Fk[(int64_t)J * ld];
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double v = __builtin_inf();
    int32_t idx = kNoIndex, slot = -1;
    if (t < Lg) {
        const int32_t c = cols[t];
        if (c >= 0) {
            const double *col = T + (int64_t)c * ld;
            double y = col[r];
            double d = J == 0 ? col[0] : D[t];
            double Rkt[J > 0 ? J : 1];
#pragma unroll
            for (int k = 0; k < J; ++k) Rkt[k] = Rk[(int64_t)k * Lg + t];
#pragma unroll
            for (int k = 0; k < J; ++k) y = (r == rk[k]) ? Rkt[k] : fma(-fr[k], Rkt[k], y);
            const double R = y / p;
            Rk[(int64_t)J * Lg + t] = R;
            d = fma(-f0, R, d);
            D[t] = d;
            if (c != n + m) {
                v = d;
                idx = c;
                slot = (int32_t)t;
            }
        }
    }
    block_argmin_t(v, idx, slot, sv, si, sl);
    if (threadIdx.x == 0) sparts[blockIdx.x] = SPart{v, idx, slot};
}

// ---------------------------------------------------------------------------
// All decisions of a group in one launch.
//
// Reductions of the decision kernel. Within a row of 16 lanes the wave
// argmin exchanges values by DPP (quad permutations, then the half-row and
// row mirrors: after these four steps every lane holds its row's winner);
// the last two steps cross rows with the lane swaps of gfx950
// (v_permlane16_swap, v_permlane32_swap: VALU exchanges, no LDS round trip).
// Every step is compares and selects, without branches. The argmin is unique
// under the (value, index) order of lex_less, so the result does not depend
// on the order of the reduction: every wave that reduces the same candidates
// gets the same winner.
__device__ __forceinline__ double readlane_f64(double x, int32_t lane) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), lane),
                            __builtin_amdgcn_readlane(__double2loint(x), lane));
}

// Keeps the smaller of (v, i, t) and (ov, oi, ot) under lex_less.
__device__ __forceinline__ void argmin_take(double &v, int32_t &i, int32_t &t, double ov, int32_t oi, int32_t ot) {
    const bool take = lex_less(ov, oi, v, i);
    v = take ? ov : v;
    i = take ? oi : i;
    t = take ? ot : t;
}

template <int CTRL>
__device__ __forceinline__ void dpp_step(double &v, int32_t &i, int32_t &t) {
    argmin_take(v, i, t, dpp_f64<CTRL>(v), dpp_i32<CTRL>(i), dpp_i32<CTRL>(t));
}

template <int W>
__device__ __forceinline__ void swap_step(double &v, int32_t &i, int32_t &t) {
    argmin_take(v, i, t, swap_f64<W>(v), swap_i32<W>(i), swap_i32<W>(t));
}

// wave argmin of (v, i) carrying t; every lane gets the winner
__device__ __forceinline__ void wave_argmin_dpp(double &v, int32_t &i, int32_t &t) {
    dpp_step<0xB1>(v, i, t);   // quad_perm [1,0,3,2]
    dpp_step<0x4E>(v, i, t);   // quad_perm [2,3,0,1]
    dpp_step<0x141>(v, i, t);  // row_half_mirror
    dpp_step<0x140>(v, i, t);  // row_mirror
    swap_step<16>(v, i, t);    // rows 0 <-> 1, 2 <-> 3
    swap_step<32>(v, i, t);    // lanes 0-31 <-> 32-63
}

// Block argmin with one barrier: `sv`, `si`, `sl` (one entry per wave) must
// belong to this call site alone, and a block-wide barrier must separate two
// of its calls (the next call's writes then cannot meet this call's reads).
template <int BD>
__device__ __forceinline__ void block_argmin_dpp(double &v, int32_t &i, int32_t &t, double *sv, int32_t *si,
                                                 int32_t *sl) {
    wave_argmin_dpp(v, i, t);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        sv[wave] = v;
        si[wave] = i;
        sl[wave] = t;
    }
    __syncthreads();
    // the wave winners, read by every lane (one LDS address per read) and
    // reduced in registers
    v = sv[0];
    i = si[0];
    t = sl[0];
#pragma unroll
    for (int u = 1; u < BD / 64; ++u) argmin_take(v, i, t, sv[u], si[u], sl[u]);
}

// k_gdecide runs the group's Steps 1-2 and the Step 3 inputs (what k_gselect
// and k_gstage compute, with the same arithmetic in the same order) for up
// to K pivots in one launch of G workgroups of BD threads (256 or 512),
// G*BD covering both the rows 0..m and the list slots. It starts by closing the previous
// group and by reducing the slots' row-0 entries (the update pass leaves row
// 0 in the tableau) to the first pivot's Step 1 partials, and ends by storing
// identities for the pivots the group did not reach and counting the changed
// columns, which is all the pure update pass needs. Thread (w, x) owns row
// w*BD+x and slot w*BD+x for the whole group, and keeps their chain state in
// registers across pivots: the row's entries of the group's pivot columns
// (F_k[i]), the slot's normalised pivot-row entries (R_k[t]), its row-0
// entry, its column, and the row's basic column. Per pivot, two grid
// barriers separate the phases:
//   pricing (every workgroup, over all staging partials) and the ratio test
//     of its rows -> one Step 2 partial per workgroup;   barrier
//   the decision (every workgroup reduces all Step 2 partials, so all agree;
//     workgroup 0 records it) and the Step 3 inputs of its slots -> one
//     Step 1 partial per workgroup;                       barrier.
// A barrier carries the partials it waits for: each workgroup publishes its
// partial as a record of 64-bit words in a line of its own, each word 32 bits
// of the partial with the launch's flag in the upper half (an aligned 64-bit
// store is single-copy atomic, so a word with the current flag holds current
// data), and waits by reading every workgroup's record until all words carry
// the flag: the partials arrive with the wait, with no counter and no second
// read. Every barrier of a launch has records of its own and every launch a
// flag of its own (epoch + 1, the epoch advanced by the last workgroup to
// leave), so no record is reused within a launch and an old record never
// passes for a new one. The wait is bounded (spin_limit polls): if some
// workgroup never arrives (the G workgroups were not all resident), the
// waiting ones set LP_STALLED and leave, so every wave exits.
constexpr int kXchWords = 16;  // words per record: one 128-byte line
constexpr int kMaxDecideBarriers = 2 * kMaxFuse + 2;
constexpr int kMaxDecideWgsXch = 128;  // records per barrier (the decision kernel's workgroup limit)
struct GridSync {
    uint32_t count;  // check-in gate: workgroups arrived, kGateClosed once closed
    uint32_t exits;  // workgroups that have left this launch
    uint32_t epoch;  // launches completed
    uint32_t pad_[29];
    uint64_t xch[kMaxDecideBarriers][kMaxDecideWgsXch][kXchWords];
};

// The check-in gate at the start of a launch: the barriers below wait for
// all G workgroups, so they must all be resident at once, which nothing
// guarantees when other work shares the device. Each workgroup adds one to
// the gate and waits until it reads G. One that has polled spin_limit times
// closes the gate with a compare-and-swap of the count it last read, which
// fails if another workgroup arrived meanwhile (it then reads again): the
// count reaches G or the gate closes, never both, so either every workgroup
// passes or none does. Workgroups that find the gate closed leave at once;
// nothing before the gate writes to memory, so a closed gate leaves the
// solve as it was (the group is marked kStallGate and the status LP_STALLED,
// from which the host resumes on the barrier-free kernels). The last
// workgroup to leave the launch reopens the gate.
constexpr uint32_t kGateClosed = 0x80000000u;

__device__ __forceinline__ bool gate_pass(GridSync *gsync, int G, uint32_t spin_limit, DevState *st, GroupState *gs,
                                          int32_t *s_ok) {
    if (threadIdx.x == 0) {
        uint32_t v = atomicAdd(&gsync->count, 1u) + 1u;
        uint32_t it = 0;
        bool ok = false;
        for (;;) {
            if (v & kGateClosed) break;
            if (v == (uint32_t)G) {
                ok = true;
                break;
            }
            if (++it > spin_limit) {
                const uint32_t old = atomicCAS(&gsync->count, v, v | kGateClosed);
                if (old == v) break;  // closed
                v = old;
                continue;
            }
            __builtin_amdgcn_s_sleep(1);
            v = __hip_atomic_load(&gsync->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (ok) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        } else {  // (every workgroup that finds the gate closed: the same marks)
            atomicExch(&gs->stalled, kStallGate);
            atomicCAS(&st->status, (int32_t)LP_RUNNING, (int32_t)LP_STALLED);
        }
        *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

// Publishes this workgroup's record for a barrier: one thread, after a
// workgroup barrier that follows the workgroup's writes, so that the release
// fence makes them visible with the record (fence synchronisation with the
// waiters' acquire fence).
template <int N>
__device__ __forceinline__ void xch_publish(uint64_t *rec, const uint32_t (&d)[N], uint32_t flag) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
#pragma unroll
    for (int k = 0; k < N; ++k)
        __hip_atomic_store(rec + k, ((uint64_t)flag << 32) | d[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits for the records of all G workgroups (N words each) at `recs`: wave 0
// polls (lane l reads record l and record l + 64) and copies the data words
// to LDS (xs[w][k]), then the workgroup passes its barrier. A wait that gives
// up marks the solve LP_STALLED and the group as stalled. A workgroup that
// arrives late can still find every record of a barrier that others abandoned
// (those who gave up had published theirs), so the poll also reads the status
// and a stalled solve fails the wait: the final status is written only over
// LP_RUNNING (finish_status), so LP_STALLED is never overwritten.
template <int N>
__device__ __forceinline__ bool xch_wait(const uint64_t (*recs)[kXchWords], int G, uint32_t flag, uint32_t spin_limit,
                                         DevState *st, GroupState *gs, uint32_t (*xs)[N], int32_t *s_ok) {
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        uint64_t a[N], b[N];
        uint32_t it = 0;
        bool ok = false;
        for (;;) {
            // the status first, by every lane (one request): issued with the
            // record loads, not after them
            const int32_t stv = __hip_atomic_load(&st->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            bool mine = true;
            if (lane < G) {
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    a[k] = __hip_atomic_load(&recs[lane][k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    mine &= (uint32_t)(a[k] >> 32) == flag;
                }
            }
            if (lane + 64 < G) {
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    b[k] = __hip_atomic_load(&recs[lane + 64][k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    mine &= (uint32_t)(b[k] >> 32) == flag;
                }
            }
            const bool stalled = __builtin_amdgcn_readfirstlane(stv) == LP_STALLED;
            const bool all = __ballot(!mine) == 0;
            if (stalled) break;
            if (all) {
                ok = true;
                break;
            }
            if (++it > spin_limit) {
                if (lane == 0) {
                    atomicExch(&st->status, (int32_t)LP_STALLED);
                    atomicExch(&gs->stalled, kStallBarrier);
                }
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (ok) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if (lane < G) {
#pragma unroll
                for (int k = 0; k < N; ++k) xs[lane][k] = (uint32_t)a[k];
            }
            if (lane + 64 < G) {
#pragma unroll
                for (int k = 0; k < N; ++k) xs[lane + 64][k] = (uint32_t)b[k];
            }
        }
        if (lane == 0) *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

__device__ __forceinline__ uint32_t lo32(double v) { return (uint32_t)__double_as_longlong(v); }
__device__ __forceinline__ uint32_t hi32(double v) { return (uint32_t)((uint64_t)__double_as_longlong(v) >> 32); }
__device__ __forceinline__ double as_f64(uint32_t lo, uint32_t hi) {
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// The status that ends the solve, written only while it is LP_RUNNING.
__device__ __forceinline__ void finish_status(DevState *st, int32_t status) {
    atomicCAS(&st->status, (int32_t)LP_RUNNING, status);
}

// Steps k < j of a chain (rows: x <- R_k if the row is r_k, else
// fma(-F_k, R_k, x)), unrolled over the first N of the KM entries (N >= j;
// the steps k >= j are masked out). Tiers of N keep the work near j.
// The chain of the group's pivots 0 .. j-1 on one entry (row `row`): at each
// pivot k, the entry becomes R_k if `row` is the pivot row r_k, else
// fma(-F_k, R_k, entry). One factor is the entry's own (per thread, in
// registers: OWN_F selects which), the other and the pivot rows are the same
// for every thread and live one per lane of the wave (lane k holds pivot k's,
// read with readlane), so that no register array grows with the group size
// beyond the thread's own history.
template <int N, int KM, bool OWN_F>
__device__ __forceinline__ double chain_steps(double x, int j, int32_t row, int32_t rk_l, const double (&own)[KM],
                                              double sh_l) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const int32_t rk = __builtin_amdgcn_readlane(rk_l, k);
        const double sh = readlane_f64(sh_l, k);
        const double F = OWN_F ? own[k] : sh, R = OWN_F ? sh : own[k];
        const double nx = (row == rk) ? R : fma(-F, R, x);
        x = k < j ? nx : x;
    }
    return x;
}

template <int KM, bool OWN_F>
__device__ __forceinline__ double chain_tiered(double x, int j, int32_t row, int32_t rk_l, const double (&own)[KM],
                                               double sh_l) {
    constexpr int N1 = KM < 8 ? KM : 8, N2 = KM < 16 ? KM : 16, N3 = KM < 32 ? KM : 32;
    if (j <= N1) return chain_steps<N1, KM, OWN_F>(x, j, row, rk_l, own, sh_l);
    if (j <= N2) return chain_steps<N2, KM, OWN_F>(x, j, row, rk_l, own, sh_l);
    if (j <= N3) return chain_steps<N3, KM, OWN_F>(x, j, row, rk_l, own, sh_l);
    return chain_steps<KM, KM, OWN_F>(x, j, row, rk_l, own, sh_l);
}

// Entry (row, col) of the tableau at the start of the group. The first group
// after a deferred build reads the structural columns from A and c (the
// tableau holds them only after that group's update pass); everything else
// is read from the tableau.
template <bool First>
__device__ __forceinline__ double start_entry(const double *__restrict__ T, int64_t ld, int32_t n,
                                              const double *__restrict__ A, const double *__restrict__ cv,
                                              int32_t col, int32_t row) {
    if (First && col < n) return row == 0 ? -cv[col] : A[(int64_t)(row - 1) * n + col];
    return T[(int64_t)col * ld + row];
}

template <int BD, bool First, int KM>
__device__ __forceinline__ void decide_body(double *__restrict__ T, int64_t ld, int32_t m, int32_t n,
                                            const double *__restrict__ A, const double *__restrict__ cv,
                                            int32_t K, int32_t KF, SPart *__restrict__ sparts,
                                            unsigned long long *__restrict__ cols_done,
                                            DevState *__restrict__ st, GroupState *__restrict__ gs,
                                            double *__restrict__ Fk, double *__restrict__ Rk,
                                            int32_t *__restrict__ cols, int32_t *__restrict__ pos,
                                            int32_t *__restrict__ basis, int32_t *__restrict__ log_r,
                                            int32_t *__restrict__ log_q, GRatio *__restrict__ rparts,
                                            GridSync *__restrict__ gsync, uint32_t spin_limit,
                                            uint32_t gate_spin, double *__restrict__ PV) {
    // one set of reduction slots per call site (ratio test, staging, start)
    __shared__ double sv_r[BD / 64], sv_s[BD / 64], sv_0[BD / 64];
    __shared__ int32_t si_r[BD / 64], si_s[BD / 64], si_0[BD / 64];
    __shared__ int32_t sl_r[BD / 64], sl_s[BD / 64], sl_0[BD / 64];
    (void)rparts;  // (the Step 2 partials travel with the barrier here)
    __shared__ int32_t s_ok;
    // the partials the barriers carry: Step 1 (value, column, slot) and Step 2
    // (row, leaving column with the in-list flag, pivot value, RHS entry)
    __shared__ uint32_t xs_s[kMaxDecideWgsXch][4];
    __shared__ uint32_t xs_r[kMaxDecideWgsXch][6];
    // each row's Step 2 candidate (pivot entry, RHS entry, leaving column and
    // whether it has a slot), read by thread 0 for the workgroup's winner
    __shared__ double sc_a[BD], sc_b[BD];
    __shared__ uint32_t sc_l[BD];
    const int tid = threadIdx.x;
    const int G = gridDim.x, w = blockIdx.x;
    const int64_t Lg = (int64_t)n + 1 + K;
    const int64_t W = (int64_t)n + m + 1;
    uint32_t nbar = 0;                             // barriers passed in this launch
    const uint32_t flag = gsync->epoch + 1u;       // this launch's record flag
    if (!gate_pass(gsync, G, gate_spin, st, gs, &s_ok)) return;

    const DevState s0 = *st;
    const int32_t t = w * BD + tid;
    const bool has_slot = t < Lg;
    int32_t c_t = has_slot ? cols[t] : -1;

    // The close of the previous group (see close_group), computed by every
    // wave from the group record: lane k holds pivot k's entering column, its
    // slot, its leaving column and the column appended in slot n+1+k. Every
    // thread applies the result to its own slot; workgroup 0 stores it once
    // every workgroup has read the list (after the first barrier, or on the
    // way out).
    const int lane = tid & 63;
    const int32_t kd0 = gs->kdone, na0 = gs->napp;
    int32_t cq = -1, cl = -1, ca = -1, cp = -1;
    if (lane < KM) {
        cq = gs->q[lane];
        cl = gs->l[lane];
        ca = cols[n + 1 + lane];
    }
    if (lane >= kd0) {
        cq = -1;
        cl = -1;
    }
    if (lane >= na0) ca = -1;
    if (cq >= 0) cp = pos[cq];
    bool qb = false, ab = false, first = true;  // basic at the end (the last event decides)
#pragma unroll
    for (int e = 0; e < KM; ++e) {
        const int32_t qe = __builtin_amdgcn_readlane(cq, e), le = __builtin_amdgcn_readlane(cl, e);
        if (qe >= 0 && qe == cq) qb = true;
        if (le >= 0 && le == cq) qb = false;
        if (qe >= 0 && qe == ca) ab = true;
        if (le >= 0 && le == ca) ab = false;
        if (e < lane && qe >= 0 && qe == cq) first = false;  // a column entered twice holds one slot
    }
    // slots freed (entered, still basic, slot below n) and appended columns
    // that stay nonbasic, paired in order
    const uint64_t free_mask = __ballot(cq >= 0 && first && cp >= 0 && cp < n && qb);
    const uint64_t move_mask = __ballot(ca >= 0 && !ab);
    // what workgroup 0 stores: bit 0 pos[cq] = -1, bit 1 pos[ca] = -1, bit 2
    // slot n+1+lane cleared
    const int32_t cflags = (cq >= 0 && qb && cp >= 0 ? 1 : 0) | (ca >= 0 && ab ? 2 : 0) | (ca >= 0 ? 4 : 0);
    {
        uint64_t fm = free_mask, mm = move_mask;
#pragma unroll
        for (int u = 0; u < KM; ++u) {
            if (fm == 0 || mm == 0) break;
            const int32_t k = __builtin_ctzll(fm), a = __builtin_ctzll(mm);
            fm &= fm - 1;
            mm &= mm - 1;
            if (t == __builtin_amdgcn_readlane(cp, k)) c_t = __builtin_amdgcn_readlane(ca, a);
        }
        if (t > n) c_t = -1;  // appended slots are empty after the close
    }
    // Stores the close: wave 0 of workgroup 0, every lane active (no lane
    // reads another's registers inside divergent code). Lane k stores its own
    // entries; the a-th column to move takes the a-th freed slot.
    auto store_close = [&]() {
        if (cflags & 1) pos[cq] = -1;
        if (cflags & 2) pos[ca] = -1;
        if (cflags & 4) cols[n + 1 + lane] = -1;
        const int32_t rank = __popcll(move_mask & ((1ull << lane) - 1));
        uint64_t fm = free_mask;
        for (int32_t u = 0; u < rank; ++u) fm &= fm - 1;
        const int32_t ts = __shfl(cp, fm ? __builtin_ctzll(fm) : 0, 64);
        if (((move_mask >> lane) & 1) && fm) {
            cols[ts] = ca;
            pos[ca] = ts;
        }
        if (lane == 0) {
            gs->kdone = 0;
            gs->napp = 0;
        }
    };
    if (s0.status != LP_RUNNING) {
        if (w == 0 && tid < 64) store_close();
        return;
    }

    // this thread's row and slot, and their state at the start of the group;
    // after the close no basic column is in the list
    const int32_t i = w * BD + tid;
    const bool has_row = i <= m;
    const int32_t is = has_row ? i : 0;
    const double rhs0 = T[(W - 1) * ld + is];
    int32_t basis_i = (has_row && i >= 1) ? basis[i - 1] : -1;
    bool inlist_i = false;
    double bcur = rhs0;  // this row's RHS entry after the pivots decided so far
    double D_t = c_t >= 0 ? start_entry<First>(T, ld, n, A, cv, c_t, 0) : 0.0;
    if (s0.fresh) {
        // Step 1 partials of the first pivot after the build (later groups
        // find them where the previous group's last staging left them: its
        // row-0 entries after its last pivot, the values the update wrote)
        double dv = __builtin_inf();
        int32_t di = kNoIndex, ds = -1;
        if (c_t >= 0 && c_t != n + m) {
            dv = D_t;
            di = c_t;
            ds = t;
        }
        block_argmin_dpp<BD>(dv, di, ds, sv_0, si_0, sl_0);
        if (tid == 0) {
            const uint32_t d[4] = {lo32(dv), hi32(dv), (uint32_t)di, (uint32_t)ds};
            xch_publish<4>(gsync->xch[nbar][w], d, flag);
        }
        if (!xch_wait<4>(gsync->xch[nbar], G, flag, spin_limit, st, gs, xs_s, &s_ok)) return;
        ++nbar;
    }
    double frow[KM], rslot[KM];
    int32_t rk_l = -1;  // lane k: the pivot row of pivot k
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        frow[k] = 0.0;
        rslot[k] = 0.0;
    }
    int32_t napp = 0;
    int kd = 0;  // pivots decided in this group

    for (int j = 0; j < K; ++j) {
        const bool budget = s0.pivots + j >= s0.stop_at;

        // Step 1
        // (every wave reduces all G partials itself: no LDS, no barrier)
        double v = __builtin_inf();
        int32_t q = kNoIndex, tq = -1;
        if (!budget) {
            // the partials of the last barrier, or at a group's first pivot
            // those the previous group's last staging left
            const SPart none{__builtin_inf(), kNoIndex, -1};
            SPart a = none, b = none;
            if (j == 0 && !s0.fresh) {
                if (lane < G) a = sparts[lane];
                if (lane + 64 < G) b = sparts[lane + 64];
            } else {
                if (lane < G) a = SPart{as_f64(xs_s[lane][0], xs_s[lane][1]), (int32_t)xs_s[lane][2],
                                        (int32_t)xs_s[lane][3]};
                if (lane + 64 < G)
                    b = SPart{as_f64(xs_s[lane + 64][0], xs_s[lane + 64][1]), (int32_t)xs_s[lane + 64][2],
                              (int32_t)xs_s[lane + 64][3]};
            }
            if (lex_less(b.v, b.i, a.v, a.i)) a = b;
            v = a.v;
            q = a.i;
            tq = a.t;
            wave_argmin_dpp(v, q, tq);
        }
        // (the same decisions in every workgroup: the same partials)
        bool stop = budget;
        if (!stop && (step1_bad(v) || v >= -s0.eps_d)) {
            if (w == 0 && tid == 0) finish_status(st, step1_bad(v) ? LP_NUMERICAL : LP_OPTIMAL);
            stop = true;
        }
        if (!stop && tq < 0) {  // a broken list ends the solve instead of reading outside R
            if (w == 0 && tid == 0) finish_status(st, LP_NUMERICAL);
            stop = true;
        }
        if (stop) {
            if (j == 0) {  // the close is stored once every workgroup has read the list
                __syncthreads();  // every wave has read the Step 1 partials (wave 0 rewrites them)
                if (tid == 0) {
                    const uint32_t d[4] = {0u, 0u, 0u, 0u};
                    xch_publish<4>(gsync->xch[nbar][w], d, flag);
                }
                if (!xch_wait<4>(gsync->xch[nbar], G, flag, spin_limit, st, gs, xs_s, &s_ok)) return;
                ++nbar;
                if (w == 0 && tid < 64) store_close();
            }
            break;
        }

        // Step 2 on this thread's row of column q and the RHS after the j
        // earlier pivots; the row's entry of column q is kept as F_j[i]. The
        // R entries of slot tq are loaded one per lane (lane k: R_k, index
        // clamped into the buffer), in the same batch as the entry, and the
        // steps k >= j are masked out by selects. The RHS entry is carried
        // from pivot to pivot (bcur) with the same operations.
        const int32_t tqs = tq < 0 ? 0 : tq;
        const double rq_l = Rk[(int64_t)(lane < K ? lane : K - 1) * Lg + tqs];
        const double a =
            chain_tiered<KM, true>(start_entry<First>(T, ld, n, A, cv, q, is), j, i, rk_l, frow, rq_l);
        const double bb = bcur;
#pragma unroll
        for (int k = 0; k < KM; ++k)
            if (k == j) frow[k] = a;
        if (has_row) Fk[(int64_t)j * ld + i] = a;
        // a non-finite column entry or a NaN RHS entry (step2_bad) becomes
        // a NaN candidate, which wins the argmin and so reaches the decision
        // as "bad"
        double rv = __builtin_inf();
        int32_t r = kNoIndex;
        if (has_row && i >= 1) {
            if (step2_bad(a, bb)) {
                rv = __builtin_nan("");
                r = i;
            } else if (a > s0.eps_p) {
                rv = bb / a;
                r = i;
            }
        }
        if (r != kNoIndex) {
            sc_a[tid] = a;
            sc_b[tid] = bb;
            sc_l[tid] = (uint32_t)basis_i | (inlist_i ? 0x80000000u : 0u);
        }
        {
            int32_t unused = 0;
            block_argmin_dpp<BD>(rv, r, unused, sv_r, si_r, sl_r);
        }
        // the workgroup's Step 2 partial, published by thread 0 (the
        // argmin's barrier ordered the winner's candidate before the reads):
        // the row, its leaving column with "has a slot" in bit 31, its pivot
        // and RHS entries. The ratio itself is not sent: the readers compute
        // it from the two entries as the rows did (the same division, so the
        // same bits; a NaN candidate is recognised by step2_bad again).
        if (tid == 0) {
            uint32_t d[6] = {(uint32_t)kNoIndex, 0xffffffffu, 0u, 0u, 0u, 0u};
            if (r != kNoIndex) {
                const int32_t o = r - w * BD;
                const double ca = sc_a[o], cb = sc_b[o];
                d[0] = (uint32_t)r;
                d[1] = sc_l[o];
                d[2] = lo32(ca);
                d[3] = hi32(ca);
                d[4] = lo32(cb);
                d[5] = hi32(cb);
            }
            xch_publish<6>(gsync->xch[nbar][w], d, flag);
        }
        if (!xch_wait<6>(gsync->xch[nbar], G, flag, spin_limit, st, gs, xs_r, &s_ok)) return;
        ++nbar;
        if (j == 0 && w == 0) {  // every workgroup has read the list
            if (tid < 64) store_close();
            __syncthreads();  // before the decision record below
        }

        // the decision, reduced by every workgroup from all Step 2 partials
        // (every wave reduces all G partials itself; the winner's payload
        // is read from the lane that holds it)
        double p, rb;
        int32_t leave, inl;
        {
            const GRatio none{__builtin_inf(), kNoIndex, 0, 0.0, -1, 0, 0.0};
            auto rec = [&](int u) {
                const int32_t rr = (int32_t)xs_r[u][0];
                const uint32_t lw = xs_r[u][1];
                const double ca = as_f64(xs_r[u][2], xs_r[u][3]), cb = as_f64(xs_r[u][4], xs_r[u][5]);
                const double cv = rr == kNoIndex ? __builtin_inf() : (step2_bad(ca, cb) ? __builtin_nan("") : cb / ca);
                return GRatio{cv, rr, 0, ca, (int32_t)(lw & 0x7fffffffu), (int32_t)(lw >> 31), cb};
            };
            GRatio pa = lane < G ? rec(lane) : none;
            const GRatio pb = lane + 64 < G ? rec(lane + 64) : none;
            if (lex_less(pb.v, pb.r, pa.v, pa.r)) pa = pb;
            rv = pa.v;
            r = pa.r;
            int32_t wl = lane;
            wave_argmin_dpp(rv, r, wl);
            p = readlane_f64(pa.p, wl);
            rb = readlane_f64(pa.rb, wl);
            leave = __builtin_amdgcn_readlane(pa.leave, wl);
            inl = __builtin_amdgcn_readlane(pa.lpos, wl);
        }
        const int bad_all = rv != rv;
        if (bad_all || r == kNoIndex || s0.pivots + j >= s0.max_pivots) {
            if (w == 0 && tid == 0)
                finish_status(st, bad_all ? LP_NUMERICAL : (r == kNoIndex ? LP_UNBOUNDED : LP_ITER_LIMIT));
            break;
        }
        const int32_t aslot = inl ? -1 : n + 1 + napp;  // appended slot of the leaving column
        if (aslot >= 0) ++napp;
        // The loads of the Step 3 inputs first, so that their latency covers
        // the bookkeeping below: F_k at the pivot row (lane k), F_j[0], and
        // this slot's pivot-row entry at the group's start (R = 0 for a slot
        // not filled yet: its column is a unit vector that no pivot of the
        // group has changed; the slot just appended holds e_r, whose entry in
        // row r is 1, taken as is since its store below may not be visible
        // yet)
        const int32_t c_new = t == aslot ? leave : c_t;
        const double fr_l = Fk[(int64_t)(lane < K ? lane : K - 1) * ld + r];  // lane k: F_k[r]
        const double F0 = Fk[(int64_t)j * ld];
        const double y0 = c_new < 0 ? 0.0 : (t == aslot ? 1.0 : start_entry<First>(T, ld, n, A, cv, c_new, r));
        if (w == 0 && tid == 0) {
            gs->r[j] = r;
            gs->q[j] = q;
            gs->l[j] = leave;
            gs->p[j] = p;
            gs->napp = napp;
            gs->kdone = j + 1;
            if (aslot >= 0) {
                cols[aslot] = leave;
                pos[leave] = aslot;
            }
            basis[r - 1] = q;
            const int64_t pv = s0.pivots + j;
            if (pv < s0.log_cap) {
                log_r[pv] = r;
                log_q[pv] = q;
            }
            st->pivots = pv + 1;
            st->fresh = 0;
        }
        kd = j + 1;
        {
            // the RHS after pivot j: R_j of the RHS slot is its row-r entry
            // over p, the value the slot's own staging computes
            const double Rn = rb / p;
            bcur = (i == r) ? Rn : fma(-a, Rn, bcur);
        }
        if (lane == j) rk_l = r;
        if (i == r) {
            basis_i = q;
            inlist_i = true;
        }
        c_t = c_new;
        // a column that leaves the basis for the first time in this group is
        // stored now as the unit vector it is (e_r: its basic row is the
        // pivot row), which makes it readable by the later pivots of the
        // group (after the barrier) and by the update pass; a column stored
        // before is that unit vector already. After a deferred build the
        // slack columns are not stored until they leave.
        if (aslot >= 0 && i < ld) T[(int64_t)leave * ld + i] = (i == r) ? 1.0 : 0.0;

        // Step 3 inputs of this thread's slot: the pivot-row entry after the
        // j earlier pivots, R_j[t] = that / p, and the row-0 entry after
        // pivot j
        double R = 0.0;
        {
            // The chain runs with every lane active: it reads the shared
            // factors from lanes 0 .. j-1, which must hold them
            const double y = chain_tiered<KM, false>(y0, j, r, rk_l, rslot, fr_l);
            if (c_t >= 0) {
                R = y / p;
                D_t = fma(-F0, R, D_t);
            }
        }
#pragma unroll
        for (int k = 0; k < KM; ++k)
            if (k == j) rslot[k] = R;
        if (has_slot) Rk[(int64_t)j * Lg + t] = R;
        double dv = __builtin_inf();
        int32_t di = kNoIndex, ds = -1;
        if (c_t >= 0 && c_t != n + m) {
            dv = D_t;
            di = c_t;
            ds = t;
        }
        block_argmin_dpp<BD>(dv, di, ds, sv_s, si_s, sl_s);
        // (also stored plainly: the next group's first pricing reads them,
        // whichever pivot of this group is the last)
        if (tid == 0) sparts[w] = SPart{dv, di, ds};
        if (j + 1 < K) {
            if (tid == 0) {
                const uint32_t d[4] = {lo32(dv), hi32(dv), (uint32_t)di, (uint32_t)ds};
                xch_publish<4>(gsync->xch[nbar][w], d, flag);
            }
            if (!xch_wait<4>(gsync->xch[nbar], G, flag, spin_limit, st, gs, xs_s, &s_ok)) return;
            ++nbar;
        }
    }

    // The pivot rows after the group, for every slot: the row of pivot a
    // takes R_a[t] at pivot a (the select of the chain), then the later
    // pivots' fma (or their R if the row pivots again): the operations of the
    // chain in its order. k_gfix stores them after the update pass, which
    // runs the chain without the select.
    if (kd > 0) {
        __shared__ double sM[KM][KM];  // sM[b][a] = F_b[r_a] for a < b < kd
        // thread b < kd loads F_b at the earlier pivot rows (one batch)
#pragma unroll
        for (int a = 0; a < KM; ++a)
            if (tid > a && tid < kd) sM[tid][a] = Fk[(int64_t)tid * ld + __builtin_amdgcn_readlane(rk_l, a)];
        __syncthreads();
        if (has_slot) {
            // every earlier pivot row updated by pivot b, b in order: for each
            // row the operations of its chain in its order, and b independent
            // updates per step
            double pv[KM];
#pragma unroll
            for (int a = 0; a < KM; ++a) pv[a] = rslot[a];
#pragma unroll
            for (int b = 1; b < KM; ++b) {
                if (b < kd) {
#pragma unroll
                    for (int a = 0; a < b; ++a)
                        pv[a] = (__builtin_amdgcn_readlane(rk_l, a) == __builtin_amdgcn_readlane(rk_l, b))
                                    ? rslot[b]
                                    : fma(-sM[b][a], rslot[b], pv[a]);
                }
            }
#pragma unroll
            for (int a = 0; a < KM; ++a)
                if (a < kd) PV[(int64_t)a * Lg + t] = pv[a];
        }
    }

    // The update pass applies KF pivots: the ones the group did not reach
    // become exact identities (F = 0, R = 0, no pivot row).
    for (int k = kd; k < KF; ++k) {
        if (has_row) Fk[(int64_t)k * ld + i] = 0.0;
        if (has_slot) Rk[(int64_t)k * Lg + t] = 0.0;
        if (w == 0 && tid == 0) gs->r[k] = -1;
    }
    // columns the group changes: some R entry of the slot nonzero
    bool nz = false;
#pragma unroll
    for (int k = 0; k < KM; ++k) nz |= k < kd && rslot[k] != 0.0;
    const unsigned long long cnt = __popcll(__ballot(nz));
    if ((tid & 63) == 0 && cnt) {
        atomicAdd(cols_done, cnt);
        if (First) atomicAdd(cols_done + 1, cnt);
    }
    if (First && w == 0 && tid == 0) {
        cols_done[2] = (unsigned long long)kd;
        cols_done[3] = (unsigned long long)napp;
    }
}

template <int BD, bool First, int KM>
__global__ __launch_bounds__(BD) void k_gdecide(double *__restrict__ T, int64_t ld, int32_t m, int32_t n,
                                                 const double *__restrict__ A, const double *__restrict__ cv,
                                                 int32_t K, int32_t KF, SPart *__restrict__ sparts,
                                                 unsigned long long *__restrict__ cols_done, DevState *__restrict__ st,
                                                 GroupState *__restrict__ gs, double *__restrict__ Fk,
                                                 double *__restrict__ Rk, int32_t *__restrict__ cols,
                                                 int32_t *__restrict__ pos, int32_t *__restrict__ basis,
                                                 int32_t *__restrict__ log_r, int32_t *__restrict__ log_q,
                                                 GRatio *__restrict__ rparts, GridSync *__restrict__ gsync,
                                                 uint32_t spin_limit, uint32_t gate_spin, double *__restrict__ PV,
                                                 unsigned char *pub, int32_t pub_words, uint32_t *pub_seq_at,
                                                 uint32_t pub_seq, unsigned long long *t_mark) {
    // the start of a solve, by the device's constant-rate clock (instead of
    // an event in the stream, which would delay this dispatch)
    if (t_mark && blockIdx.x == 0 && threadIdx.x == 0)
        __hip_atomic_store(t_mark, (unsigned long long)wall_clock64(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    decide_body<BD, First, KM>(T, ld, m, n, A, cv, K, KF, sparts, cols_done, st, gs, Fk, Rk, cols, pos, basis, log_r,
                               log_q, rparts, gsync, spin_limit, gate_spin, PV);
    // every workgroup leaves through here; the last one advances the epoch,
    // so the next launch's records carry a new flag, and reopens the gate
    __shared__ int32_t s_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const bool last = atomicAdd(&gsync->exits, 1u) == (uint32_t)gridDim.x - 1;
        if (last) {
            gsync->exits = 0;
            gsync->count = 0;  // the gate opens for the next launch
            gsync->epoch = gsync->epoch + 1u;
            __threadfence();
        }
        s_last = last;
    }
    __syncthreads();
    // The last workgroup also hands the solver state and the work counters
    // to the host: every workgroup's writes to them came before its exit
    // count (fences), the copy goes to mapped host memory, then the sequence
    // word after a system-scope fence. The host reads them there while the
    // update pass runs, with no copy and no event in the stream.
    if (pub && s_last) {
        const uint64_t *src = reinterpret_cast<const uint64_t *>(st);
        uint64_t *dst = reinterpret_cast<uint64_t *>(pub);
        for (int k = threadIdx.x; k < pub_words; k += BD)
            dst[k] = __hip_atomic_load(src + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence_system();
        __syncthreads();
        if (threadIdx.x == 0) __hip_atomic_store(pub_seq_at, pub_seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// Closes the gate of the next decision launch (kGateClosed): its workgroups
// then find it closed, as they would when they could not all be resident
// (a host-forced test of the fallback).
static __global__ void k_gate_close(GridSync *gsync) { gsync->count = kGateClosed; }

// Resumes a solve whose decision launch closed its gate (kStallGate; nothing
// of that launch was written): the open group is closed (groups of up to
// kMaxFuse pivots), the status returns to LP_RUNNING and the next Step 1
// scans row 0 (the pure update pass leaves no partials for the barrier-free
// kernels). One thread.
static __global__ void k_grecover(DevState *st, GroupState *gs, int32_t *__restrict__ cols, int32_t *__restrict__ pos,
                                  int32_t n) {
    if (gs->stalled != kStallGate) return;
    close_group_n<kMaxFuse>(gs, cols, pos, n);
    gs->stalled = 0;
    if (st->status == LP_STALLED) st->status = LP_RUNNING;
    st->fresh = 1;
}

// Step 3 for the whole group in one pass over (row chunk, slot group) tiles:
// every listed column is read once, has the group's pivots applied in order,
// and is written once. A row chunk is B rows (one per thread: with two, the
// compiler runs one row's whole chain before the other's and keeps every R
// entry of the tile live in between); a slot group is C consecutive list
// slots. The row-chunk-0 workgroup of each slot group reduces its new row-0
// entries to one Step 1 partial and counts the columns the group changed
// (some R_k nonzero).
//
// KF >= the context's group size K (instances exist for a few sizes). Full
// slot groups take a straight-line path: the pivot-column loads, the tile's
// columns, the tile's R entries into LDS, one barrier, the chain, and stores
// predicated on the row range (threads past row m load row 0 and store
// nothing), so the last row chunk needs no separate code. Pivots the group
// did not reach (kd <= k < KF) are applied as exact identities, with R = 0,
// F = 0 and no pivot row: fma(-0, 0, x) returns x for every x, signed zeros,
// infinities and NaN included. The last, partial slot group takes a plain
// loop.
template <int B, int C, int KF>
__global__ __launch_bounds__(B) void k_gupdate(double *__restrict__ T, int64_t ld, int32_t m, int32_t n, int64_t Lg,
                                               int32_t rowchunks, const int32_t *__restrict__ cols,
                                               const double *__restrict__ Rk, const double *__restrict__ Fk,
                                               const GroupState *__restrict__ gs, ArgMin *__restrict__ parts,
                                               unsigned long long *__restrict__ cols_done) {
    __shared__ double sR[C][KF];
    const int kd = gs->kdone;
    if (kd == 0) return;
    const int32_t Lv = n + 1 + gs->napp;
    const int32_t rc = (int32_t)(blockIdx.x % (uint32_t)rowchunks);
    const int32_t g = (int32_t)(blockIdx.x / (uint32_t)rowchunks);
    const int32_t c0 = g * C;
    const bool row0 = rc == 0 && threadIdx.x == 0;  // holds row 0, never a pivot row
    if (c0 >= Lv) {
        if (row0) parts[g] = ArgMin{__builtin_inf(), kNoIndex};
        return;
    }
    const int32_t i = rc * B + (int32_t)threadIdx.x;
    const bool live = i <= m;
    const int32_t is = live ? i : 0;

    if (c0 + C <= Lv) {
        int32_t rk[KF];
        double f[KF];
#pragma unroll
        for (int k = 0; k < KF; ++k) {
            const bool on = k < kd;
            rk[k] = on ? gs->r[k] : -1;
            f[k] = Fk[(int64_t)k * ld + is];
            if (!on) f[k] = 0.0;
        }
        double *p[C];
        double x[C];
#pragma unroll
        for (int c = 0; c < C; ++c) p[c] = T + (int64_t)cols[c0 + c] * ld + is;
#pragma unroll
        for (int c = 0; c < C; ++c) x[c] = *p[c];
        for (int t = threadIdx.x; t < C * KF; t += B) {  // C * KF may exceed B
            const int k = t % KF, c = t / KF;
            sR[c][k] = k < kd ? Rk[(int64_t)k * Lg + c0 + c] : 0.0;
        }
        __syncthreads();
        const int32_t wrow0 = rc * B + (int32_t)(threadIdx.x & ~63u);  // first row of this wave
#pragma unroll
        for (int k = 0; k < KF; ++k) {
            double R[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                R[c] = sR[c][k];
                x[c] = fma(-f[k], R[c], x[c]);
            }
            // only the wave that holds pivot row r_k replaces that row's
            // entries by R (a uniform test; the fma results there are dropped)
            if ((uint32_t)(rk[k] - wrow0) < 64u) {
#pragma unroll
                for (int c = 0; c < C; ++c)
                    if (i == rk[k]) x[c] = R[c];
            }
        }
        if (live) {
#pragma unroll
            for (int c = 0; c < C; ++c) *p[c] = x[c];
        }
        if (row0) {
            double val = __builtin_inf();
            int32_t idx = kNoIndex;
            unsigned long long changed = 0;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int32_t jc = cols[c0 + c];
                if (jc != n + m && lex_less(x[c], jc, val, idx)) {
                    val = x[c];
                    idx = jc;
                }
                bool nz = false;
                for (int k = 0; k < kd; ++k) nz |= Rk[(int64_t)k * Lg + c0 + c] != 0.0;
                changed += nz;
            }
            parts[g] = ArgMin{val, idx};
            if (changed) atomicAdd(cols_done, changed);
        }
        return;
    }

    // The last, partial slot group.
    const int cn = min(C, Lv - c0);
    double val = __builtin_inf();
    int32_t idx = kNoIndex;
    unsigned long long changed = 0;
    for (int c = 0; c < cn; ++c) {
        const int32_t jc = cols[c0 + c];
        double *cp = T + (int64_t)jc * ld + is;
        double x = *cp;
        bool nz = false;
#pragma unroll 1
        for (int k = 0; k < kd; ++k) {
            const double R = Rk[(int64_t)k * Lg + c0 + c];
            const int32_t r = gs->r[k];
            nz |= R != 0.0;
            x = (i == r) ? R : fma(-Fk[(int64_t)k * ld + is], R, x);
        }
        if (live) *cp = x;
        changed += nz;
        if (row0 && jc != n + m && lex_less(x, jc, val, idx)) {
            val = x;
            idx = jc;
        }
    }
    if (row0) {
        parts[g] = ArgMin{val, idx};
        if (changed) atomicAdd(cols_done, changed);
    }
}

// The update pass used with the one-launch decision kernel: loads, the
// chain, stores, and nothing else (any conditional work after the chain --
// a row-0 reduction, a partial last tile -- made the compiler keep far more
// live: 360 VGPRs instead of 125 at 8 slots x 16 pivots). The decision kernel
// does that work instead: it reads row 0 after the update for the next
// pricing, counts the changed columns, and stores exact identities for the
// pivots a group did not reach (F = 0, R = 0, pivot row -1), so every pass
// applies KF pivots without masking. A thread owns one row pair (two rows),
// threads past the last pair load pair 0 and store nothing; slots past the
// list (and the padding to a whole slot group) point at a zero column `dump`
// whose R entries are 0, so every workgroup takes the same straight path.
template <int B, int C, int KF>
__device__ __forceinline__ void pure_tile(double *__restrict__ T, int64_t ld, int32_t m, int64_t Lg, int32_t Lv,
                                          int32_t rc, int32_t c0, const int32_t *__restrict__ cols,
                                          const double *__restrict__ Rk, const double *__restrict__ Fk,
                                          const GroupState *__restrict__ gs, double *__restrict__ dump) {
    __shared__ double sR[C][KF];
    const int32_t nvec = (m + 2) / 2;
    const int32_t v = rc * B + (int32_t)threadIdx.x;
    const bool live = v < nvec;
    const int32_t vs = live ? v : 0;
    const int32_t i0 = 2 * v;
    const int64_t ldv = ld / 2;
    const double2 *F2 = reinterpret_cast<const double2 *>(Fk);
    double2 f[KF];
#pragma unroll
    for (int k = 0; k < KF; ++k) f[k] = F2[k * ldv + vs];
    double2 *p[C];
    double2 x[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int32_t jc = cols[c0 + c];
        p[c] = reinterpret_cast<double2 *>(jc >= 0 && c0 + c < Lv ? T + (int64_t)jc * ld : dump) + vs;
    }
#pragma unroll
    for (int c = 0; c < C; ++c) x[c] = nt_load2(p[c]);
    for (int t = threadIdx.x; t < C * KF; t += B) {  // C * KF may exceed B
        const int k = t % KF, c = t / KF;
        sR[c][k] = c0 + c < Lv ? Rk[(int64_t)k * Lg + c0 + c] : 0.0;
    }
    __syncthreads();
    // the chain without the pivot-row select: k_gfix then stores the pivot
    // rows (their values after the group, from the decision kernel)
#pragma unroll
    for (int k = 0; k < KF; ++k)
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const double R = sR[c][k];
            x[c].x = fma(-f[k].x, R, x[c].x);
            x[c].y = fma(-f[k].y, R, x[c].y);
        }
    if (live) {
#pragma unroll
        for (int c = 0; c < C; ++c) nt_store2(p[c], x[c]);
    }
}

template <int B, int C, int KF>
__global__ __launch_bounds__(B) void k_gupdate_pure(double *__restrict__ T, int64_t ld, int32_t m, int32_t n,
                                                    int64_t Lg, int32_t rowchunks, const int32_t *__restrict__ cols,
                                                    const double *__restrict__ Rk, const double *__restrict__ Fk,
                                                    const GroupState *__restrict__ gs, double *__restrict__ dump,
                                                    int32_t slot0) {
    if (gs->kdone == 0 || gs->stalled) return;
    const int32_t Lv = n + 1 + gs->napp;
    const int32_t rc = (int32_t)(blockIdx.x % (uint32_t)rowchunks);
    const int32_t g = (int32_t)(blockIdx.x / (uint32_t)rowchunks);
    const int32_t c0 = slot0 + g * C;  // slots from slot0 on
    if (c0 >= Lv) return;
    pure_tile<B, C, KF>(T, ld, m, Lg, Lv, rc, c0, cols, Rk, Fk, gs, dump);
}

// The first update pass after a deferred build: the Initialization Step of
// the structural columns and the first group's Step 3 in one pass. Column
// j < n sits in list slot j during the first group, so a tile of A (row 0:
// -c) is read row-major, transposed through LDS and written to the tableau
// after the group's KF pivots are applied to it, with the same chain as the
// pure pass applies to a built column (the same operations in the same order
// on the same start value, hence the same bits; like the pure pass it runs
// the chain without the pivot-row select, and k_gfix stores the pivot rows).
// A group of no pivots writes the tile as the plain build does. The pure
// pass takes the slots from n on (the right-hand side, built by k_ginit, and
// the columns appended during the group, which the decision kernel stored as
// unit vectors when they left the basis).
constexpr int kFirstRows = 32;  // tile rows (tableau rows)
constexpr int kFirstTile = 64;  // tile columns
constexpr int kFirstTailC = 1;  // slots per workgroup of the tail (few registers: the tile's F stays the largest)

// Workgroups from `tiles` on take the tail instead: the pure pass over the
// slots from n on (the RHS and the columns appended during the group),
// kFirstTailC slots by 512 rows each, in the same launch.
template <int KF>
__global__ __launch_bounds__(256) void k_gfirst(double *__restrict__ T, int64_t ld, int32_t m, int32_t n, int64_t Lg,
                                                int32_t ntx, const double *__restrict__ A, const double *__restrict__ cv,
                                                const double *__restrict__ Rk, const double *__restrict__ Fk,
                                                const GroupState *__restrict__ gs, int32_t tiles, int32_t rowchunks,
                                                const int32_t *__restrict__ cols, double *__restrict__ dump) {
    if ((int32_t)blockIdx.x >= tiles) {
        if (gs->kdone == 0 || gs->stalled) return;
        const int32_t Lv = n + 1 + gs->napp;
        const int32_t b = (int32_t)blockIdx.x - tiles;
        const int32_t rc = b % rowchunks, g = b / rowchunks;
        const int32_t c0 = n + g * kFirstTailC;
        if (c0 >= Lv) return;
        pure_tile<256, kFirstTailC, KF>(T, ld, m, Lg, Lv, rc, c0, cols, Rk, Fk, gs, dump);
        return;
    }
    constexpr int TR = kFirstRows, TC = kFirstTile;
    constexpr int NP = TR / 2;          // row pairs of a tile
    constexpr int CG = 256 / NP;        // column groups of the write phase
    constexpr int NR = (KF * TC + 255) / 256;  // R entries per thread to stage
    constexpr int NF = (KF * NP + 255) / 256;  // F pairs per thread to stage
    const int32_t kd = gs->stalled ? 0 : gs->kdone;  // a stalled group: the build alone
    __shared__ double tile[TR][TC + 1];
    __shared__ double sR[KF][TC];
    __shared__ double2 sF[KF][NP];
    const int64_t j0 = (int64_t)(blockIdx.x % (uint32_t)ntx) * TC;
    const int64_t i0 = (int64_t)(blockIdx.x / (uint32_t)ntx) * TR;
    const int tid = threadIdx.x;
    // the group's R entries of the tile's columns and F entries of its rows,
    // loaded first so that they arrive with the tile
    double rv[NR];
    double2 fv[NF];
    if (kd > 0) {
        const double2 *F2 = reinterpret_cast<const double2 *>(Fk);
        const int64_t ldv = ld / 2;
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const int t = tid + 256 * u, k = t / TC, cl = t % TC;
            rv[u] = t < KF * TC && j0 + cl < n ? Rk[(int64_t)k * Lg + j0 + cl] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NF; ++u) {
            const int t = tid + 256 * u, k = t / NP, v = t % NP;
            fv[u] = t < KF * NP && i0 + 2 * v < ld ? F2[k * ldv + i0 / 2 + v] : double2{0.0, 0.0};
        }
    }
    {  // the tile of A: 16-byte loads need an even n and a 16-byte aligned A
        const int pr = tid & 31, rw = tid >> 5;  // column pair, row group
        const bool vec_a = (n & 1) == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0;
        double2 va[TR / 8];
#pragma unroll
        for (int k = 0; k < TR / 8; ++k) {
            const int64_t i = i0 + rw + 8 * k, j = j0 + 2 * pr;
            double2 v = {0.0, 0.0};
            if (i == 0) {
                if (j < n) v.x = -cv[j];
                if (j + 1 < n) v.y = -cv[j + 1];
            } else if (i <= m) {
                const double *a = A + (i - 1) * n + j;
                if (vec_a && j + 1 < n) {  // j is even
                    v = nt_load2(a);
                } else {
                    if (j < n) v.x = a[0];
                    if (j + 1 < n) v.y = a[1];
                }
            }
            va[k] = v;
        }
        if (kd > 0) {
#pragma unroll
            for (int u = 0; u < NR; ++u) {
                const int t = tid + 256 * u;
                if (t < KF * TC) sR[t / TC][t % TC] = rv[u];
            }
#pragma unroll
            for (int u = 0; u < NF; ++u) {
                const int t = tid + 256 * u;
                if (t < KF * NP) sF[t / NP][t % NP] = fv[u];
            }
        }
#pragma unroll
        for (int k = 0; k < TR / 8; ++k) {
            tile[rw + 8 * k][2 * pr] = va[k].x;
            tile[rw + 8 * k][2 * pr + 1] = va[k].y;
        }
    }
    __syncthreads();
    // write phase: row pair p of the tile (rows iw, iw + 1; ld is even, so
    // both exist when the first does), columns cg + CG u
    const int p = tid % NP, cg = tid / NP;
    const int64_t iw = i0 + 2 * p;
    if (iw >= ld) return;
    if (kd == 0) {
#pragma unroll
        for (int u = 0; u < TC / CG; ++u) {
            const int cl = cg + CG * u;
            const int64_t j = j0 + cl;
            if (j < n) nt_store2(T + j * ld + iw, double2{tile[2 * p][cl], tile[2 * p + 1][cl]});
        }
        return;
    }
    // the chain without the pivot-row select: k_gfix then stores the pivot
    // rows (their values after the group, from the decision kernel)
    if constexpr (KF >= 32) {
        // F read from LDS in the chain (one column at a time), not held in
        // 4 KF registers: the occupancy of the smaller groups
#pragma unroll 1
        for (int u = 0; u < TC / CG; ++u) {
            const int cl = cg + CG * u;
            const int64_t j = j0 + cl;
            double2 x{tile[2 * p][cl], tile[2 * p + 1][cl]};
#pragma unroll
            for (int k = 0; k < KF; ++k) {
                const double R = sR[k][cl];
                const double2 f = sF[k][p];
                x.x = fma(-f.x, R, x.x);
                x.y = fma(-f.y, R, x.y);
            }
            if (j < n) nt_store2(T + j * ld + iw, x);
        }
    } else {
        double2 f[KF];
#pragma unroll
        for (int k = 0; k < KF; ++k) f[k] = sF[k][p];
#pragma unroll
        for (int u = 0; u < TC / CG; ++u) {
            const int cl = cg + CG * u;
            const int64_t j = j0 + cl;
            double2 x{tile[2 * p][cl], tile[2 * p + 1][cl]};
#pragma unroll
            for (int k = 0; k < KF; ++k) {
                const double R = sR[k][cl];
                x.x = fma(-f[k].x, R, x.x);
                x.y = fma(-f[k].y, R, x.y);
            }
            if (j < n) nt_store2(T + j * ld + iw, x);
        }
    }
}

// Row-lane tiles of the update pass (the form for groups of kRlFromKF
// pivots and more): a workgroup of 256 threads takes 128 rows by 64 list
// slots, wave w the slots 16w .. 16w+15 and lane l the row pair i0 + 2l,
// i0 + 2l + 1, so each load or store of a slot's column covers 128
// consecutive rows (1 KB, 16 bytes per lane) and each thread keeps 2 x 16
// entries. Per pivot k it reads F_k of its two rows (one 16-byte LDS read)
// and R_k of its 16 slots (scalar loads: the addresses are the same across the
// wave) for 32 fmas, so F and R stay out of the registers and the register
// count does not grow with KF. Rows past m are not stored (they hold zeros
// that no pivot changes). The chain runs without the pivot-row select
// (k_gfix stores the pivot rows): the same operations in the same order as
// pure_tile and k_gfirst.
constexpr int kRlRows = 128;  // rows per tile: a row pair per lane
constexpr int kRlSlots = 64;  // slots per tile: 16 per wave
constexpr int kRlPer = 16;    // slots per thread
constexpr int kRlFromKF = 32;  // groups of this many pivots and more take the row-lane tiles

// The pivots a row-lane or matrix-core pass applies: the group's kd rounded
// up to the chain's step (2 pivots, or 4 on the matrix cores), at most KF.
// The decision kernel stores the pivots from kd on as exact identities, so
// stopping there gives the same bits as running all KF.
template <int KF, int STEP>
__device__ __forceinline__ int chain_len(int32_t kd) {
    const int kn = (kd + STEP - 1) / STEP * STEP;
    return kn < KF ? kn : KF;
}

template <int KF>
__device__ __forceinline__ void rl_stage(double2 (*sF)[kRlRows / 2], const double *__restrict__ Fk, int64_t ld,
                                         int64_t i0, int kn) {
    const double2 *F2 = reinterpret_cast<const double2 *>(Fk);
    const int64_t ldv = ld / 2;  // (ld and i0 are even)
    for (int t = threadIdx.x; t < kn * (kRlRows / 2); t += 256) {
        const int k = t / (kRlRows / 2), v = t % (kRlRows / 2);
        const int64_t i = i0 + 2 * v;
        sF[k][v] = i < ld ? F2[(int64_t)k * ldv + i / 2] : double2{0.0, 0.0};
    }
}

// The chain over the wave's 16 slots for the lane's row pair: R_k of those
// slots through scalar loads (Rw points at R_0 of the wave's first slot;
// slots past the list read entries that are never stored), F_k from LDS;
// pivots 0 .. kn-1 (kn even).
template <int KF>
__device__ __forceinline__ void rl_chain(double2 (&x)[kRlPer], const double2 (*sF)[kRlRows / 2], const double *Rw,
                                         int64_t Lg, int lane, int kn) {
#pragma unroll 2
    for (int k = 0; k < kn; ++k) {
        const double2 f = sF[k][lane];
        const double *Rr = Rw + (int64_t)k * Lg;
#pragma unroll
        for (int u = 0; u < kRlPer; ++u) {
            const double R = Rr[u];
            x[u].x = fma(-f.x, R, x[u].x);
            x[u].y = fma(-f.y, R, x[u].y);
        }
    }
}

// The pure pass in row-lane tiles over slots slot0 .. n+napp.
template <int KF>
__global__ __launch_bounds__(256) void k_gpure_rl(double *__restrict__ T, int64_t ld, int32_t m, int32_t n,
                                                  int64_t Lg, int32_t nrt, const int32_t *__restrict__ cols,
                                                  const double *__restrict__ Rk, const double *__restrict__ Fk,
                                                  const GroupState *__restrict__ gs, int32_t slot0) {
    if (gs->kdone == 0 || gs->stalled) return;
    const int32_t Lv = n + 1 + gs->napp;
    const int32_t rt = (int32_t)(blockIdx.x % (uint32_t)nrt), ct = (int32_t)(blockIdx.x / (uint32_t)nrt);
    const int32_t s0 = slot0 + ct * kRlSlots;
    if (s0 >= Lv) return;
    __shared__ double2 sF[KF][kRlRows / 2];
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t i0 = (int64_t)rt * kRlRows, i = i0 + 2 * lane;  // the lane's first row
    const bool row_ok = i <= m;  // (then i + 1 < ld: ld is even)
    const int32_t sw = s0 + kRlPer * w;  // this wave's first slot
    // the wave's 16 columns: one load by lanes 0..15, then read from those
    // lanes (wave-uniform); every load address is valid (the row clamped into
    // the column, an unused slot reading column 0), the stores are masked
    const int32_t cl = lane < kRlPer && sw + lane < Lv ? cols[sw + lane] : -1;
    int32_t jc[kRlPer];
    double2 x[kRlPer];
    const int64_t ic = row_ok ? i : 0;
#pragma unroll
    for (int u = 0; u < kRlPer; ++u) {
        jc[u] = __builtin_amdgcn_readlane(cl, u);
        x[u] = *reinterpret_cast<const double2 *>(T + (int64_t)(jc[u] >= 0 ? jc[u] : 0) * ld + ic);
    }
    const int kn = chain_len<KF, 2>(gs->kdone);
    rl_stage<KF>(sF, Fk, ld, i0, kn);
    __syncthreads();
    rl_chain<KF>(x, sF, Rk + sw, Lg, lane, kn);
    if (row_ok) {
#pragma unroll
        for (int u = 0; u < kRlPer; ++u)
            if (jc[u] >= 0) *reinterpret_cast<double2 *>(T + (int64_t)jc[u] * ld + i) = x[u];
    }
}

// The first pass after a deferred build in row-lane tiles: slot j < n holds
// structural column j during the first group, so lane l reads rows i, i+1 of
// A (16 consecutive entries of each, row 0: -c; rows past m: zeros) and
// writes the entries after the group's pivots to the tableau, padding rows
// included. A group of no pivots writes the build alone. The slots from n on
// take the pure pass (slot0 = n).
template <int KF>
__global__ __launch_bounds__(256) void k_gfirst_rl(double *__restrict__ T, int64_t ld, int32_t m, int32_t n,
                                                   int64_t Lg, int32_t nrt, const double *__restrict__ A,
                                                   const double *__restrict__ cv, const double *__restrict__ Rk,
                                                   const double *__restrict__ Fk, const GroupState *__restrict__ gs) {
    const int32_t kd = gs->stalled ? 0 : gs->kdone;  // a stalled group: the build alone
    const int32_t rt = (int32_t)(blockIdx.x % (uint32_t)nrt), ct = (int32_t)(blockIdx.x / (uint32_t)nrt);
    const int32_t s0 = ct * kRlSlots;
    __shared__ double2 sF[KF][kRlRows / 2];
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t i0 = (int64_t)rt * kRlRows, i = i0 + 2 * lane;
    const int32_t sw = s0 + kRlPer * w;  // this wave's first structural column
    // 16-byte loads need an even n and a 16-byte aligned A (then every row
    // and every wave's first column are 16-byte aligned)
    const bool vec = (n & 1) == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0 && sw + kRlPer <= n;
    double e[2][kRlPer];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int64_t r = i + h;
        if (r == 0) {
#pragma unroll
            for (int u = 0; u < kRlPer; ++u) e[h][u] = sw + u < n ? -cv[sw + u] : 0.0;
        } else if (r <= m) {
            const double *a = A + (r - 1) * (int64_t)n + sw;
            if (vec) {
#pragma unroll
                for (int u = 0; u < kRlPer / 2; ++u) {
                    const double2 v = reinterpret_cast<const double2 *>(a)[u];
                    e[h][2 * u] = v.x;
                    e[h][2 * u + 1] = v.y;
                }
            } else {
#pragma unroll
                for (int u = 0; u < kRlPer; ++u) e[h][u] = sw + u < n ? a[u] : 0.0;
            }
        } else {
#pragma unroll
            for (int u = 0; u < kRlPer; ++u) e[h][u] = 0.0;
        }
    }
    double2 x[kRlPer];
#pragma unroll
    for (int u = 0; u < kRlPer; ++u) x[u] = double2{e[0][u], e[1][u]};
    if (kd > 0) {
        const int kn = chain_len<KF, 2>(kd);
        rl_stage<KF>(sF, Fk, ld, i0, kn);
        __syncthreads();
        rl_chain<KF>(x, sF, Rk + sw, Lg, lane, kn);
    }
    if (i < ld) {
#pragma unroll
        for (int u = 0; u < kRlPer; ++u)
            if (sw + u < n) *reinterpret_cast<double2 *>(T + (int64_t)(sw + u) * ld + i) = x[u];
    }
}

// The pure pass on the matrix cores. The pass is a rank-KF update of every
// listed column, X -= F R (F: the group's pivot columns, R: their
// normalised pivot rows), each entry a chain of fmas in pivot order. The FP64
// MFMA v_mfma_f64_16x16x4f64 computes D = A B + C as four fmas per entry in k
// order, one rounding each (the same bits as the chain, special values
// included), so four pivots at a time run as one MFMA with A = -R (16 slots by
// 4 pivots), B = F (4 pivots by 16 rows) and C = the entries (16 slots by 16
// rows): fma(-R_k, F_k, x) equals fma(-F_k, R_k, x) (one exact product, one
// rounding). A workgroup takes 64 rows by 64 slots: wave w the slots
// 16w .. 16w+15 over four tiles of 16 rows. The matrix layout of the
// instruction: A lane l = A[l % 16][l / 16], B lane l = B[l / 16][l % 16],
// C/D lane l element e = D[4e + l / 16][l % 16], so element e of a lane is row
// l % 16 of slot 4e + l / 16: every load and store covers 16 consecutive rows
// (128 bytes) of four columns. Rows up to the padded length are rewritten
// (the padding holds zeros that no pivot changes).
typedef double v4d_t __attribute__((ext_vector_type(4)));
constexpr int kMfWr = 1;                    // waves stacked along the rows of a tile
constexpr int kMfRows = 64 * kMfWr;         // rows per tile
constexpr int kMfSlots = 16 * (4 / kMfWr);  // slots per tile

template <int KF>
__device__ __forceinline__ void mf_stage(double (*sF)[kMfRows], const double *__restrict__ Fk, int64_t ld, int64_t i0,
                                         int kn) {
    for (int t = threadIdx.x; t < kn * kMfRows; t += 256) {
        const int k = t / kMfRows, l = t % kMfRows;
        const int64_t i = i0 + l;
        sF[k][l] = i < ld ? Fk[(int64_t)k * ld + i] : 0.0;
    }
}

// acc[rt] (row tile rt of the wave's 64 rows, from tile row r0) after
// pivots 0 .. kn-1 (kn a multiple of 4): the A operand (-R of the lane's
// slot row l % 16, pivot 4s + l / 16) from memory, the B operand (F of row
// r0 + 16 rt + l % 16, pivot 4s + l / 16) from LDS.
template <int KF>
__device__ __forceinline__ void mf_chain(v4d_t (&acc)[4], const double (*sF)[kMfRows], const double *__restrict__ Rk,
                                         int64_t Lg, int32_t sw, int r0, int lane, int kn) {
    const int kq = lane >> 4, ll = lane & 15;
#pragma unroll 4
    for (int s = 0; s < kn / 4; ++s) {
        const double r = -Rk[(int64_t)(4 * s + kq) * Lg + sw + ll];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
            const double f = sF[4 * s + kq][r0 + 16 * rt + ll];
            acc[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(r, f, acc[rt], 0, 0, 0);
        }
    }
}

template <int KF>
__global__ __launch_bounds__(256) void k_gpure_mf(double *__restrict__ T, int64_t ld, int32_t m, int32_t n, int64_t Lg,
                                                  int32_t nrt, const int32_t *__restrict__ cols,
                                                  const double *__restrict__ Rk, const double *__restrict__ Fk,
                                                  const GroupState *__restrict__ gs, int32_t slot0) {
    static_assert(KF % 4 == 0, "four pivots per MFMA");
    if (gs->kdone == 0 || gs->stalled) return;
    const int32_t Lv = n + 1 + gs->napp;
    const int32_t rtile = (int32_t)(blockIdx.x % (uint32_t)nrt), ct = (int32_t)(blockIdx.x / (uint32_t)nrt);
    const int32_t s0 = slot0 + ct * kMfSlots;
    if (s0 >= Lv) return;
    __shared__ double sF[KF][kMfRows];
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wr = w % kMfWr, ws = w / kMfWr;
    const int64_t i0 = (int64_t)rtile * kMfRows;
    const int r0 = 64 * wr;  // the wave's first row in the tile
    const int32_t sw = s0 + 16 * ws;
    const int kq = lane >> 4, ll = lane & 15;
    // element e of the lane: slot sw + 4e + kq; its column (or -1)
    int32_t jc[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int32_t sl = sw + 4 * e + kq;
        jc[e] = sl < Lv ? cols[sl] : -1;
    }
    v4d_t acc[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
        const int64_t row = i0 + r0 + 16 * rt + ll;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            acc[rt][e] = jc[e] >= 0 && row < ld ? T[(int64_t)jc[e] * ld + row] : 0.0;
    }
    const int kn = chain_len<KF, 4>(gs->kdone);
    mf_stage<KF>(sF, Fk, ld, i0, kn);
    __syncthreads();
    mf_chain<KF>(acc, sF, Rk, Lg, sw, r0, lane, kn);
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
        const int64_t row = i0 + r0 + 16 * rt + ll;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (jc[e] >= 0 && row < ld) T[(int64_t)jc[e] * ld + row] = acc[rt][e];
    }
}

// The pivot rows of the group's list columns after its update pass: row
// r_a of the column in slot t takes PV[a][t], its value after the group that
// the decision kernel computed (the pass applied the chain without the
// pivot-row select, which only these rows need). A row that pivots twice gets
// the same value from both entries.
static __global__ __launch_bounds__(256) void k_gfix(double *__restrict__ T, int64_t ld, int32_t n, int64_t Lg,
                                                     const int32_t *__restrict__ cols, const double *__restrict__ PV,
                                                     const GroupState *__restrict__ gs) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t a = (int32_t)(idx / Lg), t = (int32_t)(idx % Lg);
    if (a >= gs->kdone || gs->stalled || t > n + gs->napp) return;
    const int32_t c = cols[t];
    if (c >= 0) T[(int64_t)c * ld + gs->r[a]] = PV[idx];
}

}  // namespace lpgpu
