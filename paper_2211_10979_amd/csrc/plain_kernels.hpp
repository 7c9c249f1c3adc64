// Kernels of the single-LP solver. The tableau is column-major with a padded
// leading dimension `ld` (multiple of 16 doubles): T[i][j] = T[j*ld + i].
//
// One pivot is two launches on one stream:
//   k_select  one workgroup: final stage of the Step 1 argmin over the
//             per-workgroup partials of the previous update (or a scan of
//             row 0 on the first pivot), the Step 2 ratio test over column q,
//             the snapshot F of column q, and the pivot log;
//   k_update  one workgroup per tile of whole columns: Step 3 (normalise the
//             pivot row and eliminate) in place, plus the first stage of the
//             next Step 1 argmin over the tile's new row-0 entries.
// Stream order is the only synchronisation: no host round trip per pivot.
#pragma once

#include "common.hpp"

namespace lpgpu {

constexpr int kBuildTile = 64;

// Initialization Step, structural part: column j < n of T gets -c_j in row 0
// and column j of A in rows 1..m (Table I); padding rows are zero. A is
// row-major, so each 64x64 tile is transposed through LDS; both sides move
// 16 bytes per thread access (two columns of a row of A, two rows of a
// column of T).
static __global__ __launch_bounds__(256) void k_build_struct(double *__restrict__ T, int64_t ld, int32_t m, int32_t n,
                                                             const double *__restrict__ A, const double *__restrict__ c) {
    __shared__ double tile[kBuildTile][kBuildTile + 1];
    const int64_t j0 = (int64_t)blockIdx.x * kBuildTile;
    const int64_t i0 = (int64_t)blockIdx.y * kBuildTile;
    const int pr = threadIdx.x & 31, rw = threadIdx.x >> 5;  // pair within a tile row, row group
    // 16-byte loads of A need an even n (every row starts 16-byte aligned)
    // and an aligned A (a caller's device array may be any view)
    const bool vec_a = (n & 1) == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0;
#pragma unroll
    for (int k = 0; k < kBuildTile / 8; ++k) {
        const int r = rw + 8 * k;
        const int64_t i = i0 + r, j = j0 + 2 * pr;
        double2 v = {0.0, 0.0};
        if (i == 0) {
            if (j < n) v.x = -c[j];
            if (j + 1 < n) v.y = -c[j + 1];
        } else if (i <= m) {
            const double *a = A + (i - 1) * n + j;
            if (vec_a && j + 1 < n) {  // j is even
                v = *reinterpret_cast<const double2 *>(a);
            } else {
                if (j < n) v.x = a[0];
                if (j + 1 < n) v.y = a[1];
            }
        }
        tile[r][2 * pr] = v.x;
        tile[r][2 * pr + 1] = v.y;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kBuildTile / 8; ++k) {
        const int cl = rw + 8 * k;
        const int64_t j = j0 + cl, i = i0 + 2 * pr;
        if (j < n && i + 1 < ld) {  // ld is even: rows i, i+1 both exist
            double2 v;
            v.x = tile[2 * pr][cl];
            v.y = tile[2 * pr + 1][cl];
            *reinterpret_cast<double2 *>(T + j * ld + i) = v;
        }
    }
}

// Initialization Step, slack identity and right-hand side: columns
// n .. n+ncols-1, where ncols is m (the slack columns only; b is not read) or
// m + 1 (and the RHS column from b).
static __global__ __launch_bounds__(256) void k_build_slack(double *__restrict__ T, int64_t ld, int32_t m, int32_t n,
                                                     const double *__restrict__ b, int32_t ncols) {
    const int64_t half = ld / 2;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)ncols * half) return;
    const int64_t s = idx / half, v = idx % half;
    const int64_t i0 = 2 * v, i1 = 2 * v + 1;
    double2 y;
    if (s < m) {
        y.x = (i0 == s + 1) ? 1.0 : 0.0;
        y.y = (i1 == s + 1) ? 1.0 : 0.0;
    } else {
        y.x = (i0 >= 1 && i0 <= m) ? b[i0 - 1] : 0.0;
        y.y = (i1 >= 1 && i1 <= m) ? b[i1 - 1] : 0.0;
    }
    reinterpret_cast<double2 *>(T + (n + s) * ld)[v] = y;
}

// Solver state, slack basis, a zeroed pivot-column buffer, the list of
// columns Step 3 rewrites and the work counter.
//   cols[0..n)  the nonbasic columns (any order); cols[n] the entering column
//               of the current pivot; cols[n+1] the right-hand side W-1;
//   pos[j]      position of column j in cols[0..n), or -1 when j is basic.
static __global__ void k_init(DevState *st, DevState init, int32_t *__restrict__ basis, int32_t m, int32_t n,
                       double *__restrict__ F, int64_t ld, int32_t *__restrict__ cols, int32_t *__restrict__ pos,
                       unsigned long long *__restrict__ cols_done) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx == 0) {
        *st = init;
        *cols_done = 0;
        cols[n] = 0;
        cols[n + 1] = n + m;
    }
    if (idx < m) basis[idx] = n + (int32_t)idx;
    if (idx < ld) F[idx] = 0.0;
    if (idx < n) cols[idx] = (int32_t)idx;
    if (idx < (int64_t)n + m) pos[idx] = idx < n ? (int32_t)idx : -1;
}

static __global__ void k_set_stop(DevState *st, int64_t stop_at) { st->stop_at = stop_at; }

// Zeroes `words` 8-byte words (grid-stride): the clear of a new work block.
static __global__ __launch_bounds__(256) void k_zero_words(uint64_t *__restrict__ p, int64_t words) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// A forced pivot (r, q) = (st->force_r, st->force_q): column q copied to F,
// then the decision recorded as after Steps 1-2 (the cap still applies);
// the force is cleared. Used only by the general form's drive-out, whose host
// loop picks (r, q) with |T[r][q]| > eps_p.
__device__ __forceinline__ void select_forced(const double *__restrict__ T, int64_t ld, int32_t m, const DevState &s,
                                              DevState *__restrict__ st, double *__restrict__ F,
                                              int32_t *__restrict__ basis, int32_t *__restrict__ log_r,
                                              int32_t *__restrict__ log_q, const int32_t *__restrict__ pos, int tid,
                                              int nt) {
    const int32_t q = s.force_q, r = s.force_r;
    const double *colq = T + (int64_t)q * ld;
    for (int32_t i = tid; i <= m; i += nt) F[i] = colq[i];
    if (tid != 0) return;
    st->force_q = -1;
    st->force_r = -1;
    if (s.pivots >= s.max_pivots) {
        st->status = LP_ITER_LIMIT;
        st->go = 0;
        return;
    }
    st->r = r;
    st->q = q;
    st->p = colq[r];
    st->leave = basis[r - 1];
    st->pq = pos[q];
    basis[r - 1] = q;
    if (s.pivots < s.log_cap) {
        log_r[s.pivots] = r;
        log_q[s.pivots] = q;
    }
    st->pivots = s.pivots + 1;
    st->go = 1;
}

// Steps 1 and 2 for the next pivot; one workgroup of 1024 threads.
//   Step 1   final stage of the argmin over the update's per-group partials
//            (a scan of row 0 before the first pivot);
//   Step 2   ratio test over column q, copying column q to F on the way;
//   then the decision (r, q, p, leaving column), the basis and the log.
// Basic columns other than the leaving one are exact unit vectors with a zero
// in row r and in row 0, so leaving them out of R, of the rewrite and of the
// Step 1 scan changes no value and no decision.
static __global__ __launch_bounds__(1024) void k_select(const double *__restrict__ T, int64_t ld, int32_t m, int32_t n,
                                                const ArgMin *__restrict__ parts, DevState *__restrict__ st,
                                                double *__restrict__ F, int32_t *__restrict__ basis,
                                                int32_t *__restrict__ log_r, int32_t *__restrict__ log_q,
                                                const int32_t *__restrict__ pos) {
    __shared__ double sv[16];
    __shared__ int32_t si[16];
    const int tid = threadIdx.x, nt = blockDim.x;
    const DevState s = *st;
    if (s.status != LP_RUNNING || s.pivots >= s.stop_at) {
        if (tid == 0) st->go = 0;
        return;
    }
    const int64_t W = (int64_t)n + m + 1;
    if (s.force_q >= 0) {  // a forced pivot: no Steps 1-2
        select_forced(T, ld, m, s, st, F, basis, log_r, log_q, pos, tid, nt);
        return;
    }
    const int32_t bar = s.bar;
    // the anti-cycling fallback: Bland's rule after bland_after degenerate pivots in a row
    const bool bland = s.bland_after > 0 && s.degen >= s.bland_after;

    // Step 1: most negative objective-row entry, lowest column on ties (under
    // Bland's rule the scan also finds the lowest column below -eps_d; the
    // minimum still decides optimality and the non-finite stop).
    double v = __builtin_inf();
    int32_t q = kNoIndex;
    int32_t qb = kNoIndex;
    if (s.fresh || bland) {
        for (int32_t j = tid; j < bar; j += nt) {
            const double t = T[(int64_t)j * ld];
            if (lex_less(t, j, v, q)) {
                v = t;
                q = j;
            }
            if (t < -s.eps_d && j < qb) qb = j;
        }
    } else {
        for (int32_t k = tid; k < s.nparts; k += nt) {
            const ArgMin a = parts[k];
            if (lex_less(a.v, a.i, v, q)) {
                v = a.v;
                q = a.i;
            }
        }
    }
    block_argmin(v, q, sv, si);
    if (step1_bad(v) || v >= -s.eps_d) {
        if (tid == 0) {
            st->status = step1_bad(v) ? LP_NUMERICAL : LP_OPTIMAL;
            st->go = 0;
        }
        return;
    }
    if (bland) {  // the lowest eligible column
        double zb = qb == kNoIndex ? __builtin_inf() : 0.0;
        block_argmin(zb, qb, sv, si);
        q = qb;
    }

    // Step 2: minimum ratio over rows with T[i][q] > eps_p, lowest row on ties
    // (under Bland's rule, the row whose basic variable has the lowest index).
    // The pivot column is also copied to F on the way (used only if a pivot
    // follows).
    const double *colq = T + (int64_t)q * ld;
    const double *rhs = T + (W - 1) * ld;
    const int32_t pq = pos[q];
    double rv = __builtin_inf();
    int32_t r = kNoIndex;
    int bad = 0;
    const bool barred_rows = bar < n + m;  // the general form: some rows may not leave
    if (tid == 0) F[0] = colq[0];
    for (int32_t i = 1 + tid; i <= m; i += nt) {
        const double a = colq[i], bb = rhs[i];
        F[i] = a;
        if (step2_bad(a, bb)) {
            bad = 1;
        } else if (a > s.eps_p && (!barred_rows || basis[i - 1] < bar)) {
            const double ratio = bb / a;
            const int32_t key = bland ? basis[i - 1] : i;
            if (lex_less(ratio, key, rv, r)) {
                rv = ratio;
                r = key;
            }
        }
    }
    bad = __syncthreads_or(bad);
    block_argmin(rv, r, sv, si);
    if (bland && !bad && r != kNoIndex) {  // the row of the winning basic variable
        __shared__ int32_t s_row;
        const int32_t kb = r;
        for (int32_t i = 1 + tid; i <= m; i += nt)
            if (basis[i - 1] == kb) s_row = i;
        __syncthreads();
        r = s_row;
    }
    if (bad || r == kNoIndex || s.pivots >= s.max_pivots) {
        if (tid == 0) {
            st->status = bad ? LP_NUMERICAL : (r == kNoIndex ? LP_UNBOUNDED : LP_ITER_LIMIT);
            st->go = 0;
        }
        return;
    }

    // Decision made: the staging kernel prepares Step 3's inputs.
    if (tid == 0) {
        const int32_t leave = basis[r - 1];
        st->r = r;
        st->q = q;
        st->p = colq[r];
        st->leave = leave;
        st->pq = pq;
        basis[r - 1] = q;
        if (s.pivots < s.log_cap) {
            log_r[s.pivots] = r;
            log_q[s.pivots] = q;
        }
        st->pivots = s.pivots + 1;
        st->fresh = 0;
        st->degen = rv <= s.eps_p ? s.degen + 1 : 0;  // the step of this pivot
        st->go = 1;
    }
}

// Steps 1 and 2 spread over G workgroups of 1024 threads. Every workgroup
// reduces all Step 1 partials itself (so all agree on q without waiting for
// each other), then takes rows [1 + w*span, ...) of the ratio test and of the
// copy of column q to F, and writes one (ratio, row) partial. The last
// workgroup to finish (atomic ticket, device-scope fences around it) reduces
// those partials and records the decision exactly as k_select does.
struct RatioPart {
    double v;
    int32_t i;
    int32_t bad;
};

static __global__ __launch_bounds__(1024) void k_select_mw(const double *__restrict__ T, int64_t ld, int32_t m,
                                                           int32_t n, const ArgMin *__restrict__ parts,
                                                           DevState *__restrict__ st, double *__restrict__ F,
                                                           int32_t *__restrict__ basis, int32_t *__restrict__ log_r,
                                                           int32_t *__restrict__ log_q, const int32_t *__restrict__ pos,
                                                           RatioPart *__restrict__ rparts, uint32_t *__restrict__ ticket) {
    __shared__ double sv[16];
    __shared__ int32_t si[16];
    __shared__ uint32_t s_last;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int G = gridDim.x, w = blockIdx.x;
    const DevState s = *st;
    if (s.status != LP_RUNNING || s.pivots >= s.stop_at) {
        if (w == 0 && tid == 0) st->go = 0;
        return;
    }
    const int64_t W = (int64_t)n + m + 1;
    double v = __builtin_inf();
    int32_t q = kNoIndex;
    if (s.fresh) {
        for (int32_t j = tid; j < n + m; j += nt) {
            const double t = T[(int64_t)j * ld];
            if (lex_less(t, j, v, q)) {
                v = t;
                q = j;
            }
        }
    } else {
        for (int32_t k = tid; k < s.nparts; k += nt) {
            const ArgMin a = parts[k];
            if (lex_less(a.v, a.i, v, q)) {
                v = a.v;
                q = a.i;
            }
        }
    }
    block_argmin(v, q, sv, si);
    if (step1_bad(v) || v >= -s.eps_d) {
        if (w == 0 && tid == 0) {
            st->status = step1_bad(v) ? LP_NUMERICAL : LP_OPTIMAL;
            st->go = 0;
        }
        return;
    }
    const double *colq = T + (int64_t)q * ld;
    const double *rhs = T + (W - 1) * ld;
    const int32_t span = (m + G - 1) / G;
    const int32_t i0 = 1 + w * span, i1 = min(m, i0 + span - 1);
    double rv = __builtin_inf();
    int32_t r = kNoIndex;
    int bad = 0;
    if (w == 0 && tid == 0) F[0] = colq[0];
    for (int32_t i = i0 + tid; i <= i1; i += nt) {
        const double a = colq[i], bb = rhs[i];
        F[i] = a;
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
    block_argmin(rv, r, sv, si);
    if (tid == 0) {
        rparts[w] = RatioPart{rv, r, bad};
        __threadfence();
        s_last = atomicAdd(ticket, 1u) == (uint32_t)(G - 1);
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    // last workgroup: the decision
    rv = __builtin_inf();
    r = kNoIndex;
    bad = 0;
    for (int k = tid; k < G; k += nt) {
        const RatioPart pr = rparts[k];
        bad |= pr.bad;
        if (lex_less(pr.v, pr.i, rv, r)) {
            rv = pr.v;
            r = pr.i;
        }
    }
    bad = __syncthreads_or(bad);
    block_argmin(rv, r, sv, si);
    if (tid != 0) return;
    *ticket = 0;  // ready for the next launch (ordered by the kernel boundary)
    if (bad || r == kNoIndex || s.pivots >= s.max_pivots) {
        st->status = bad ? LP_NUMERICAL : (r == kNoIndex ? LP_UNBOUNDED : LP_ITER_LIMIT);
        st->go = 0;
        return;
    }
    const int32_t leave = basis[r - 1];
    st->r = r;
    st->q = q;
    st->p = colq[r];
    st->leave = leave;
    st->pq = pos[q];
    basis[r - 1] = q;
    if (s.pivots < s.log_cap) {
        log_r[s.pivots] = r;
        log_q[s.pivots] = q;
    }
    st->pivots = s.pivots + 1;
    st->fresh = 0;
    st->go = 1;
}

// Inputs of Step 3 for the pivot k_select decided, one list position per
// thread: R_t = T[r][j_t] / p for the rewrite list with the leaving column in
// the entering column's place, and the count of nonzero R. Workgroup 0 then
// swaps the two columns in the list itself; no thread of this kernel reads
// the two entries it writes (positions pq and n), so the swap is race-free.
static __global__ __launch_bounds__(256) void k_stage(const double *__restrict__ T, int64_t ld, int32_t m, int32_t n,
                                                     const DevState *__restrict__ st, int32_t *__restrict__ cols,
                                                     int32_t *__restrict__ pos, double *__restrict__ Rl,
                                                     unsigned long long *__restrict__ cols_done) {
    if (!st->go) return;
    const int32_t r = st->r, q = st->q, leave = st->leave, pq = st->pq;
    const double p = st->p;
    const int32_t t = (int32_t)(blockIdx.x * 256 + threadIdx.x);
    bool nz = false;
    if (t < n + 2) {
        const int32_t j = t == pq ? leave : (t == n ? q : (t == n + 1 ? n + m : cols[t]));
        const double R = T[(int64_t)j * ld + r] / p;
        Rl[t] = R;
        nz = R != 0.0;
    }
    const unsigned long long cnt = __popcll(__ballot(nz));
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(cols_done, cnt);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        cols[pq] = leave;
        pos[leave] = pq;
        pos[q] = -1;
        cols[n] = q;
    }
}

// Step 3 as a streaming kernel over (row chunk, column group) tiles. A row
// chunk is B*RV row pairs (double2): thread t owns pairs v_k = base + k*B + t,
// k < RV, of each of the group's C listed columns. Every entry is read once
// and rewritten once:
//     T[i][j] = R_j                        for i = r,
//     T[i][j] = fma(-F_i, R_j, T[i][j])    otherwise.
// The row-chunk-0 workgroup of each column group also reduces its columns'
// new row-0 entries to one (value, column) partial for the next Step 1.
// 16-byte loads and stores, optionally with the non-temporal hint (the
// tableau streams through once per pivot).
typedef double v2d __attribute__((ext_vector_type(2)));

template <bool NT>
__device__ __forceinline__ double2 ld2(const double2 *p) {
    if constexpr (NT) {
        const v2d v = __builtin_nontemporal_load(reinterpret_cast<const v2d *>(p));
        return double2{v.x, v.y};
    } else {
        return *p;
    }
}

template <bool NT>
__device__ __forceinline__ void st2(double2 *p, const double2 &y) {
    if constexpr (NT) {
        v2d v = {y.x, y.y};
        __builtin_nontemporal_store(v, reinterpret_cast<v2d *>(p));
    } else {
        *p = y;
    }
}

template <int B, int C, int RV, int NTL = 0, int NTS = 0>
__global__ __launch_bounds__(B) void k_update(double *__restrict__ T, int64_t ld, int32_t m, int32_t n,
                                              int32_t rowchunks, const int32_t *__restrict__ cols,
                                              const double *__restrict__ Rl, const double *__restrict__ F,
                                              const DevState *__restrict__ st, ArgMin *__restrict__ parts) {
    if (!st->go) return;
    const int32_t r = st->r;
    const int32_t bar = st->bar;  // columns >= bar (the RHS among them) are no Step 1 candidates
    const int32_t ncols = n + 2;
    const int32_t rc = (int32_t)(blockIdx.x % (uint32_t)rowchunks);
    const int32_t g = (int32_t)(blockIdx.x / (uint32_t)rowchunks);
    const int32_t c0 = g * C;
    const int32_t nvec = (m + 2) / 2;
    const int32_t base = rc * B * RV + (int32_t)threadIdx.x;
    const double2 *F2 = reinterpret_cast<const double2 *>(F);
    const bool row0 = rc == 0 && threadIdx.x == 0;  // holds row 0, never the pivot row

    if (c0 + C <= ncols && (rc + 1) * B * RV <= nvec) {
        // Full tile: straight-line code, so that all C*RV loads are in flight
        // before the first store and no wait covers a store.
        double Rj[C];
        double2 *col[C];
        double2 f[RV];
        double2 x[C][RV];
#pragma unroll
        for (int k = 0; k < RV; ++k) f[k] = F2[base + k * B];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            Rj[c] = Rl[c0 + c];
            col[c] = reinterpret_cast<double2 *>(T + (int64_t)cols[c0 + c] * ld);
        }
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int k = 0; k < RV; ++k) x[c][k] = ld2<NTL != 0>(col[c] + base + k * B);
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int k = 0; k < RV; ++k) {
                const int32_t v = base + k * B;
                double2 y;
                y.x = (2 * v == r) ? Rj[c] : fma(-f[k].x, Rj[c], x[c][k].x);
                y.y = (2 * v + 1 == r) ? Rj[c] : fma(-f[k].y, Rj[c], x[c][k].y);
                st2<NTS != 0>(col[c] + v, y);
            }
        if (row0) {
            double val = __builtin_inf();
            int32_t idx = kNoIndex;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int32_t j = cols[c0 + c];
                const double y0 = fma(-f[0].x, Rj[c], x[c][0].x);
                if (j < bar && lex_less(y0, j, val, idx)) {
                    val = y0;
                    idx = j;
                }
            }
            parts[g] = ArgMin{val, idx};
        }
        return;
    }

    // Edge tile: the last column group or the last row chunk.
    const int cn = min(C, ncols - c0);
    double val = __builtin_inf();
    int32_t idx = kNoIndex;
    for (int c = 0; c < cn; ++c) {
        const double R = Rl[c0 + c];
        const int32_t j = cols[c0 + c];
        double2 *cp = reinterpret_cast<double2 *>(T + (int64_t)j * ld);
        for (int k = 0; k < RV; ++k) {
            const int32_t v = base + k * B;
            if (v < nvec) {
                const double2 f = F2[v];
                const double2 xx = cp[v];
                double2 y;
                y.x = (2 * v == r) ? R : fma(-f.x, R, xx.x);
                y.y = (2 * v + 1 == r) ? R : fma(-f.y, R, xx.y);
                cp[v] = y;
                if (row0 && k == 0 && j < bar && lex_less(y.x, j, val, idx)) {
                    val = y.x;
                    idx = j;
                }
            }
        }
    }
    if (row0) parts[g] = ArgMin{val, idx};
}

// Step 3, grid-stride form: a fixed grid walks the (row chunk, column) tiles
// of one column and B row pairs each, U tiles in flight per thread (all U
// loads issued before the first store). Tile t covers column list position
// t / rowchunks and row chunk t % rowchunks. Same arithmetic and Step 1
// partials (one per list position) as k_update<B, 1, 1>.
template <int B, int U>
__global__ __launch_bounds__(B) void k_update_gs(double *__restrict__ T, int64_t ld, int32_t m, int32_t n,
                                                 int32_t rowchunks, const int32_t *__restrict__ cols,
                                                 const double *__restrict__ Rl, const double *__restrict__ F,
                                                 const DevState *__restrict__ st, ArgMin *__restrict__ parts) {
    if (!st->go) return;
    const int32_t r = st->r;
    const int32_t nvec = (m + 2) / 2;
    const int64_t tiles = (int64_t)rowchunks * (n + 2);
    const double2 *F2 = reinterpret_cast<const double2 *>(F);
    const int32_t bar = st->bar;  // columns >= bar (the RHS among them) are no Step 1 candidates
    for (int64_t t0 = blockIdx.x; t0 < tiles; t0 += (int64_t)gridDim.x * U) {
        double2 x[U], f[U];
        double2 *addr[U];
        double Rt[U];
        int32_t v[U];
        bool live[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t t = t0 + (int64_t)u * gridDim.x;
            const int32_t g = (int32_t)(t / rowchunks), rc = (int32_t)(t % rowchunks);
            v[u] = rc * B + (int32_t)threadIdx.x;
            live[u] = t < tiles && v[u] < nvec;
            if (t < tiles) {
                Rt[u] = Rl[g];
                addr[u] = reinterpret_cast<double2 *>(T + (int64_t)cols[g] * ld) + v[u];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (live[u]) {
                x[u] = *addr[u];
                f[u] = F2[v[u]];
            }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!live[u]) continue;
            double2 y;
            y.x = (2 * v[u] == r) ? Rt[u] : fma(-f[u].x, Rt[u], x[u].x);
            y.y = (2 * v[u] + 1 == r) ? Rt[u] : fma(-f[u].y, Rt[u], x[u].y);
            *addr[u] = y;
            if (v[u] == 0) {  // row 0 of list position g: its Step 1 partial
                const int64_t t = t0 + (int64_t)u * gridDim.x;
                const int32_t g = (int32_t)(t / rowchunks);
                const int32_t j = cols[g];
                parts[g] = ArgMin{j < bar ? y.x : __builtin_inf(), j < bar ? j : kNoIndex};
            }
        }
    }
}

// Finalization: x (n), y (m) and the objective into out[0 .. n+m], in two
// launches of one thread per entry. First x = 0, y_i = the row-0 entry of
// slack column n+i-1 (0 when that column is basic: row 0 of every slack
// column is stored, also by a deferred build) and the objective, for the
// entries from `from` on (n when the caller has zeroed x); then x_j = the
// RHS entry of the row in which structural column j is basic.
// With `out` in host memory mapped into the device the host learns the end
// from the second launch instead of waiting for the stream: the first one
// stores the device's constant-rate clock at t_mark (non-NULL: the end of
// the solve's pivoting, which precedes it in the stream), and in the second
// the last workgroup to finish (counted on `ticket`, zero between launches)
// stores `seq` at seq_at after a system-scope fence (ticket NULL: no
// signal).
static __global__ __launch_bounds__(256) void k_extract_y(const double *__restrict__ T, int64_t ld, int32_t m,
                                                          int32_t n, double *__restrict__ out, int64_t from,
                                                          unsigned long long *t_mark) {
    if (t_mark && blockIdx.x == 0 && threadIdx.x == 0)
        __hip_atomic_store(t_mark, (unsigned long long)wall_clock64(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    const int64_t idx = from + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n)
        out[idx] = 0.0;
    else if (idx <= (int64_t)n + m)
        out[idx] = T[idx * ld];  // column idx: slack idx - n, or the RHS (the objective)
    if (t_mark) __threadfence_system();
}

static __global__ __launch_bounds__(256) void k_extract_x(const double *__restrict__ T, int64_t ld, int32_t m,
                                                          int32_t n, const int32_t *__restrict__ basis,
                                                          double *__restrict__ out, uint32_t *ticket,
                                                          uint32_t *seq_at, uint32_t seq) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (i <= m) {
        const int32_t bv = basis[i - 1];
        if (bv < n) out[bv] = T[((int64_t)n + m) * ld + i];
    }
    if (!ticket) return;
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0 && atomicAdd(ticket, 1u) == gridDim.x - 1) {
        *ticket = 0u;  // (the stream orders the next launch after this one)
        __threadfence_system();
        __hip_atomic_store(seq_at, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// Stores every basic column as the unit vector it is: the basic column of
// row i is e_i (rows 0 .. ld-1, padding zero). A column stored before holds
// exactly that already; one never stored (a slack column after a deferred
// build) gets its value.
static __global__ __launch_bounds__(256) void k_store_basic(double *__restrict__ T, int64_t ld, int32_t m,
                                                            const int32_t *__restrict__ basis) {
    const int64_t half = ld / 2;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)m * half) return;
    const int64_t r = idx / half + 1, v = idx % half;  // tableau row r, row pair v
    const int64_t col = basis[r - 1];
    double2 y;
    y.x = (2 * v == r) ? 1.0 : 0.0;
    y.y = (2 * v + 1 == r) ? 1.0 : 0.0;
    reinterpret_cast<double2 *>(T + col * ld)[v] = y;
}

// ---- general form (two-phase method) -------------------------------------
// Tableau of the general form, kernel sizes m = m_in + 1 rows (row m is the
// caller's objective, carried through Phase I) and n = n' = n_in + surplus
// columns. Row t (1..m_in) is the caller's row perm[t-1] times sgn[t-1], its
// surplus column surplus[t-1] (or -1) holds -1, and its identity column is
// n'+t-1; row m holds -c, then zeros, and its own identity column n'+m_in.
// Row 0 is left 0 here (k_phase1_row0 writes it). One thread per entry,
// column-major order.
static __global__ __launch_bounds__(256) void k_build_general(double *__restrict__ T, int64_t ld, int32_t m,
                                                              int32_t n, int32_t n_in, const double *__restrict__ A,
                                                              const double *__restrict__ b,
                                                              const double *__restrict__ c,
                                                              const int32_t *__restrict__ perm,
                                                              const double *__restrict__ sgn,
                                                              const int32_t *__restrict__ surplus) {
    const int64_t W = (int64_t)n + m + 1;
    const int64_t total = ld * W;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = idx / ld;
        const int32_t i = (int32_t)(idx - j * ld);
        double v = 0.0;
        if (i >= 1 && i < m) {  // a constraint row
            const int32_t k = perm[i - 1];
            const bool neg = sgn[i - 1] != 1.0;
            if (j < n_in) {
                const double a = A[(int64_t)k * n_in + j];
                v = neg ? -a : a;
            } else if (j < n) {
                v = surplus[i - 1] == j ? -1.0 : 0.0;
            } else if (j < W - 1) {
                v = j == (int64_t)n + i - 1 ? 1.0 : 0.0;
            } else {
                v = neg ? -b[k] : b[k];
            }
        } else if (i == m) {  // the carried objective row
            if (j < n_in)
                v = -c[j];
            else if (j == (int64_t)n + m - 1)
                v = 1.0;
        }
        T[idx] = v;
    }
}

// Row 0 of Phase I, one thread per column: 1 under each artificial column
// [art_c0, art_c1), 0 elsewhere, minus the artificial rows [art_r0, art_r1)
// one by one in row order.
static __global__ __launch_bounds__(256) void k_phase1_row0(double *__restrict__ T, int64_t ld, int64_t W,
                                                            int32_t art_r0, int32_t art_r1, int32_t art_c0,
                                                            int32_t art_c1) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= W) return;
    const double *col = T + j * ld;
    double v = (j >= art_c0 && j < art_c1) ? 1.0 : 0.0;
    for (int32_t t = art_r0; t < art_r1; ++t) v = v - col[t];
    T[j * ld] = v;
}

// Swaps rows r1 and r2 over all W columns (Phase II takes the carried
// objective as row 0).
static __global__ __launch_bounds__(256) void k_swap_rows(double *__restrict__ T, int64_t ld, int64_t W, int32_t r1,
                                                          int32_t r2) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= W) return;
    double *col = T + j * ld;
    const double a = col[r1];
    col[r1] = col[r2];
    col[r2] = a;
}

// The lowest column j < limit with |T[row][j]| > eps (or -1), one workgroup:
// the column of an artificial variable's drive-out.
static __global__ __launch_bounds__(256) void k_find_driveout(const double *__restrict__ T, int64_t ld, int32_t row,
                                                              int32_t limit, double eps, int32_t *__restrict__ out) {
    __shared__ int32_t s_min[4];
    int32_t best = kNoIndex;
    for (int32_t j = threadIdx.x; j < limit; j += blockDim.x)
        if (fabs(T[(int64_t)j * ld + row]) > eps) {
            best = j;
            break;  // later j of this thread are larger
        }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) best = min(best, __shfl_xor(best, off, 64));
    if ((threadIdx.x & 63) == 0) s_min[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t b0 = s_min[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) b0 = min(b0, s_min[w]);
        *out = b0 == kNoIndex ? -1 : b0;
    }
}

// Solver-state edits of the general form's host loop.
static __global__ void k_set_force(DevState *st, int32_t r, int32_t q) {
    st->force_r = r;
    st->force_q = q;
    st->status = LP_RUNNING;
}
static __global__ void k_set_status(DevState *st, int32_t status) { st->status = status; }
// Sets the columns and rows barred from now on and rescans row 0 at the next
// select (the start of a phase).
static __global__ void k_set_bar(DevState *st, int32_t bar) {
    st->bar = bar;
    st->fresh = 1;
    st->degen = 0;  // the anti-cycling count restarts with each phase
    st->status = LP_RUNNING;
}

}  // namespace lpgpu
