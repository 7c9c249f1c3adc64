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
// group changes (their pivot-row entry is 0), so they are left out. A
// column's slot t indexes R_k[t] (the normalised pivot-row entry of pivot k)
// and D[t] (its row-0 entry after the pivots staged so far).
//
// Launches per group, on one stream:
//   k_gselect(j), k_gstage(j)   for j = 0 .. K-1
//   k_gupdate                   applies the kdone pivots the group decided.
// k_gselect(0) first closes the previous group: the columns that entered and
// stay basic give up their slots to the appended columns that stay nonbasic.
#pragma once

#include "common.hpp"

namespace lpgpu {

constexpr int kMaxFuse = 8;

// Decisions of the current group, resident in device memory.
struct GroupState {
    int32_t kdone;  // pivots decided in this group
    int32_t napp;   // leaving columns appended to the list (slots n+1 ..)
    int32_t r[kMaxFuse];
    int32_t q[kMaxFuse];
    int32_t l[kMaxFuse];  // leaving column of pivot k
    double p[kMaxFuse];
};

// State, slack basis, list and zeroed pivot-column buffers for a new solve.
static __global__ void k_ginit(DevState *st, DevState init, GroupState *gs, int32_t *__restrict__ basis, int32_t m,
                               int32_t n, int32_t K, double *__restrict__ Fk, int64_t ld, int32_t *__restrict__ cols,
                               int32_t *__restrict__ pos, unsigned long long *__restrict__ cols_done) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t Lg = (int64_t)n + 1 + K;
    if (idx == 0) {
        *st = init;
        gs->kdone = 0;
        gs->napp = 0;
        *cols_done = 0;
    }
    if (idx < m) basis[idx] = n + (int32_t)idx;
    if (idx < (int64_t)K * ld) Fk[idx] = 0.0;
    if (idx < Lg) cols[idx] = idx < n ? (int32_t)idx : (idx == n ? n + m : -1);
    if (idx < (int64_t)n + m) pos[idx] = idx < n ? (int32_t)idx : -1;
}

// Closes the finished group (one thread). Entered columns that are still
// basic give their slots below n to the appended columns that are nonbasic
// at the end; the two counts are equal, since the group started with n
// nonbasic columns in slots 0..n-1 and ends with n nonbasic columns, each of
// which is either one that stayed in its slot or an appended one. The
// group's columns are held in registers (fully unrolled loops, no local
// arrays indexed at run time).
static __device__ void close_group(GroupState *gs, int32_t *__restrict__ cols, int32_t *__restrict__ pos, int32_t n) {
    const int kd = gs->kdone;
    if (kd == 0) return;
    const int na = gs->napp;
    int32_t qk[kMaxFuse], lk[kMaxFuse];
#pragma unroll
    for (int k = 0; k < kMaxFuse; ++k) {
        qk[k] = k < kd ? gs->q[k] : -1;
        lk[k] = k < kd ? gs->l[k] : -1;
    }
    // the last event of the group decides: entered -> basic, left -> nonbasic
    auto basic_at_end = [&](int32_t c) {
        bool b = false;
#pragma unroll
        for (int k = 0; k < kMaxFuse; ++k) {
            if (qk[k] == c) b = true;
            if (lk[k] == c) b = false;
        }
        return b;
    };
    int next = 0;  // entered columns before `next` have been examined
    for (int32_t s = n + 1; s < n + 1 + na; ++s) {
        const int32_t c = cols[s];
        if (basic_at_end(c)) {
            pos[c] = -1;  // left and entered again within the group
        } else {
            // the next entered column that is still basic and holds a slot below n
            int32_t t = -1;
#pragma unroll
            for (int k = 0; k < kMaxFuse; ++k) {
                if (t < 0 && k >= next && k < kd) {
                    const int32_t e = qk[k];
                    const int32_t te = pos[e];
                    if (te >= 0 && te < n && basic_at_end(e)) {
                        pos[e] = -1;
                        t = te;
                        next = k + 1;
                    }
                }
            }
            if (t >= 0) {
                cols[t] = c;
                pos[c] = t;
            }
        }
        cols[s] = -1;
    }
    gs->kdone = 0;
    gs->napp = 0;
}

// Steps 1 and 2 of pivot J of the group; one workgroup of 1024 threads.
//   Step 1  J = 0: final stage of the argmin over the update's partials (a
//           scan of row 0 before the first pivot); J > 0: over the staging
//           kernel's partials of row 0 after pivot J-1;
//   Step 2  column q and the RHS column after the J earlier pivots, rebuilt
//           from the tableau by the chain above; column q is kept as F_J.
// The decision (r, q, p, leaving column), the basis, the log and, if the
// leaving column is not in the list yet, its appended slot. J is a template
// argument so that the chain's coefficients load without a wait per pivot.
template <int J>
__global__ __launch_bounds__(1024) void k_gselect(const double *__restrict__ T, int64_t ld, int32_t m, int32_t n,
                                                  int32_t K, const ArgMin *__restrict__ parts,
                                                  const ArgMin *__restrict__ sparts, int32_t nsparts,
                                                  DevState *__restrict__ st, GroupState *__restrict__ gs,
                                                  double *__restrict__ Fk, double *__restrict__ Rk,
                                                  double *__restrict__ D, int32_t *__restrict__ cols,
                                                  int32_t *__restrict__ pos, int32_t *__restrict__ basis,
                                                  int32_t *__restrict__ log_r, int32_t *__restrict__ log_q) {
    __shared__ double sv[16];
    __shared__ int32_t si[16];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int64_t Lg = (int64_t)n + 1 + K;
    if constexpr (J == 0) {
        if (tid == 0) close_group(gs, cols, pos, n);
        // appended slots start with R = 0 and a row-0 entry of 0: the exact
        // values for a column that is basic (a unit vector) before it leaves
        if (tid < K * K) Rk[(int64_t)(tid / K) * Lg + n + 1 + tid % K] = 0.0;
        if (tid < K) D[n + 1 + tid] = 0.0;
        __syncthreads();
    }
    const DevState s = *st;
    if (s.status != LP_RUNNING || s.pivots >= s.stop_at) return;
    if (J > 0 && gs->kdone != J) return;  // the group ended early
    const int64_t W = (int64_t)n + m + 1;

    // Step 1
    double v = __builtin_inf();
    int32_t q = kNoIndex;
    if (J == 0 && s.fresh) {
        for (int32_t c = tid; c < n + m; c += nt) {
            const double t = T[(int64_t)c * ld];
            if (lex_less(t, c, v, q)) {
                v = t;
                q = c;
            }
        }
    } else {
        const ArgMin *pp = J == 0 ? parts : sparts;
        const int32_t np = J == 0 ? s.nparts : nsparts;
        for (int32_t k = tid; k < np; k += nt) {
            const ArgMin a = pp[k];
            if (lex_less(a.v, a.i, v, q)) {
                v = a.v;
                q = a.i;
            }
        }
    }
    block_argmin(v, q, sv, si);
    if (v != v || v >= -s.eps_d) {
        if (tid == 0) st->status = (v != v) ? LP_NUMERICAL : LP_OPTIMAL;
        return;
    }

    // Step 2 on column q and the RHS after the J earlier pivots. Every
    // nonbasic column has a slot; a missing one would be a broken list, which
    // ends the solve instead of reading outside R.
    const int32_t tq = pos[q];
    if (tq < 0) {
        if (tid == 0) st->status = LP_NUMERICAL;
        return;
    }
    int32_t rk[J > 0 ? J : 1];
    double Rq[J > 0 ? J : 1], Rb[J > 0 ? J : 1];
#pragma unroll
    for (int k = 0; k < J; ++k) {
        rk[k] = gs->r[k];
        Rq[k] = Rk[(int64_t)k * Lg + tq];
        Rb[k] = Rk[(int64_t)k * Lg + n];
    }
    const double *colq = T + (int64_t)q * ld;
    const double *rhs = T + (W - 1) * ld;
    double *Fj = Fk + (int64_t)J * ld;
    double rv = __builtin_inf();
    int32_t r = kNoIndex;
    int bad = 0;
    for (int32_t i = tid; i <= m; i += nt) {
        double a = colq[i], bb = rhs[i];
        double f[J > 0 ? J : 1];
#pragma unroll
        for (int k = 0; k < J; ++k) f[k] = Fk[(int64_t)k * ld + i];
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
        if (a != a || bb != bb) {
            bad = 1;
        } else if (a > s.eps_p) {
            const double ratio = bb / a;
            if (ratio != ratio)
                bad = 1;
            else if (lex_less(ratio, i, rv, r)) {
                rv = ratio;
                r = i;
            }
        }
    }
    bad = __syncthreads_or(bad);
    block_argmin(rv, r, sv, si);
    if (bad || r == kNoIndex || s.pivots >= s.max_pivots) {
        if (tid == 0) st->status = bad ? LP_NUMERICAL : (r == kNoIndex ? LP_UNBOUNDED : LP_ITER_LIMIT);
        return;
    }
    if (tid != 0) return;
    // p = entry r of column q after the J earlier pivots, by the same chain
    double p = colq[r];
#pragma unroll
    for (int k = 0; k < J; ++k) p = (r == rk[k]) ? Rq[k] : fma(-Fk[(int64_t)k * ld + r], Rq[k], p);
    const int32_t leave = basis[r - 1];
    const int32_t na = gs->napp;
    gs->r[J] = r;
    gs->q[J] = q;
    gs->l[J] = leave;
    gs->p[J] = p;
    if (pos[leave] < 0) {
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
// (D, column) pairs to one Step 1 partial for pivot J+1.
template <int J>
__global__ __launch_bounds__(256) void k_gstage(const double *__restrict__ T, int64_t ld, int32_t m, int32_t n,
                                                int32_t K, const GroupState *__restrict__ gs,
                                                const double *__restrict__ Fk, double *__restrict__ Rk,
                                                double *__restrict__ D, const int32_t *__restrict__ cols,
                                                ArgMin *__restrict__ sparts) {
    __shared__ double sv[4];
    __shared__ int32_t si[4];
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
    int32_t idx = kNoIndex;
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
            }
        }
    }
    block_argmin(v, idx, sv, si);
    if (threadIdx.x == 0) sparts[blockIdx.x] = ArgMin{v, idx};
}

// Step 3 for the whole group in one pass over (row chunk, slot group) tiles:
// every listed column is read once, has the group's pivots applied in order,
// and is written once. A row chunk is B row pairs (one double2 per thread);
// a slot group is C consecutive list slots. The row-chunk-0 workgroup of each
// slot group reduces its new row-0 entries to one Step 1 partial and counts
// the columns the group changed (some R_k nonzero).
//
// KF is the group size of the context. Full slot groups take a straight-line
// path: the pivot-column loads, then the tile's columns, one wait, the chain,
// and stores predicated on the row range (threads past the last row pair load
// row pair 0 and store nothing), so the last row chunk needs no separate
// code. A group cut short (the solve ended, or a pivot budget ran out) has
// kd < KF pivots; the missing ones are applied as exact identities, with
// R = 0, F = 0 and no pivot row: fma(-0, 0, x) returns x for every x,
// signed zeros, infinities and NaN included. The last, partial slot group
// takes a plain loop.
template <int B, int C, int KF>
__global__ __launch_bounds__(B) void k_gupdate(double *__restrict__ T, int64_t ld, int32_t m, int32_t n,
                                               int32_t rowchunks, const int32_t *__restrict__ cols,
                                               const double *__restrict__ Rk, const double *__restrict__ Fk,
                                               const GroupState *__restrict__ gs, ArgMin *__restrict__ parts,
                                               unsigned long long *__restrict__ cols_done) {
    const int kd = gs->kdone;
    if (kd == 0) return;
    const int32_t Lv = n + 1 + gs->napp;
    const int64_t Lg = (int64_t)n + 1 + KF;
    const int32_t rc = (int32_t)(blockIdx.x % (uint32_t)rowchunks);
    const int32_t g = (int32_t)(blockIdx.x / (uint32_t)rowchunks);
    const int32_t c0 = g * C;
    const bool row0 = rc == 0 && threadIdx.x == 0;  // holds row 0, never a pivot row
    if (c0 >= Lv) {
        if (row0) parts[g] = ArgMin{__builtin_inf(), kNoIndex};
        return;
    }
    const int32_t nvec = (m + 2) / 2;
    const int32_t v = rc * B + (int32_t)threadIdx.x;
    const bool live = v < nvec;
    const int32_t vs = live ? v : 0;
    const int32_t i0 = 2 * v;
    const int64_t ldv = ld / 2;
    const double2 *F2 = reinterpret_cast<const double2 *>(Fk);

    if (c0 + C <= Lv) {
        int32_t rk[KF];
        double2 f[KF];
#pragma unroll
        for (int k = 0; k < KF; ++k) {
            const bool on = k < kd;
            rk[k] = on ? gs->r[k] : -1;
            f[k] = F2[k * ldv + vs];
            if (!on) f[k] = double2{0.0, 0.0};
        }
        double2 *p[C];
        double Rj[C][KF];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            p[c] = reinterpret_cast<double2 *>(T + (int64_t)cols[c0 + c] * ld) + vs;
#pragma unroll
            for (int k = 0; k < KF; ++k) Rj[c][k] = k < kd ? Rk[(int64_t)k * Lg + c0 + c] : 0.0;
        }
        double2 x[C];
#pragma unroll
        for (int c = 0; c < C; ++c) x[c] = *p[c];
#pragma unroll
        for (int k = 0; k < KF; ++k)
#pragma unroll
            for (int c = 0; c < C; ++c) {
                x[c].x = (i0 == rk[k]) ? Rj[c][k] : fma(-f[k].x, Rj[c][k], x[c].x);
                x[c].y = (i0 + 1 == rk[k]) ? Rj[c][k] : fma(-f[k].y, Rj[c][k], x[c].y);
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
                if (jc != n + m && lex_less(x[c].x, jc, val, idx)) {
                    val = x[c].x;
                    idx = jc;
                }
                bool nz = false;
#pragma unroll
                for (int k = 0; k < KF; ++k) nz |= Rj[c][k] != 0.0;
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
        double2 *cp = reinterpret_cast<double2 *>(T + (int64_t)jc * ld) + vs;
        double2 x = *cp;
        bool nz = false;
#pragma unroll 1
        for (int k = 0; k < kd; ++k) {
            const double R = Rk[(int64_t)k * Lg + c0 + c];
            const double2 ff = F2[k * ldv + vs];
            const int32_t r = gs->r[k];
            nz |= R != 0.0;
            x.x = (i0 == r) ? R : fma(-ff.x, R, x.x);
            x.y = (i0 + 1 == r) ? R : fma(-ff.y, R, x.y);
        }
        if (live) *cp = x;
        changed += nz;
        if (row0 && jc != n + m && lex_less(x.x, jc, val, idx)) {
            val = x.x;
            idx = jc;
        }
    }
    if (row0) {
        parts[g] = ArgMin{val, idx};
        if (changed) atomicAdd(cols_done, changed);
    }
}

}  // namespace lpgpu
