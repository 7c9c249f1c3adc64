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
constexpr int kMaxColsPerBlock = 64;

// Initialization Step, structural part: column j < n of T gets -c_j in row 0
// and column j of A in rows 1..m (Table I); padding rows are zero. A is
// row-major, so each 64x64 tile is transposed through LDS.
__global__ __launch_bounds__(256) void k_build_struct(double *__restrict__ T, int64_t ld, int32_t m, int32_t n,
                                                      const double *__restrict__ A, const double *__restrict__ c) {
    __shared__ double tile[kBuildTile][kBuildTile + 1];
    const int64_t j0 = (int64_t)blockIdx.x * kBuildTile;
    const int64_t i0 = (int64_t)blockIdx.y * kBuildTile;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll 4
    for (int k = 0; k < kBuildTile / 4; ++k) {
        const int64_t i = i0 + ty + 4 * k, j = j0 + tx;
        double v = 0.0;
        if (j < n) {
            if (i == 0)
                v = -c[j];
            else if (i <= m)
                v = A[(i - 1) * n + j];
        }
        tile[ty + 4 * k][tx] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < kBuildTile / 4; ++k) {
        const int64_t j = j0 + ty + 4 * k, i = i0 + tx;
        if (j < n && i < ld) T[j * ld + i] = tile[tx][ty + 4 * k];
    }
}

// Initialization Step, slack identity and right-hand side (columns n..W-1).
__global__ __launch_bounds__(256) void k_build_slack(double *__restrict__ T, int64_t ld, int32_t m, int32_t n,
                                                     const double *__restrict__ b) {
    const int64_t half = ld / 2;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)(m + 1) * half) return;
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

// Solver state, slack basis and a zeroed pivot-column buffer.
__global__ void k_init(DevState *st, DevState init, int32_t *__restrict__ basis, int32_t m, int32_t n,
                       double *__restrict__ F, int64_t ld) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx == 0) *st = init;
    if (idx < m) basis[idx] = n + (int32_t)idx;
    if (idx < ld) F[idx] = 0.0;
}

__global__ void k_set_stop(DevState *st, int64_t stop_at) { st->stop_at = stop_at; }

// Steps 1 and 2 for the next pivot; one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_select(const double *__restrict__ T, int64_t ld, int32_t m, int32_t n,
                                                const ArgMin *__restrict__ parts, DevState *__restrict__ st,
                                                double *__restrict__ F, int32_t *__restrict__ basis,
                                                int32_t *__restrict__ log_r, int32_t *__restrict__ log_q) {
    __shared__ double sv[16];
    __shared__ int32_t si[16];
    const int tid = threadIdx.x, nt = blockDim.x;
    const DevState s = *st;
    if (s.status != LP_RUNNING || s.pivots >= s.stop_at) {
        if (tid == 0) st->go = 0;
        return;
    }
    const int64_t W = (int64_t)n + m + 1;

    // Step 1: most negative objective-row entry, lowest column on ties.
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
    if (v != v || v >= -s.eps_d) {
        if (tid == 0) {
            st->status = (v != v) ? LP_NUMERICAL : LP_OPTIMAL;
            st->go = 0;
        }
        return;
    }

    // Step 2: minimum ratio over rows with T[i][q] > eps_p, lowest row on ties.
    const double *colq = T + (int64_t)q * ld;
    const double *rhs = T + (W - 1) * ld;
    double rv = __builtin_inf();
    int32_t r = kNoIndex;
    int bad = 0;
    for (int32_t i = 1 + tid; i <= m; i += nt) {
        const double a = colq[i], bb = rhs[i];
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
        if (tid == 0) {
            st->status = bad ? LP_NUMERICAL : (r == kNoIndex ? LP_UNBOUNDED : LP_ITER_LIMIT);
            st->go = 0;
        }
        return;
    }

    // Snapshot of the pivot column for the elimination.
    for (int32_t i = tid; i <= m; i += nt) F[i] = colq[i];
    if (tid == 0) {
        st->r = r;
        st->q = q;
        st->p = colq[r];
        basis[r - 1] = q;
        if (s.pivots < s.log_cap) {
            log_r[s.pivots] = r;
            log_q[s.pivots] = q;
        }
        st->pivots = s.pivots + 1;
        st->fresh = 0;
        st->go = 1;
    }
}

// Step 3 on a tile of whole columns, plus the first stage of the next Step 1.
// Thread t owns the row pairs {2v, 2v+1}, v = t + k*blockDim.x, k < VPT, and
// keeps their F values in registers across the tile's columns. VPT = 0 is
// the general form for any m, which re-reads F for every column. The launch
// must use exactly B threads.
template <int B, int VPT>
__global__ __launch_bounds__(B) void k_update(double *__restrict__ T, int64_t ld, int32_t m, int32_t n,
                                                 int32_t cols_per_block, const double *__restrict__ F,
                                                 const DevState *__restrict__ st, ArgMin *__restrict__ parts) {
    __shared__ double sR[kMaxColsPerBlock];
    if (!st->go) return;
    const int32_t r = st->r;
    const double p = st->p;
    const int64_t W = (int64_t)n + m + 1;
    const int64_t j0 = (int64_t)blockIdx.x * cols_per_block;
    const int jn = (int)min<int64_t>(cols_per_block, W - j0);
    const int tid = threadIdx.x;
    constexpr int nt = B;

    // Normalised pivot row for this tile (Step 3) and the tile's new row-0
    // entries, reduced to one (value, column) partial for the next Step 1.
    // Row 0 is never the pivot row, so its new entry is fma(-F_0, R_j, T_0j).
    if (tid < 64) {
        double val = __builtin_inf();
        int32_t idx = kNoIndex;
        if (tid < jn) {
            const int64_t j = j0 + tid;
            const double *col = T + j * ld;
            const double Rj = col[r] / p;
            const double t0 = col[0];
            sR[tid] = Rj;
            const double new0 = (Rj == 0.0) ? t0 : fma(-F[0], Rj, t0);
            if (j < (int64_t)n + m) {
                val = new0;
                idx = (int32_t)j;
            }
        }
        wave_argmin(val, idx);
        if (tid == 0) parts[blockIdx.x] = ArgMin{val, idx};
    }
    __syncthreads();

    const int nvec = (m + 2) / 2;  // double2 vectors covering rows 0..m
    const double2 *F2 = reinterpret_cast<const double2 *>(F);
    if constexpr (VPT > 0) {
        double2 f[VPT];
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            const int v = tid + k * nt;
            f[k] = v < nvec ? F2[v] : double2{0.0, 0.0};
        }
        for (int jj = 0; jj < jn; ++jj) {
            const double Rj = sR[jj];
            if (Rj == 0.0) continue;  // column unchanged up to the sign of zeros
            double2 *col = reinterpret_cast<double2 *>(T + (j0 + jj) * ld);
            double2 x[VPT];
#pragma unroll
            for (int k = 0; k < VPT; ++k) {
                const int v = tid + k * nt;
                if (v < nvec) x[k] = col[v];
            }
#pragma unroll
            for (int k = 0; k < VPT; ++k) {
                const int v = tid + k * nt;
                if (v < nvec) {
                    double2 y;
                    y.x = (2 * v == r) ? Rj : fma(-f[k].x, Rj, x[k].x);
                    y.y = (2 * v + 1 == r) ? Rj : fma(-f[k].y, Rj, x[k].y);
                    col[v] = y;
                }
            }
        }
    } else {
        for (int jj = 0; jj < jn; ++jj) {
            const double Rj = sR[jj];
            if (Rj == 0.0) continue;
            double2 *col = reinterpret_cast<double2 *>(T + (j0 + jj) * ld);
            for (int v = tid; v < nvec; v += nt) {
                const double2 f = F2[v];
                const double2 x = col[v];
                double2 y;
                y.x = (2 * v == r) ? Rj : fma(-f.x, Rj, x.x);
                y.y = (2 * v + 1 == r) ? Rj : fma(-f.y, Rj, x.y);
                col[v] = y;
            }
        }
    }
}

// Finalization: x (n), y (m) and the objective into out[0 .. n+m].
__global__ __launch_bounds__(1024) void k_extract(const double *__restrict__ T, int64_t ld, int32_t m, int32_t n,
                                                 const int32_t *__restrict__ basis, double *__restrict__ out) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int64_t W = (int64_t)n + m + 1;
    for (int32_t j = tid; j < n; j += nt) out[j] = 0.0;
    __syncthreads();
    for (int32_t i = 1 + tid; i <= m; i += nt) {
        const int32_t bv = basis[i - 1];
        if (bv < n) out[bv] = T[(W - 1) * ld + i];
        out[n + i - 1] = T[((int64_t)n + i - 1) * ld];
    }
    if (tid == 0) out[n + m] = T[(W - 1) * ld];
}

}  // namespace lpgpu
