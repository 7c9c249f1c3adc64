// Internal definitions shared by the lpgpu kernels and host code.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "lpgpu.h"

namespace lpgpu {

// Rows of the column-major tableau are padded to a multiple of 16 doubles so
// that every column starts on a 128-byte line.
constexpr int kRowAlign = 16;

inline int64_t padded_ld(int32_t m) { return ((int64_t)m + 1 + kRowAlign - 1) / kRowAlign * kRowAlign; }

// Per-LP solver state, resident in device memory. The kernels read and write
// it; the host only reads it back between graph replays.
struct DevState {
    int32_t status;      // LP_RUNNING until Step 1 or 2 ends the solve
    int32_t go;          // 1: the update kernel applies pivot (r, q, p) now
    int32_t r, q;        // pivot row in [1, m], pivot column in [0, n+m)
    double p;            // T[r][q]
    int64_t pivots;      // pivots decided (and applied once the update ran)
    int64_t stop_at;     // pause (status stays RUNNING) when pivots reaches this
    int64_t max_pivots;  // iteration cap
    int64_t log_cap;     // entries in the pivot log
    double eps_d, eps_p;
    int32_t fresh;       // 1: no pricing partials yet, scan row 0 instead
    int32_t nparts;      // number of pricing partials written by the update kernel
    int32_t leave;       // column leaving the basis at the current pivot
    int32_t pq;          // position of the entering column in the rewrite list
    // General form (two-phase method; the one-pivot kernels only): columns
    // >= bar never enter, and rows whose basic column is >= bar never leave.
    // n + m (no effect) for the standard form.
    int32_t bar;
    // >= 0: the next select takes pivot (force_r, force_q) without Steps 1-2
    // (the drive-out of an artificial variable after Phase I), then clears it.
    int32_t force_r, force_q;
    // Anti-cycling fallback (the one-pivot kernels only): with bland_after =
    // k > 0, Bland's rule decides while the last k or more pivots were all
    // degenerate (a ratio <= eps_p); degen counts them.
    int32_t bland_after;
    int32_t degen;
    int32_t pad_;
};

// (value, index) pair of the two-stage argmin.
struct ArgMin {
    double v;
    int32_t i;
};

// Lexicographic order: smaller value first, then the lower index. A NaN wins
// over every number so that it reaches the final stage, which reports it.
// (Written with bitwise operators and one select, so that it compiles to
// compares and mask logic without branches.)
__device__ __forceinline__ bool lex_less(double av, int32_t ai, double bv, int32_t bi) {
    const bool an = av != av, bn = bv != bv, ilt = ai < bi;
    const bool lt = (av < bv) | ((av == bv) & ilt);
    const bool nl = an & (!bn | ilt);
    return (an | bn) ? nl : lt;
}

// Non-finite values (the paper does not discuss them; the reading shared with
// the CPU reference): Step 1 stops with LP_NUMERICAL when its minimum over
// row 0 is a NaN (a NaN wins every argmin, so the minimum is NaN iff row 0
// holds one) or -inf; Step 2 stops with LP_NUMERICAL when, in some row 1..m,
// the entering column's entry is not finite or the RHS entry is a NaN. A
// ratio is then never a NaN (finite over finite, or +-inf over finite), and
// the pivot column F is finite, so every basic column's normalised pivot-row
// entry is exactly +-0 and skipping basic columns in Step 3 changes no value.
__device__ __forceinline__ bool step1_bad(double v) { return v != v || v == -__builtin_inf(); }
__device__ __forceinline__ bool step2_bad(double a, double rhs) {
    return !__builtin_isfinite(a) || rhs != rhs;
}

// An empty slot: +inf with the largest index loses to every real candidate.
constexpr int32_t kNoIndex = 0x7fffffff;

// Cross-lane exchanges of a wave (every lane active): DPP within rows of 16
// lanes, and the gfx950 lane swaps across rows (v_permlane16_swap,
// v_permlane32_swap: VALU exchanges, no LDS round trip).
template <int CTRL>
__device__ __forceinline__ int32_t dpp_i32(int32_t x) {
    return __builtin_amdgcn_update_dpp(x, x, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
    return __hiloint2double(dpp_i32<CTRL>(__double2hiint(x)), dpp_i32<CTRL>(__double2loint(x)));
}

// x of lane l ^ 16 (W = 16) or l ^ 32 (W = 32): the swap of a register with
// itself leaves, in the first result, rows 0 and 2 (lanes 0-31 for W = 32)
// in their place and their copies in rows 1 and 3 (lanes 32-63), and in the
// second result rows 1 and 3 (lanes 32-63) with their copies in rows 0 and 2
// (lanes 0-31).
template <int W>
__device__ __forceinline__ int32_t swap_i32(int32_t x) {
    const bool hi = (threadIdx.x & W) != 0;
    if constexpr (W == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
        return hi ? r[0] : r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
        return hi ? r[0] : r[1];
    }
}

template <int W>
__device__ __forceinline__ double swap_f64(double x) {
    return __hiloint2double(swap_i32<W>(__double2hiint(x)), swap_i32<W>(__double2loint(x)));
}

// Keeps the smaller of (v, i) and (ov, oi) under lex_less.
__device__ __forceinline__ void argmin_take(double &v, int32_t &i, double ov, int32_t oi) {
    const bool take = lex_less(ov, oi, v, i);
    v = take ? ov : v;
    i = take ? oi : i;
}

// Wave argmin of (v, i); every lane gets the winner. Within a row of 16
// lanes: the quad permutations [1,0,3,2] and [2,3,0,1], the half-row mirror
// and the row mirror; then rows 0 <-> 1, 2 <-> 3 and lanes 0-31 <-> 32-63.
// The argmin is unique under lex_less, so the order of the steps does not
// change the result. Call with every lane of the wave active.
__device__ __forceinline__ void wave_argmin(double &v, int32_t &i) {
    argmin_take(v, i, dpp_f64<0xB1>(v), dpp_i32<0xB1>(i));
    argmin_take(v, i, dpp_f64<0x4E>(v), dpp_i32<0x4E>(i));
    argmin_take(v, i, dpp_f64<0x141>(v), dpp_i32<0x141>(i));
    argmin_take(v, i, dpp_f64<0x140>(v), dpp_i32<0x140>(i));
    argmin_take(v, i, swap_f64<16>(v), swap_i32<16>(i));
    argmin_take(v, i, swap_f64<32>(v), swap_i32<32>(i));
}

// Sum of x over a wave (every lane active); every lane gets it.
__device__ __forceinline__ int32_t wave_sum_i32(int32_t x) {
    x += dpp_i32<0xB1>(x);
    x += dpp_i32<0x4E>(x);
    x += dpp_i32<0x141>(x);
    x += dpp_i32<0x140>(x);
    x += swap_i32<16>(x);
    x += swap_i32<32>(x);
    return x;
}

// Block-wide lexicographic argmin; every thread gets the result. `sv`/`si`
// are LDS scratch of at least blockDim.x / 64 entries.
__device__ __forceinline__ void block_argmin(double &v, int32_t &i, double *sv, int32_t *si) {
    wave_argmin(v, i);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
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

// The options of a call with its tuning record resolved (a NULL lp_options
// or a NULL tuning pointer gives the defaults).
struct Options : lp_tuning {
    double eps_dual, eps_pivot;
    int64_t max_pivots;
    int32_t record_pivots;
    void *stream;
    void *device_buffer;
    size_t device_buffer_bytes;
    int32_t device;
    int32_t bland_after;
};
Options resolve_options(const lp_options *opt);

// Thread-local last error text and a setter returning the code.
int set_error(int code, const std::string &msg);

#define LP_HIP_CHECK(expr)                                                                    \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return ::lpgpu::set_error(LP_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

}  // namespace lpgpu
