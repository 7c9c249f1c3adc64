// A reusable single-LP solver bound to one stream, for the server's lane of
// large LPs: the tableau is built and resident already; each solve brings it
// and a work block (carved like a context's buffers), so nothing is allocated
// per LP. Host resources (events, pinned memory) are made once, for LPs up to
// max_m x max_n.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "common.hpp"

namespace lpgpu {

struct Lane;

struct LaneResult {
    int32_t status = LP_RUNNING;
    int64_t pivots = 0;
    double objective = 0.0;
    std::vector<double> x, y;
    std::vector<int32_t> rows, cols;
};

// opt: the server's options (tolerances, cap, pivot log); the lane runs
// pivot fusion with the per-pivot decision kernels (no grid barrier, so no
// co-residency need beside other kernels), plain launches.
int lane_create(Lane **out, int device, hipStream_t stream, const Options &opt, int32_t max_m, int32_t max_n);
// Bytes of the work block an m x n LP needs (0 if the lane cannot take it).
size_t lane_work_bytes(const Lane *L, int32_t m, int32_t n);
// Entries of the pivot log the lane keeps for an m x n LP.
int64_t lane_log_cap(const Lane *L, int32_t m, int32_t n);
// Solves the LP whose Table I tableau is built in T (ld = padded_ld(m)),
// using `work` (lane_work_bytes) for every other buffer; blocks until done.
int lane_solve(Lane *L, int32_t m, int32_t n, double *T, unsigned char *work, LaneResult *out);
void lane_destroy(Lane *L);

}  // namespace lpgpu
