// Launchers of the pivot-fusion kernels (instances live in fused_launch.hip,
// compiled on their own).
#pragma once

#include <hip/hip_runtime.h>

#include "fused_kernels.hpp"

namespace lpgpu {

// Device buffers and sizes shared by the kernels of one group.
struct FusedArgs {
    double *T;
    int64_t ld;
    int32_t m, n, K;
    int32_t rowchunks;  // update tiles: row chunks
    int32_t nsparts;    // staging workgroups (= Step 1 partials of the staging kernel)
    int32_t nparts;     // update slot groups (= Step 1 partials of the update kernel)
    DevState *st;
    GroupState *gs;
    double *Fk;   // K columns of ld doubles
    double *Rk;   // K rows of n + 1 + K doubles
    double *D;    // n + 1 + K doubles
    int32_t *cols, *pos, *basis, *log_r, *log_q;
    ArgMin *parts, *sparts;
    unsigned long long *cols_done;
};

// True when an update kernel instance exists for this tile shape and group size.
bool fused_update_supported(int block, int cols, int rv, int K);

// Steps 1-2 (select) and the Step 3 inputs (stage) of pivot j of a group.
void launch_fused_select(const FusedArgs &a, int j, hipStream_t s);
void launch_fused_stage(const FusedArgs &a, int j, hipStream_t s);

// The group's update pass; with events, timed by the dispatch.
void launch_fused_update(const FusedArgs &a, int block, int cols, int rv, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1);

}  // namespace lpgpu
