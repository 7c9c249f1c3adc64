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
    int32_t KF;         // pivots per update pass of the update instance (>= K; the surplus are identities)
    int32_t rowchunks;  // update tiles: row chunks of one row per thread
    int32_t nsparts;    // staging workgroups (= Step 1 partials of the staging kernel)
    int32_t nparts;     // update slot groups (= Step 1 partials of the update kernel)
    DevState *st;
    GroupState *gs;
    double *Fk;   // K columns of ld doubles
    double *Rk;   // K rows of n + 1 + K doubles
    double *D;    // n + 1 + K doubles
    int32_t *cols, *pos, *basis, *log_r, *log_q;
    ArgMin *parts;
    SPart *sparts;
    unsigned long long *cols_done;  // [0] columns changed by all passes; the first pass after a deferred
                                    // build: [1] its changed columns, [2] its pivots, [3] its appended
                                    // columns
    int32_t select_wgs;  // workgroups of the select kernel (at most kMaxSelectWgs)
    GRatio *rparts;      // their Step 2 partials
    uint32_t *ticket;    // their arrival counter, zero between launches
    int32_t decide_wgs;  // > 0: workgroups of the one-launch decision kernel
    int32_t decide_block;  // its threads per workgroup (256 or 512)
    GridSync *gsync;     // its barrier counters, zero between launches
    uint32_t decide_spin;
    uint32_t gate_spin;  // polls before its check-in gate closes
    double *dump;       // a zero column the pure update pass writes for slots past the list
    double *PV;         // the group's pivot rows after the group, K rows of n + 1 + K doubles
    // The one-launch decision kernel's last workgroup copies the solver state
    // and the work counters (pub_words 8-byte words from st) to `pub`, host
    // memory mapped into the device, then stores pub_seq at pub_seq_at
    // (NULL pub: no copy).
    unsigned char *pub;
    uint32_t pub_seq;
    int32_t pub_words;
    uint32_t *pub_seq_at;
    // non-NULL: the decision kernel stores the device's constant-rate clock
    // there when it starts (the start of a solve, in host memory mapped into
    // the device)
    unsigned long long *t_mark;
};

// Update instances exist for groups of up to 2, 4, 8, 12, 16, 24, 32 and
// 48 pivots (above 16 with the one-launch decision kernel only).
inline int32_t fused_update_kf(int32_t K) {
    return K <= 2 ? 2 : K <= 4 ? 4 : K <= 8 ? 8 : K <= 12 ? 12 : K <= 16 ? 16 : K <= 24 ? 24 : K <= 32 ? 32 : 48;
}

// The one-launch decision kernel: G workgroups of `block` threads, one row
// and one list slot per thread; used when G <= kMaxDecideWgs.
constexpr int kMaxDecideWgs = 128;
inline int32_t decide_workgroups_for(int32_t m, int64_t Lg, int32_t block) {
    const int64_t rows = (int64_t)m + 1;
    const int64_t span = rows > Lg ? rows : Lg;
    return (int32_t)((span + block - 1) / block);
}
constexpr uint32_t kDefaultDecideSpin = 1u << 22;

// Select workgroups: enough for about one Step 2 row per thread.
constexpr int kMaxSelectWgs = 64;
inline int32_t select_workgroups_for(int32_t m) {
    const int32_t g = (m + 1 + 255) / 256;
    return g < 1 ? 1 : (g > kMaxSelectWgs ? kMaxSelectWgs : g);
}

// True when an update kernel instance exists for this tile shape and group
// size, with the one-launch decision kernel (the pure pass) or without.
bool fused_update_supported(int block, int cols, int rv, int K, bool one_launch);

// Workgroups of the one-launch decision kernel (threads `block`, group size
// instance KF) that one compute unit holds at once, the smaller of its two
// forms (reading the tableau, or A and c after a deferred build); 0 if the
// instance does not exist. Its grid barriers need all G workgroups resident,
// so the kernel is used only while G <= this figure times the compute units.
int decide_blocks_per_cu(int block, int KF);

// All decisions of a group in one launch (a.decide_wgs > 0).
void launch_fused_decide(const FusedArgs &a, hipStream_t s);

// The first group after a deferred build: its decisions read the structural
// columns from A (row-major m x n) and c, and its update pass writes them
// (the Initialization Step of those columns fused with the group's Step 3).
void launch_first_decide(const FusedArgs &a, const double *A, const double *c, hipStream_t s);
void launch_first_update(const FusedArgs &a, const double *A, const double *c, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1);

// Steps 1-2 (select) and the Step 3 inputs (stage) of pivot j of a group.
void launch_fused_select(const FusedArgs &a, int j, hipStream_t s);
void launch_fused_stage(const FusedArgs &a, int j, hipStream_t s);

// The pivot rows after the pure pass (k_gfix; the pure passes launch it).
void launch_fix(const FusedArgs &a, hipStream_t s);

// The group's update pass; with events, timed by the dispatch.
void launch_fused_update(const FusedArgs &a, int block, int cols, int rv, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1);

}  // namespace lpgpu
