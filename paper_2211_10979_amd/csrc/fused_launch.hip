// Instances and launchers of the pivot-fusion kernels.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <atomic>

#include "fused_launch.hpp"

namespace lpgpu {

namespace {

template <int J>
void select_j(const FusedArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_gselect<J>), dim3((unsigned)a.select_wgs), dim3(256), 0, s, (const double *)a.T, a.ld, a.m,
                       a.n, a.K, (const ArgMin *)a.parts, (const SPart *)a.sparts, a.nsparts, a.st, a.gs, a.Fk, a.Rk,
                       a.D, a.cols, a.pos, a.basis, a.log_r, a.log_q, a.rparts, a.ticket);
}

template <int J>
void stage_j(const FusedArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_gstage<J>), dim3((unsigned)a.nsparts), dim3(256), 0, s, (const double *)a.T, a.ld, a.m,
                       a.n, a.K, (const GroupState *)a.gs, (const double *)a.Fk, a.Rk, a.D, (const int32_t *)a.cols,
                       a.sparts);
}

template <int B, int C, int KF>
void update(const FusedArgs &a, unsigned grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const int64_t Lg = (int64_t)a.n + 1 + a.K;
    if (e0)
        hipExtLaunchKernelGGL((k_gupdate<B, C, KF>), dim3(grid), dim3(B), 0, s, e0, e1, 0, a.T, a.ld, a.m, a.n, Lg,
                              a.rowchunks, (const int32_t *)a.cols, (const double *)a.Rk, (const double *)a.Fk,
                              (const GroupState *)a.gs, a.parts, a.cols_done);
    else
        hipLaunchKernelGGL((k_gupdate<B, C, KF>), dim3(grid), dim3(B), 0, s, a.T, a.ld, a.m, a.n, Lg, a.rowchunks,
                           (const int32_t *)a.cols, (const double *)a.Rk, (const double *)a.Fk,
                           (const GroupState *)a.gs, a.parts, a.cols_done);
}

template <int B, int C, int KF>
void update_pure(const FusedArgs &a, unsigned, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const int64_t Lg = (int64_t)a.n + 1 + a.K;
    const int32_t rowchunks = (int32_t)((((int64_t)a.m + 2) / 2 + B - 1) / B);  // row pairs
    const unsigned grid = (unsigned)((int64_t)rowchunks * a.nparts);
    if (e0)
        hipExtLaunchKernelGGL((k_gupdate_pure<B, C, KF>), dim3(grid), dim3(B), 0, s, e0, e1, 0, a.T, a.ld, a.m, a.n,
                              Lg, rowchunks, (const int32_t *)a.cols, (const double *)a.Rk, (const double *)a.Fk,
                              (const GroupState *)a.gs, a.dump, 0);
    else
        hipLaunchKernelGGL((k_gupdate_pure<B, C, KF>), dim3(grid), dim3(B), 0, s, a.T, a.ld, a.m, a.n, Lg, rowchunks,
                           (const int32_t *)a.cols, (const double *)a.Rk, (const double *)a.Fk,
                           (const GroupState *)a.gs, a.dump, 0);
}

// The pure pass in row-lane tiles (k_gpure_rl) over slots slot0 .. n+K.
template <int KF>
void launch_pure_rl(const FusedArgs &a, int32_t slot0, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const int64_t Lg = (int64_t)a.n + 1 + a.K;
    const int32_t nrt = (a.m + kRlRows) / kRlRows;  // tiles of rows 0..m
    const unsigned grid = (unsigned)((int64_t)nrt * ((Lg - slot0 + kRlSlots - 1) / kRlSlots));
    if (e0 || e1)
        hipExtLaunchKernelGGL((k_gpure_rl<KF>), dim3(grid), dim3(256), 0, s, e0, e1, 0, a.T, a.ld, a.m, a.n, Lg, nrt,
                              (const int32_t *)a.cols, (const double *)a.Rk, (const double *)a.Fk,
                              (const GroupState *)a.gs, slot0);
    else
        hipLaunchKernelGGL((k_gpure_rl<KF>), dim3(grid), dim3(256), 0, s, a.T, a.ld, a.m, a.n, Lg, nrt,
                           (const int32_t *)a.cols, (const double *)a.Rk, (const double *)a.Fk,
                           (const GroupState *)a.gs, slot0);
}

// The pure pass on the matrix cores (k_gpure_mf) over slots slot0 .. n+K.
template <int KF>
void launch_pure_mf(const FusedArgs &a, int32_t slot0, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const int64_t Lg = (int64_t)a.n + 1 + a.K;
    const int32_t nrt = (int32_t)((a.ld + kMfRows - 1) / kMfRows);
    const unsigned grid = (unsigned)((int64_t)nrt * ((Lg - slot0 + kMfSlots - 1) / kMfSlots));
    if (e0 || e1)
        hipExtLaunchKernelGGL((k_gpure_mf<KF>), dim3(grid), dim3(256), 0, s, e0, e1, 0, a.T, a.ld, a.m, a.n, Lg, nrt,
                              (const int32_t *)a.cols, (const double *)a.Rk, (const double *)a.Fk,
                              (const GroupState *)a.gs, slot0);
    else
        hipLaunchKernelGGL((k_gpure_mf<KF>), dim3(grid), dim3(256), 0, s, a.T, a.ld, a.m, a.n, Lg, nrt,
                           (const int32_t *)a.cols, (const double *)a.Rk, (const double *)a.Fk,
                           (const GroupState *)a.gs, slot0);
}

template <int B, int C, int KF>
void update_pure_mf(const FusedArgs &a, unsigned, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    launch_pure_mf<KF>(a, 0, s, e0, e1);
}

using UpdateFn = void (*)(const FusedArgs &, unsigned, hipStream_t, hipEvent_t, hipEvent_t);

template <int B, int C>
UpdateFn pick_pure(int K) {
    switch (fused_update_kf(K)) {
        case 2: return update_pure<B, C, 2>;
        case 4: return update_pure<B, C, 4>;
        case 8: return update_pure<B, C, 8>;
        case 12: return update_pure<B, C, 12>;
        case 16: return update_pure<B, C, 16>;
        default: break;
    }
    if constexpr (C >= 4) {  // groups above 16 pivots: 4 or 8 slots per workgroup; 48 on the matrix cores
        switch (fused_update_kf(K)) {
            case 24: return update_pure<B, C, 24>;
            case 32: return update_pure<B, C, 32>;
            case 48: return update_pure_mf<B, C, 48>;
            default: break;
        }
    }
    return nullptr;
}

// The pure update pass (with the one-launch decision kernel), same shapes.
UpdateFn find_update_pure(int block, int cols, int rv, int K) {
    if (rv != 1 || K < 2 || K > kMaxFuse) return nullptr;
#define LP_PSHAPE(B, C) \
    if (block == B && cols == C) return pick_pure<B, C>(K);
    LP_PSHAPE(256, 1) LP_PSHAPE(256, 2) LP_PSHAPE(256, 4) LP_PSHAPE(256, 8)
    LP_PSHAPE(128, 1) LP_PSHAPE(128, 2) LP_PSHAPE(128, 4) LP_PSHAPE(128, 8)
    LP_PSHAPE(64, 1) LP_PSHAPE(64, 2) LP_PSHAPE(64, 4) LP_PSHAPE(64, 8)
#undef LP_PSHAPE
    return nullptr;
}

// Update instances exist for groups of up to 2, 4, 8, 12 and 16 pivots; a
// group size in between takes the next larger instance (its surplus pivots
// are exact identities).
template <int B, int C>
UpdateFn pick_k(int K) {
    if (K < 2) return nullptr;
    if (K <= 2) return update<B, C, 2>;
    if (K <= 4) return update<B, C, 4>;
    if (K <= 8) return update<B, C, 8>;
    if (K <= 12) return update<B, C, 12>;
    if (K <= 16) return update<B, C, 16>;
    return nullptr;
}

// Tile shapes with instances: 64, 128 or 256 threads (one row pair each) by
// 1, 2, 4 or 8 list slots.
UpdateFn find_update(int block, int cols, int rv, int K) {
    if (rv != 1 || K > kMaxFuseSplit) return nullptr;
#define LP_FSHAPE(B, C) \
    if (block == B && cols == C) return pick_k<B, C>(K);
    LP_FSHAPE(256, 1) LP_FSHAPE(256, 2) LP_FSHAPE(256, 4) LP_FSHAPE(256, 8)
    LP_FSHAPE(128, 1) LP_FSHAPE(128, 2) LP_FSHAPE(128, 4) LP_FSHAPE(128, 8)
    LP_FSHAPE(64, 1) LP_FSHAPE(64, 2) LP_FSHAPE(64, 4) LP_FSHAPE(64, 8)
#undef LP_FSHAPE
    return nullptr;
}

}  // namespace

bool fused_update_supported(int block, int cols, int rv, int K, bool one_launch) {
    return (one_launch ? find_update_pure(block, cols, rv, K) : find_update(block, cols, rv, K)) != nullptr;
}

template <int BD, bool First, int KM>
void decide_bd(const FusedArgs &a, const double *A, const double *c, hipStream_t s) {
    hipLaunchKernelGGL((k_gdecide<BD, First, KM>), dim3((unsigned)a.decide_wgs), dim3(BD), 0, s, a.T, a.ld, a.m, a.n,
                       A, c, a.K, a.KF, a.sparts, a.cols_done, a.st, a.gs, a.Fk, a.Rk, a.cols, a.pos, a.basis,
                       a.log_r, a.log_q, a.rparts, a.gsync, a.decide_spin, a.gate_spin, a.PV, a.pub, a.pub_words,
                       a.pub_seq_at, a.pub_seq, a.t_mark);
}

// the instance for the group size (its KF pivot slots kept in registers)
template <int BD, bool First>
void decide_kf(const FusedArgs &a, const double *A, const double *c, hipStream_t s) {
    switch (a.KF) {
        case 2: decide_bd<BD, First, 2>(a, A, c, s); break;
        case 4: decide_bd<BD, First, 4>(a, A, c, s); break;
        case 8: decide_bd<BD, First, 8>(a, A, c, s); break;
        case 12: decide_bd<BD, First, 12>(a, A, c, s); break;
        case 16: decide_bd<BD, First, 16>(a, A, c, s); break;
        default: break;
    }
    if constexpr (BD == 256) {  // larger groups: 256 threads per workgroup only (the host checks)
        switch (a.KF) {
            case 24: decide_bd<BD, First, 24>(a, A, c, s); break;
            case 32: decide_bd<BD, First, 32>(a, A, c, s); break;
            case 48: decide_bd<BD, First, 48>(a, A, c, s); break;
            default: break;
        }
    }
}

namespace {

template <int BD, int KM>
int occupancy_pair() {
    int a = 0, b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, reinterpret_cast<const void *>(&k_gdecide<BD, false, KM>),
                                                     BD, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, reinterpret_cast<const void *>(&k_gdecide<BD, true, KM>),
                                                     BD, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return a < b ? a : b;
}

template <int BD>
int occupancy_kf(int KF) {
    switch (KF) {
        case 2: return occupancy_pair<BD, 2>();
        case 4: return occupancy_pair<BD, 4>();
        case 8: return occupancy_pair<BD, 8>();
        case 12: return occupancy_pair<BD, 12>();
        case 16: return occupancy_pair<BD, 16>();
        default: break;
    }
    if constexpr (BD == 256) {
        switch (KF) {
            case 24: return occupancy_pair<BD, 24>();
            case 32: return occupancy_pair<BD, 32>();
            case 48: return occupancy_pair<BD, 48>();
            default: break;
        }
    }
    return 0;
}

}  // namespace

// (queried once per form: the figure depends only on the compiled kernel)
int decide_blocks_per_cu(int block, int KF) {
    static std::atomic<int> cache[2][kMaxFuse + 1];
    if ((block != 256 && block != 512) || KF < 0 || KF > kMaxFuse) return 0;
    std::atomic<int> &slot = cache[block == 512][KF];
    int v = slot.load(std::memory_order_relaxed);
    if (v == 0) {
        v = (block == 512 ? occupancy_kf<512>(KF) : occupancy_kf<256>(KF)) + 1;  // stored + 1: 0 means unknown
        slot.store(v, std::memory_order_relaxed);
    }
    return v - 1;
}

void launch_fused_decide(const FusedArgs &a, hipStream_t s) {
    if (a.decide_block == 512)
        decide_kf<512, false>(a, nullptr, nullptr, s);
    else
        decide_kf<256, false>(a, nullptr, nullptr, s);
}

void launch_first_decide(const FusedArgs &a, const double *A, const double *c, hipStream_t s) {
    if (a.decide_block == 512)
        decide_kf<512, true>(a, A, c, s);
    else
        decide_kf<256, true>(a, A, c, s);
}

namespace {

// The first pass in row-lane tiles: the structural columns (rows 0 .. ld-1,
// padding written as zeros), then the pure pass over slots n .. n+K.
template <int KF>
void first_kf_rl(const FusedArgs &a, const double *A, const double *c, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const int64_t Lg = (int64_t)a.n + 1 + a.K;
    const int32_t nrt = (int32_t)((a.ld + kRlRows - 1) / kRlRows);
    const unsigned grid = (unsigned)((int64_t)nrt * ((a.n + kRlSlots - 1) / kRlSlots));
    if (e0)
        hipExtLaunchKernelGGL((k_gfirst_rl<KF>), dim3(grid), dim3(256), 0, s, e0, nullptr, 0, a.T, a.ld, a.m, a.n, Lg,
                              nrt, A, c, (const double *)a.Rk, (const double *)a.Fk, (const GroupState *)a.gs);
    else
        hipLaunchKernelGGL((k_gfirst_rl<KF>), dim3(grid), dim3(256), 0, s, a.T, a.ld, a.m, a.n, Lg, nrt, A, c,
                           (const double *)a.Rk, (const double *)a.Fk, (const GroupState *)a.gs);
    launch_pure_rl<KF>(a, a.n, s, nullptr, e1);
}

template <int KF>
void first_kf(const FusedArgs &a, const double *A, const double *c, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if constexpr (KF >= kRlFromKF) {
        first_kf_rl<KF>(a, A, c, s, e0, e1);
        return;
    }
    const int64_t Lg = (int64_t)a.n + 1 + a.K;
    const int32_t ntx = (a.n + kFirstTile - 1) / kFirstTile;
    const int32_t nty = (int32_t)((a.ld + kFirstRows - 1) / kFirstRows);
    const int32_t tiles = (int32_t)((int64_t)ntx * nty);
    // the tiles of the structural columns, then in the same launch the pure
    // pass over slots n .. n+K (the RHS and the appended columns)
    const int32_t rowchunks = (int32_t)((((int64_t)a.m + 2) / 2 + 255) / 256);  // row pairs
    const unsigned grid = (unsigned)(tiles + (int64_t)rowchunks * ((1 + a.K + kFirstTailC - 1) / kFirstTailC));
    if (e0 || e1)
        hipExtLaunchKernelGGL((k_gfirst<KF>), dim3(grid), dim3(256), 0, s, e0, e1, 0, a.T, a.ld, a.m, a.n, Lg, ntx, A,
                              c, (const double *)a.Rk, (const double *)a.Fk, (const GroupState *)a.gs, tiles,
                              rowchunks, (const int32_t *)a.cols, a.dump);
    else
        hipLaunchKernelGGL((k_gfirst<KF>), dim3(grid), dim3(256), 0, s, a.T, a.ld, a.m, a.n, Lg, ntx, A, c,
                           (const double *)a.Rk, (const double *)a.Fk, (const GroupState *)a.gs, tiles, rowchunks,
                           (const int32_t *)a.cols, a.dump);
}

}  // namespace

void launch_first_update(const FusedArgs &a, const double *A, const double *c, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1) {
    switch (a.KF) {
        case 2: first_kf<2>(a, A, c, s, e0, e1); break;
        case 4: first_kf<4>(a, A, c, s, e0, e1); break;
        case 8: first_kf<8>(a, A, c, s, e0, e1); break;
        case 12: first_kf<12>(a, A, c, s, e0, e1); break;
        case 16: first_kf<16>(a, A, c, s, e0, e1); break;
        case 24: first_kf<24>(a, A, c, s, e0, e1); break;
        case 32: first_kf<32>(a, A, c, s, e0, e1); break;
        case 48: first_kf<48>(a, A, c, s, e0, e1); break;
        default: break;
    }
    launch_fix(a, s);
}

void launch_fused_select(const FusedArgs &a, int j, hipStream_t s) {
    switch (j) {
        case 0: select_j<0>(a, s); break;
        case 1: select_j<1>(a, s); break;
        case 2: select_j<2>(a, s); break;
        case 3: select_j<3>(a, s); break;
        case 4: select_j<4>(a, s); break;
        case 5: select_j<5>(a, s); break;
        case 6: select_j<6>(a, s); break;
        case 7: select_j<7>(a, s); break;
        case 8: select_j<8>(a, s); break;
        case 9: select_j<9>(a, s); break;
        case 10: select_j<10>(a, s); break;
        case 11: select_j<11>(a, s); break;
        case 12: select_j<12>(a, s); break;
        case 13: select_j<13>(a, s); break;
        case 14: select_j<14>(a, s); break;
        case 15: select_j<15>(a, s); break;
        default: break;
    }
}

void launch_fused_stage(const FusedArgs &a, int j, hipStream_t s) {
    switch (j) {
        case 0: stage_j<0>(a, s); break;
        case 1: stage_j<1>(a, s); break;
        case 2: stage_j<2>(a, s); break;
        case 3: stage_j<3>(a, s); break;
        case 4: stage_j<4>(a, s); break;
        case 5: stage_j<5>(a, s); break;
        case 6: stage_j<6>(a, s); break;
        case 7: stage_j<7>(a, s); break;
        case 8: stage_j<8>(a, s); break;
        case 9: stage_j<9>(a, s); break;
        case 10: stage_j<10>(a, s); break;
        case 11: stage_j<11>(a, s); break;
        case 12: stage_j<12>(a, s); break;
        case 13: stage_j<13>(a, s); break;
        case 14: stage_j<14>(a, s); break;
        case 15: stage_j<15>(a, s); break;
        default: break;
    }
}

void launch_fused_update(const FusedArgs &a, int block, int cols, int rv, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1) {
    const unsigned grid = (unsigned)((int64_t)a.rowchunks * a.nparts);
    if (a.decide_wgs > 0) {
        if (UpdateFn f = find_update_pure(block, cols, rv, a.K)) f(a, grid, s, e0, e1);
        launch_fix(a, s);
    } else if (UpdateFn f = find_update(block, cols, rv, a.K)) {
        f(a, grid, s, e0, e1);
    }
}

void launch_fix(const FusedArgs &a, hipStream_t s) {
    const int64_t Lg = (int64_t)a.n + 1 + a.K;
    const int64_t total = (int64_t)a.K * Lg;
    hipLaunchKernelGGL(k_gfix, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a.T, a.ld, a.n, Lg,
                       (const int32_t *)a.cols, (const double *)a.PV, (const GroupState *)a.gs);
}

}  // namespace lpgpu
