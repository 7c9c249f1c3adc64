// Shared pieces of the batched kernel for the batch and server front ends.
#pragma once

#include <string>

#include "batch_kernels.hpp"

namespace lpgpu {

// Shape of the persistent batched kernel: threads per workgroup, update
// unroll (row-pair items in flight per thread), workgroups per CU, and the
// most parts a large LP is split into (1: every LP on one workgroup).
struct BatchShape {
    int block;
    int unroll;
    int grid_per_cu;
    int split = 1;
};

extern const BatchShape kBatchShapes[];
extern const int kNumBatchShapes;

// Dynamic LDS of one LP in the batched kernel (F, R and the rewrite list).
size_t batch_lds_bytes(int32_t m, int32_t n);
// Whether an LP can run in the batched kernel under a per-workgroup LDS limit.
bool batch_fits(int32_t m, int32_t n, size_t lds_limit);
// Size limits of the batched kernel's (column, row pair) item split.
bool batch_size_ok(int32_t m, int32_t n);
uint64_t nvec_magic(int32_t nvec);
size_t device_lds_limit(int device);
int device_cus(int device);
int set_batch_lds_limit(size_t lds);
// Enqueues {queue reset, persistent kernel} on `stream`.
int launch_batch_kernel(const BatchShape &sh, int grid, size_t lds, hipStream_t stream, const BatchDesc *desc,
                        BatchState *state, const int32_t *order, const int32_t *norder, int32_t *head,
                        int64_t budget, const int32_t *parts = nullptr, uint32_t gate_spin = kPartGateSpin);
// Workgroups of the shape's kernel instance resident per CU with `lds` bytes
// of dynamic LDS (0 if unknown).
int batch_blocks_per_cu(const BatchShape &sh, size_t lds);
std::string batch_bucket_key(int32_t count, int32_t mmax, int32_t nmax);
bool cache_lookup(const char *path, const std::string &key, BatchShape *out);
void cache_store(const char *path, const std::string &key, const BatchShape &sh, double ms);

}  // namespace lpgpu
