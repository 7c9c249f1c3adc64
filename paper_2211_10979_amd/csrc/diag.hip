// Element-wise device division and fma, for checking the device's rounding.
#include <hip/hip_runtime.h>

#include <vector>

#include "common.hpp"

using namespace lpgpu;

namespace {

__global__ void k_diag_arith(int64_t count, const double *__restrict__ a, const double *__restrict__ b,
                             const double *__restrict__ c, double *__restrict__ quot, double *__restrict__ fmav) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    quot[k] = a[k] / b[k];
    fmav[k] = fma(a[k], b[k], c[k]);
}

// Plain copy: each thread moves U 16-byte vectors, B*U apart, loads first.
template <int U>
__global__ __launch_bounds__(256) void k_diag_copy(const double2 *__restrict__ src, double2 *__restrict__ dst,
                                                   int64_t nvec) {
    const int64_t base = (int64_t)blockIdx.x * 256 * U + threadIdx.x;
    double2 x[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
        if (base + u * 256 < nvec) x[u] = src[base + u * 256];
#pragma unroll
    for (int u = 0; u < U; ++u)
        if (base + u * 256 < nvec) dst[base + u * 256] = x[u];
}

}  // namespace

extern "C" int lp_diag_copy(int32_t device, size_t bytes, int32_t reps, double *ms) {
    if (reps < 1 || bytes < 16) return set_error(LP_E_INVAL, "bytes must be >= 16 and reps >= 1");
    int prev = 0;
    LP_HIP_CHECK(hipGetDevice(&prev));
    LP_HIP_CHECK(hipSetDevice(device));
    const int64_t nvec = (int64_t)(bytes / 16);
    double2 *src = nullptr, *dst = nullptr;
    if (hipMalloc((void **)&src, nvec * 16) != hipSuccess || hipMalloc((void **)&dst, nvec * 16) != hipSuccess) {
        if (src) (void)hipFree(src);
        (void)hipSetDevice(prev);
        return set_error(LP_E_NOMEM, "hipMalloc failed");
    }
    int rc = LP_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipMemset(src, 0, nvec * 16) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        rc = set_error(LP_E_DEVICE, "setup failed");
    } else {
        const unsigned blocks = (unsigned)((nvec + 256 * 2 - 1) / (256 * 2));
        hipLaunchKernelGGL(k_diag_copy<2>, dim3(blocks), dim3(256), 0, nullptr, src, dst, nvec);  // warm-up
        (void)hipEventRecord(e0, nullptr);
        for (int r = 0; r < reps; ++r)
            hipLaunchKernelGGL(k_diag_copy<2>, dim3(blocks), dim3(256), 0, nullptr, src, dst, nvec);
        (void)hipEventRecord(e1, nullptr);
        float t = 0.f;
        if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t, e0, e1) != hipSuccess)
            rc = set_error(LP_E_DEVICE, "copy kernel failed");
        else if (ms)
            *ms = t / reps;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(src);
    (void)hipFree(dst);
    (void)hipSetDevice(prev);
    return rc;
}

extern "C" int lp_diag_arith(int32_t device, int64_t count, const double *a, const double *b, const double *c,
                             double *quot, double *fmav) {
    if (count < 0 || (count > 0 && (!a || !b || !c || !quot || !fmav))) return set_error(LP_E_INVAL, "bad argument");
    if (count == 0) return LP_OK;
    int prev = 0;
    LP_HIP_CHECK(hipGetDevice(&prev));
    LP_HIP_CHECK(hipSetDevice(device));
    double *d = nullptr;
    const size_t bytes = (size_t)count * sizeof(double);
    hipError_t e = hipMalloc((void **)&d, 5 * bytes);
    if (e != hipSuccess) {
        (void)hipSetDevice(prev);
        return set_error(LP_E_NOMEM, "hipMalloc failed");
    }
    int rc = LP_OK;
    if (hipMemcpy(d, a, bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d + count, b, bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d + 2 * count, c, bytes, hipMemcpyHostToDevice) != hipSuccess) {
        rc = set_error(LP_E_DEVICE, "copy to device failed");
    } else {
        hipLaunchKernelGGL(k_diag_arith, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, nullptr, count, d,
                           d + count, d + 2 * count, d + 3 * count, d + 4 * count);
        if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
            hipMemcpy(quot, d + 3 * count, bytes, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(fmav, d + 4 * count, bytes, hipMemcpyDeviceToHost) != hipSuccess)
            rc = set_error(LP_E_DEVICE, "diagnostic kernel failed");
    }
    (void)hipFree(d);
    (void)hipSetDevice(prev);
    return rc;
}
