// Streaming-read probe of the device memory (diagnostic, not part of the method): the rate
// that a plain read kernel reaches on a caller's buffer, as context for the product
// kernels' fractions of the HBM peak.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

#define PR_NT 256
#define PR_U 8           // 16-byte loads in flight per thread

typedef double pr_dv2 __attribute__((ext_vector_type(2)));

// Each work group reads its own contiguous share (16-byte nontemporal loads, PR_U in flight
// per thread) and writes one partial sum per thread, so that the loads are not removed.
__global__ void __launch_bounds__(PR_NT) k_probe_read(const pr_dv2* __restrict__ p, int64_t n,
                                                      double* __restrict__ out) {
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < n ? lo + per : n;
    double s = 0.0;
    for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += (int64_t)PR_NT * PR_U) {
        pr_dv2 v[PR_U];
#pragma unroll
        for (int k = 0; k < PR_U; ++k) {
            const int64_t i = i0 + (int64_t)k * PR_NT;
            v[k] = i < hi ? __builtin_nontemporal_load(p + i) : pr_dv2{0.0, 0.0};
        }
#pragma unroll
        for (int k = 0; k < PR_U; ++k) s += v[k][0] + v[k][1];
    }
    out[(int64_t)blockIdx.x * PR_NT + threadIdx.x] = s;
}

extern "C" fbc_status fbc_probe_read(const void* buf, int64_t bytes, int groups, int reps, double* gbs,
                                     void* stream) {
    if (!buf || !gbs || bytes < 16 || (bytes & 15) || ((uintptr_t)buf & 15) || groups < 1 || groups > 65536 ||
        reps < 1 || reps > 1000)
        return FBC_E_ARG;
    hipStream_t st = (hipStream_t)stream;
    double* out = nullptr;
    if (hipMalloc((void**)&out, (size_t)groups * PR_NT * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return FBC_E_NOMEM;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    fbc_status s = FBC_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) s = FBC_E_DEVICE;
    const int64_t n = bytes / 16;
    if (s == FBC_OK) {
        hipLaunchKernelGGL(k_probe_read, dim3(groups), dim3(PR_NT), 0, st, (const pr_dv2*)buf, n, out);  // warm-up
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < reps; ++r)
            hipLaunchKernelGGL(k_probe_read, dim3(groups), dim3(PR_NT), 0, st, (const pr_dv2*)buf, n, out);
        (void)hipEventRecord(e1, st);
        float ms = 0.0f;
        if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess || !(ms > 0.0f))
            s = FBC_E_DEVICE;
        else
            *gbs = (double)bytes * reps / (ms * 1e-3) / 1e9;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    return s;
}
