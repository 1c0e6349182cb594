// stream.hip -- achievable-bandwidth microbenchmark (the paper's "achievable
// roof", section 7.1: a kernel doing nothing but coalesced, aligned reads and
// writes).  Copy, read-only and write-only streams with 16-byte accesses and
// a grid-stride loop, optionally with non-temporal stores; the best of them is
// the practical ceiling the sweep kernels are compared with.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/claw.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

template <bool NT>
__global__ __launch_bounds__(256) void k_copy(const f4* __restrict__ a, f4* __restrict__ b, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        f4 v = a[i];
        if (NT) __builtin_nontemporal_store(v, &b[i]);
        else b[i] = v;
    }
}

__global__ __launch_bounds__(256) void k_read(const f4* __restrict__ a, size_t n, float* sink) {
    f4 acc = {0, 0, 0, 0};
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        acc += a[i];
    const float s = acc.x + acc.y + acc.z + acc.w;
    if (s == 1234.5f) sink[0] = s;  // keeps the loads alive; never taken for zero input
}

template <bool NT>
__global__ __launch_bounds__(256) void k_write(f4* __restrict__ b, size_t n) {
    const f4 v = {0, 0, 0, 0};
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        if (NT) __builtin_nontemporal_store(v, &b[i]);
        else b[i] = v;
    }
}

}  // namespace

extern "C" claw_status claw_stream_bench(void* a, void* b, size_t bytes, int32_t reps, void* stream,
                                         double* gbps) {
    if (!a || !b || !gbps || bytes < 4096 || reps < 1) return CLAW_E_INVALID;
    hipStream_t s = (hipStream_t)stream;
    const size_t n = bytes / sizeof(f4);
    const unsigned grid = 256 * 16;  // 16 workgroups of 256 threads per CU
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return CLAW_E_HIP;
    claw_status st = CLAW_OK;
    for (int kind = 0; kind < 5 && st == CLAW_OK; ++kind) {
        float ms = 0;
        for (int pass = 0; pass < 2; ++pass) {  // pass 0 warms up
            if (hipEventRecord(e0, s) != hipSuccess) { st = CLAW_E_HIP; break; }
            for (int r = 0; r < (pass ? reps : 1); ++r) {
                switch (kind) {
                    case 0: hipLaunchKernelGGL(k_copy<false>, dim3(grid), dim3(256), 0, s, (const f4*)a, (f4*)b, n); break;
                    case 1: hipLaunchKernelGGL(k_copy<true>, dim3(grid), dim3(256), 0, s, (const f4*)a, (f4*)b, n); break;
                    case 2: hipLaunchKernelGGL(k_read, dim3(grid), dim3(256), 0, s, (const f4*)a, n, (float*)b); break;
                    case 3: hipLaunchKernelGGL(k_write<false>, dim3(grid), dim3(256), 0, s, (f4*)b, n); break;
                    default: hipLaunchKernelGGL(k_write<true>, dim3(grid), dim3(256), 0, s, (f4*)b, n); break;
                }
            }
            if (hipGetLastError() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
                hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                st = CLAW_E_HIP;
                break;
            }
        }
        const double moved = (kind <= 1 ? 2.0 : 1.0) * (double)(n * sizeof(f4)) * reps;
        gbps[kind] = moved / (ms * 1e-3) / 1e9;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}
