// pd_probe.hip -- streaming kernels of known traffic, for measuring the
// device's achievable HBM bandwidth and for scaling the profiler's memory
// counters: a read-only pass and a copy over caller buffers.
#include <hip/hip_runtime.h>

#include "../../include/pd.h"

namespace {

// every byte of src read once as 16-byte loads, grid-stride; one word per
// workgroup is written so that the loads are not dead
__global__ __launch_bounds__(256) void k_stream_read(const uint4 *__restrict__ src, int64_t n,
                                                     uint32_t *__restrict__ sink) {
    uint32_t acc = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        const uint4 v = src[k];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    __shared__ uint32_t red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] ^= red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) sink[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_stream_copy(const uint4 *__restrict__ src, int64_t n,
                                                     uint4 *__restrict__ dst) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
        dst[k] = src[k];
}

}  // namespace

extern "C" pd_status pd_stream_probe(int32_t mode, const void *src, void *dst, int64_t bytes,
                                     int32_t reps, void *hip_stream, double *ms) {
    if (!src || !dst || bytes < 16 || bytes % 16 != 0 || reps < 1 || (mode != 0 && mode != 1) ||
        ((uintptr_t)src % 16) || ((uintptr_t)dst % 16))
        return PD_E_INVALID;
    const int64_t n = bytes / 16;
    constexpr int kBlocks = 256 * 16;  // 16 workgroups of 256 threads per compute unit
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return PD_E_DEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return PD_E_DEVICE;
    }
    pd_status st = PD_OK;
    if (hipEventRecord(e0, s) != hipSuccess) st = PD_E_DEVICE;
    for (int r = 0; r < reps && st == PD_OK; ++r) {
        if (mode == 0)
            hipLaunchKernelGGL(k_stream_read, dim3(kBlocks), dim3(256), 0, s, (const uint4 *)src, n,
                               (uint32_t *)dst);
        else
            hipLaunchKernelGGL(k_stream_copy, dim3(kBlocks), dim3(256), 0, s, (const uint4 *)src, n,
                               (uint4 *)dst);
        if (hipGetLastError() != hipSuccess) st = PD_E_DEVICE;
    }
    float t = 0.0f;
    if (st == PD_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&t, e0, e1) != hipSuccess))
        st = PD_E_DEVICE;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (ms) *ms = (double)t / reps;
    return st;
}
