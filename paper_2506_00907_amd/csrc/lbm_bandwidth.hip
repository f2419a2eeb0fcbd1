// lbm_stream_bandwidth: plain streaming kernels (read, write, copy) with
// 16-byte accesses, timed with HIP events.  They measure the HBM bandwidth a
// kernel can attain on the device, the ceiling against which the sweep's
// fraction of the 8 TB/s peak is read, and they serve as the copy of known
// size that calibrates the HBM byte counters.
#include <hip/hip_runtime.h>

#include "../../include/lbm.h"

namespace {

// Grid-stride loops over 16-byte words; each thread touches `per` words,
// consecutive threads consecutive words.
__global__ __launch_bounds__(256) void k_read(const uint4* __restrict__ src, size_t n, uint32_t* __restrict__ sink) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    uint32_t acc = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint4 v = src[i];
        acc += v.x ^ v.y ^ v.z ^ v.w;
    }
    // keeps the loads: the sum is stored only when it equals a value the
    // host never fills the buffer with
    if (acc == 0x9e3779b9u) sink[0] = acc;
}

__global__ __launch_bounds__(256) void k_write(uint4* __restrict__ dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t v = (uint32_t)i;
        dst[i] = make_uint4(v, v, v, v);
    }
}

__global__ __launch_bounds__(256) void k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

hipError_t launch(int kind, const void* src, void* dst, size_t words, unsigned blocks, hipStream_t s) {
    if (kind == 0)
        hipLaunchKernelGGL(k_read, dim3(blocks), dim3(256), 0, s, (const uint4*)src, words, (uint32_t*)dst);
    else if (kind == 1)
        hipLaunchKernelGGL(k_write, dim3(blocks), dim3(256), 0, s, (uint4*)dst, words);
    else
        hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, s, (const uint4*)src, (uint4*)dst, words);
    return hipGetLastError();
}

}  // namespace

extern "C" lbm_status lbm_stream_bandwidth(int32_t kind, const void* dev_src, void* dev_dst, size_t bytes,
                                           int32_t per_thread, int32_t reps, void* hip_stream, float* ms_out) {
    if (!ms_out || kind < 0 || kind > 2 || per_thread < 1 || per_thread > 1024 || reps < 1) return LBM_EINVAL;
    if (bytes == 0 || bytes % 16) return LBM_EINVAL;
    if ((kind != 1 && (!dev_src || (uintptr_t)dev_src % 16)) || !dev_dst || (uintptr_t)dev_dst % 16)
        return LBM_EINVAL;
    const size_t words = bytes / 16;
    const size_t threads = (words + per_thread - 1) / per_thread;
    const size_t blocks = (threads + 255) / 256;
    if (blocks > 0x7fffffffu) return LBM_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return LBM_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return LBM_EDEVICE;
    }
    lbm_status st = LBM_OK;
    // one untimed launch, then reps timed back to back
    if (launch(kind, dev_src, dev_dst, words, (unsigned)blocks, s) != hipSuccess) st = LBM_EDEVICE;
    if (!st && hipEventRecord(e0, s) != hipSuccess) st = LBM_EDEVICE;
    for (int r = 0; r < reps && !st; ++r)
        if (launch(kind, dev_src, dev_dst, words, (unsigned)blocks, s) != hipSuccess) st = LBM_EDEVICE;
    if (!st && hipEventRecord(e1, s) != hipSuccess) st = LBM_EDEVICE;
    if (!st && hipEventSynchronize(e1) != hipSuccess) st = LBM_EDEVICE;
    float ms = 0.0f;
    if (!st && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = LBM_EDEVICE;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!st) *ms_out = ms / (float)reps;
    return st;
}
