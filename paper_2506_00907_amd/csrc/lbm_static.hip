// lbm_reduce_static: the FP64 reductions of lbm_reduce with their scratch in
// a library-owned device array, for callers that cannot allocate device
// memory.  The reduction kernel stores one record of 12 sums per 256-node
// block into the array (no atomics), and one block then adds the records up
// in a fixed order.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/lbm.h"
#include "lbm_ctx.hpp"
#include "lbm_internal.hpp"

using namespace lbmh;

namespace {

constexpr uint32_t kBlockNodes = 256;  // nodes per block of the observe kernel
constexpr int kRec = lbmi::NACC;       // doubles per block record
constexpr int kSums = 12;              // sums the reduction forms (lbm_reduce's h[0..11])
constexpr int kMaxDevices = 64;

// One record per block of the largest lattice, then the kSums totals.
// Each device holds its own copy for the life of the process; host code
// passes its address from hipGetSymbolAddress, never the name.
static __device__ __align__(256) double scratch[(size_t)LBM_REDUCE_STATIC_MAX_BLOCKS * kRec + kRec];

std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on `dev` (the current device), resolved once.
hipError_t scratch_ptr(int dev, double** out) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        double* p = nullptr;
        const hipError_t e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

// Adds the kSums values of nblocks records in a fixed order: thread t sums
// blocks t, t + 256, ...; then a pairwise tree over the 256 threads.
__global__ __launch_bounds__(256) void k_sum_records(const double* __restrict__ rec, uint32_t nblocks,
                                                     double* __restrict__ out) {
    __shared__ double red[kSums][256];
    const int t = threadIdx.x;
    double s[kSums];
    for (int q = 0; q < kSums; ++q) s[q] = 0.0;
    for (uint32_t b = t; b < nblocks; b += 256)
        for (int q = 0; q < kSums; ++q) s[q] += rec[(size_t)b * kRec + q];
    for (int q = 0; q < kSums; ++q) red[q][t] = s[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int q = 0; q < kSums; ++q) red[q][t] += red[q][t + w];
        __syncthreads();
    }
    if (t < kSums) out[t] = red[t][0];
}

}  // namespace

extern "C" lbm_status lbm_reduce_static(lbm_ctx* c, double out[8]) {
    if (!c || !out) return LBM_EINVAL;
    if (!c->initialized) return set_err(c, LBM_ESTATE, "lbm_init must come first");
    const size_t nodes = c->pad.nodes;
    const size_t nblocks = (nodes + kBlockNodes - 1) / kBlockNodes;
    if (nblocks > (size_t)LBM_REDUCE_STATIC_MAX_BLOCKS)
        return set_err(c, LBM_ESIZE,
                       "lattice of " + std::to_string(nodes) + " padded nodes exceeds the static reduction scratch (" +
                           std::to_string((size_t)LBM_REDUCE_STATIC_MAX_BLOCKS * kBlockNodes) + " nodes)");
    int dev = -1;
    lbm_status st;
    if ((st = hip_check(c, hipGetDevice(&dev), "current device"))) return st;
    if (dev != c->device || dev < 0 || dev >= kMaxDevices)
        return set_err(c, LBM_EINVAL, "the context's device is not the current HIP device");
    double* ptr = nullptr;
    if ((st = hip_check(c, scratch_ptr(dev, &ptr), "static scratch address"))) return st;
    double* totals = ptr + (size_t)LBM_REDUCE_STATIC_MAX_BLOCKS * kRec;

    lbmi::KArgs a = base_args(c);
    a.mode = lbmi::OBS_REDUCE;
    a.acc = ptr;  // every block stores its record: nothing to clear
    a.acc_blocks = 1;
    a.snap = c->buf[4];
    a.snap_valid = c->snap_valid ? 1 : 0;
    if ((st = hip_check(c, c->ks.observe(a), "reduce launch"))) return st;
    hipLaunchKernelGGL(k_sum_records, dim3(1), dim3(256), 0, c->stream, ptr, (uint32_t)nblocks, totals);
    if ((st = hip_check(c, hipGetLastError(), "record sum launch"))) return st;
    double h[kSums];
    if ((st = hip_check(c, hipMemcpyAsync(h, totals, sizeof h, hipMemcpyDeviceToHost, c->stream), "reduce copy")))
        return st;
    if ((st = hip_check(c, hipStreamSynchronize(c->stream), "reduce sync"))) return st;
    return finish_reduce(c, h, out);
}
