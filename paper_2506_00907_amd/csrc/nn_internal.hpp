// Internal interface between the host side of the warm-start network
// (nn_host.cpp) and its kernels (nn_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace nnk {

// Kernels of one element type (BF16 with FP32 accumulation, or FP32 for the
// debug mode).  Activations are NHWC with the channel count of the tensor;
// every pointer is a device pointer.
struct NnKernels {
    // Y = act(conv(X, Wt) + bias): X [npix-shaped N,H,W][cin], Wt [taps][coutp][cin],
    // output channels [0, cstore) go to Y (element type) or, when yf is set,
    // to yf (FP32, added when accumulate).  cin % 16 == 0, coutp % 32 == 0.
    hipError_t (*conv)(const void* X, const void* Wt, const float* bias, int N, int H, int W, int cin, int coutp,
                       int cstore, int taps, int relu, void* Y, float* yf, int accumulate, hipStream_t s);
    // dWt[taps][coutp][cin] += sum_p dZ[p][co] X[p + tap][ci] (FP32 atomics)
    hipError_t (*wgrad)(const void* X, const void* dZ, int N, int H, int W, int cin, int coutp, int taps,
                        float* dWt, hipStream_t s);
    // db[co] += sum_p dZ[p][co] for co < cout
    hipError_t (*bgrad)(const void* dZ, int64_t npix, int coutp, int cout, float* db, hipStream_t s);
    // dZ = (Y > 0 ? G : 0) (relu) or G, in the element type
    hipError_t (*act_grad)(const float* G, const void* Y, int64_t n, int relu, void* dZ, hipStream_t s);
    // 2x2 average pooling (C channels), and its gradient added to the fine level
    hipError_t (*pool)(const void* X, int N, int H, int W, int C, void* Y, hipStream_t s);
    hipError_t (*pool_grad)(const float* dY, int N, int H, int W, int C, float* dX, hipStream_t s);
    // nearest x2 upsampling of the coarse tensor (c1 channels) concatenated with
    // the skip tensor (c2 channels) at the fine level H x W; and its gradient
    hipError_t (*upcat)(const void* coarse, const void* skip, int N, int H, int W, int c1, int c2, void* Y,
                        hipStream_t s);
    hipError_t (*upcat_grad)(const float* dY, int N, int H, int W, int c1, int c2, float* dcoarse, float* dskip,
                             hipStream_t s);
    // FP32 user input [npix][cin] -> element type [npix][cinp] (zero padded)
    hipError_t (*pack)(const float* x, int64_t npix, int cin, int cinp, void* X, hipStream_t s);
    // loss sum_p w_p sum_c (y - t)^2 / cout (FP64 atomic into loss[0]); G [npix][coutp] = d loss / d y
    hipError_t (*loss)(const float* y, const float* t, const float* w, int64_t npix, int cout, int coutp,
                       float* G, double* loss, hipStream_t s);
    // master weights W[co][ci][taps] (FP32) -> forward Wf[taps][coutp][cinp] and
    // backward Wb[taps][cinp][coutp] (mirrored taps) in the element type
    hipError_t (*prep)(const float* Wm, int cout, int cin, int coutp, int cinp, int taps, void* Wf, void* Wb,
                       hipStream_t s);
    // dWt[taps][coutp][cinp] -> master layout gradient g[co][ci][taps]
    hipError_t (*gather)(const float* dWt, int cout, int cin, int coutp, int cinp, int taps, float* g,
                         hipStream_t s);
    int elem_bytes;
};

NnKernels nn_kernels_bf16();
NnKernels nn_kernels_f32();

// FP32 helpers independent of the element type
hipError_t nn_fill(float* p, int64_t n, float v, hipStream_t s);
hipError_t nn_fill_f64(double* p, int64_t n, hipStream_t s);
hipError_t nn_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                   float eps, float bc1, float bc2, hipStream_t s);

}  // namespace nnk
