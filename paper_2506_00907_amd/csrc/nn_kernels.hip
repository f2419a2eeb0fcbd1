// Kernels of the warm-start network: implicit-GEMM convolutions on the gfx950
// matrix cores (v_mfma_f32_32x32x16_bf16 for BF16 activations and weights with
// FP32 accumulation; v_mfma_f32_32x32x2_f32 for the FP32 debug mode), their
// weight gradients, and the element-wise pieces (pooling, upsampling with
// concatenation, activation gradient, loss, Adam).
//
// Tensors are NHWC.  One wave computes a 32 (pixels) x 32 (channels) block per
// matrix instruction: lane l supplies row l % 32 of A (a pixel, or an output
// channel for the weight gradient) and column l % 32 of B, with the K slice
// of half-wave l / 32; the 16 accumulators of a lane hold column l % 32 and
// rows 8 (r / 4) + 4 (l / 32) + r % 4.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "nn_internal.hpp"

namespace nnk {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

template <class T> __device__ __forceinline__ float tof(T v) { return (float)v; }
template <class T> __device__ __forceinline__ T fromf(float v) { return (T)v; }

constexpr int kBlock = 256;

inline unsigned blocks_for(int64_t n, int per = kBlock) {
    int64_t b = (n + per - 1) / per;
    return (unsigned)(b < 1 ? 1 : (b > (1 << 30) ? (1 << 30) : b));
}

// ---------------------------------------------------------------------------
// convolution: Y[p][co] = act(bias[co] + sum_tap sum_ci X[p + tap][ci] Wt[tap][co][ci])
// ---------------------------------------------------------------------------
template <class T, int NB>
__global__ __launch_bounds__(256) void k_conv(const T* __restrict__ X, const T* __restrict__ Wt,
                                              const float* __restrict__ bias, int N, int H, int W, int cin,
                                              int coutp, int cstore, int taps, int relu, T* __restrict__ Y,
                                              float* __restrict__ yf, int accumulate) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int li = lane & 31, lh = lane >> 5;
    const int64_t npix = (int64_t)N * H * W;
    const int64_t p0 = ((int64_t)blockIdx.x * 4 + wv) * 32;
    if (p0 >= npix) return;
    const int cb = blockIdx.y * 32 * NB;
    const int64_t p = p0 + li;
    const bool pv = p < npix;
    int x = 0, y = 0, n = 0;
    if (pv) {
        x = (int)(p % W);
        const int64_t t = p / W;
        y = (int)(t % H);
        n = (int)(t / H);
    }
    f32x16 acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[b][r] = 0.f;
    for (int tap = 0; tap < taps; ++tap) {
        const int dy = taps == 9 ? tap / 3 - 1 : 0, dx = taps == 9 ? tap % 3 - 1 : 0;
        const int yy = y + dy, xx = x + dx;
        const bool in = pv && (unsigned)yy < (unsigned)H && (unsigned)xx < (unsigned)W;
        // clamped address when outside: nothing is read from it
        const T* xr = X + (((int64_t)n * H + (in ? yy : 0)) * W + (in ? xx : 0)) * cin;
        const T* wr = Wt + ((int64_t)tap * coutp + cb + li) * cin;
        for (int c0 = 0; c0 < cin; c0 += 16) {
            if constexpr (sizeof(T) == 2) {
                u16x8 ra = {0, 0, 0, 0, 0, 0, 0, 0};
                if (in) ra = *(const u16x8*)(xr + c0 + 8 * lh);
                const bf16x8 a = __builtin_bit_cast(bf16x8, ra);
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const bf16x8 w = __builtin_bit_cast(bf16x8, *(const u16x8*)(wr + (int64_t)b * 32 * cin + c0 + 8 * lh));
                    acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, w, acc[b], 0, 0, 0);
                }
            } else {
#pragma unroll
                for (int s = 0; s < 8; ++s) {
                    const float a = in ? (float)xr[c0 + 2 * s + lh] : 0.f;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const float w = (float)wr[(int64_t)b * 32 * cin + c0 + 2 * s + lh];
                        acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, w, acc[b], 0, 0, 0);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int co = cb + b * 32 + li;
        if (co >= cstore) continue;
        const float bi = bias ? bias[co] : 0.f;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t pix = p0 + 8 * (r >> 2) + 4 * lh + (r & 3);
            if (pix >= npix) continue;
            float v = acc[b][r] + bi;
            if (relu) v = fmaxf(v, 0.f);
            if (yf) {
                float* d = yf + pix * cstore + co;
                *d = accumulate ? *d + v : v;
            } else {
                Y[pix * cstore + co] = fromf<T>(v);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// weight gradient: dWt[tap][co][ci] += sum_p dZ[p][co] X[p + tap][ci]
// rows of the product: output channels (A = dZ^T), columns: input channels
// (B = shifted X), K: pixels in chunks of 16; each block sums a pixel range
// over its four waves, then one FP32 atomic per weight
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void k_wgrad(const T* __restrict__ X, const T* __restrict__ dZ, int N, int H,
                                               int W, int cin, int coutp, int taps, int64_t chunks_per_block,
                                               float* __restrict__ dWt) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int li = lane & 31, lh = lane >> 5;
    const int nci = (cin + 31) / 32, nco = coutp / 32;
    int g = blockIdx.y;
    const int cib = (g % nci) * 32;
    g /= nci;
    const int cob = (g % nco) * 32;
    const int tap = g / nco;
    const int dy = taps == 9 ? tap / 3 - 1 : 0, dx = taps == 9 ? tap % 3 - 1 : 0;
    const int64_t npix = (int64_t)N * H * W;
    const int64_t nchunks = (npix + 15) / 16;
    const int64_t c_begin = (int64_t)blockIdx.x * chunks_per_block;
    const int64_t c_end = c_begin + chunks_per_block < nchunks ? c_begin + chunks_per_block : nchunks;
    const int co = cob + li, ci = cib + li;
    const bool civ = ci < cin;
    constexpr int KL = sizeof(T) == 2 ? 8 : 1;  // K values per lane and instruction
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    for (int64_t c = c_begin + wv; c < c_end; c += 4) {
        if constexpr (sizeof(T) == 2) {
            // pixels q0 .. q0 + 7 of this half-wave
            const int64_t q0 = c * 16 + 8 * lh;
            int x = (int)(q0 % W);
            int64_t t = q0 / W;
            int y = (int)(t % H);
            int n = (int)(t / H);
            u16x8 ra, rb;
#pragma unroll
            for (int j = 0; j < KL; ++j) {
                const int64_t q = q0 + j;
                const bool qv = q < npix;
                const int yy = y + dy, xx = x + dx;
                const bool in = qv && civ && (unsigned)yy < (unsigned)H && (unsigned)xx < (unsigned)W;
                ra[j] = qv ? __builtin_bit_cast(uint16_t, dZ[q * coutp + co]) : (uint16_t)0;
                rb[j] = in ? __builtin_bit_cast(uint16_t, X[(((int64_t)n * H + yy) * W + xx) * cin + ci]) : (uint16_t)0;
                if (++x == W) {
                    x = 0;
                    if (++y == H) {
                        y = 0;
                        ++n;
                    }
                }
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ra), __builtin_bit_cast(bf16x8, rb),
                                                          acc, 0, 0, 0);
        } else {
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int64_t q = c * 16 + 2 * s + lh;
                const bool qv = q < npix;
                int x = 0, y = 0, n = 0;
                if (qv) {
                    x = (int)(q % W);
                    const int64_t t = q / W;
                    y = (int)(t % H);
                    n = (int)(t / H);
                }
                const int yy = y + dy, xx = x + dx;
                const bool in = qv && civ && (unsigned)yy < (unsigned)H && (unsigned)xx < (unsigned)W;
                const float a = qv ? (float)dZ[q * coutp + co] : 0.f;
                const float b = in ? (float)X[(((int64_t)n * H + yy) * W + xx) * cin + ci] : 0.f;
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
            }
        }
    }
    __shared__ float red[4][16][64];
#pragma unroll
    for (int r = 0; r < 16; ++r) red[wv][r][lane] = acc[r];
    __syncthreads();
    if (wv == 0) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const float s = red[0][r][lane] + red[1][r][lane] + red[2][r][lane] + red[3][r][lane];
            const int row = 8 * (r >> 2) + 4 * lh + (r & 3);
            if (civ) atomicAdd(&dWt[((int64_t)tap * coutp + cob + row) * cin + ci], s);
        }
    }
}

// BF16 weight gradient of one (output, input) channel tile for one row of
// taps (NT = 3: the taps dx = -1, 0, 1 of row dy = blockIdx.z - 1 of a 3 x 3
// kernel; NT = 1: the 1 x 1 kernel).  Per chunk of 16 pixels, lane
// (px = l % 16, g = l / 16) loads 8 channels of one pixel in one 16-byte
// access: of dZ (shared by the taps of the row) and of X at the pixel shifted
// by each tap (zero outside the image).  The values go to LDS as
// [channel][pixel], where each lane then reads the 8 pixels of its channel in
// one 16-byte access, the operand layout of the matrix instruction above
// (K = pixels).  The next chunk's loads are issued before the current chunk's
// barrier and products.  Every wave runs the same number of chunk iterations
// (chunks past the block's range contribute zeros), so the block barriers are
// uniform.  cin and coutp are multiples of 16 and 32: each 8-channel group is
// wholly inside or outside the tensor and 16-byte aligned.
template <int NT>
__global__ __launch_bounds__(256) void k_wgrad_lds(const __bf16* __restrict__ X, const __bf16* __restrict__ dZ, int N,
                                                   int H, int W, int cin, int coutp, int64_t chunks_per_block,
                                                   float* __restrict__ dWt) {
    constexpr int RS = 16;  // LDS row: 16 pixels of one channel
    __shared__ uint16_t sA[4][32 * RS];
    __shared__ uint16_t sB[4][NT][32 * RS];
    __shared__ float red[16 * 256];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int li = lane & 31, lh = lane >> 5;
    const int px = lane & 15, grp = lane >> 4;
    const int nci = (cin + 31) / 32;
    const int cib = (blockIdx.y % nci) * 32, cob = (blockIdx.y / nci) * 32;
    const int dy = NT == 3 ? (int)blockIdx.z - 1 : 0;
    const int64_t npix = (int64_t)N * H * W;
    const int64_t nchunks = (npix + 15) / 16;
    const int64_t c_begin = (int64_t)blockIdx.x * chunks_per_block;
    int64_t c_end = c_begin + chunks_per_block;
    if (c_end > nchunks) c_end = nchunks;
    const int64_t iters = (chunks_per_block + 3) / 4;
    const int ci0 = cib + 8 * grp;  // this lane's channel group
    const bool cin_ok = ci0 < cin;
    // this lane's values of chunk c: dZ at its pixel, X at the shifted pixels
    auto load = [&](int64_t c, u16x8& va, u16x8 (&vb)[NT]) {
        const int64_t q = c * 16 + px;
        const bool qv = c < c_end && q < npix;
        int x = 0, y = 0, n = 0;
        if (qv) {
            x = (int)(q % W);
            const int64_t t1 = q / W;
            y = (int)(t1 % H);
            n = (int)(t1 / H);
        }
        va = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
        if (qv) va = *(const u16x8*)(dZ + q * coutp + cob + 8 * grp);
        const int yy = y + dy;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int xx = x + (NT == 3 ? t - 1 : 0);
            const bool in = qv && cin_ok && (unsigned)yy < (unsigned)H && (unsigned)xx < (unsigned)W;
            vb[t] = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
            if (in) vb[t] = *(const u16x8*)(X + (((int64_t)n * H + yy) * W + xx) * cin + ci0);
        }
    };
    f32x16 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[t][r] = 0.f;
    u16x8 va, vb[NT];
    load(c_begin + wv, va, vb);
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 8; ++j) sA[wv][(8 * grp + j) * RS + px] = va[j];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int j = 0; j < 8; ++j) sB[wv][t][(8 * grp + j) * RS + px] = vb[t][j];
        if (it + 1 < iters) load(c_begin + wv + 4 * (it + 1), va, vb);  // in flight during the products
        __syncthreads();
        const u16x8 ra = *(const u16x8*)&sA[wv][li * RS + 8 * lh];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const u16x8 rb = *(const u16x8*)&sB[wv][t][li * RS + 8 * lh];
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ra), __builtin_bit_cast(bf16x8, rb),
                                                             acc[t], 0, 0, 0);
        }
        __syncthreads();
    }
    // sum the four waves through LDS (one tap at a time), one FP32 atomic per weight
    const int ci = cib + li;
#pragma unroll
    for (int t = 0; t < NT; ++t) {  // unrolled: acc[t] stays in registers
#pragma unroll
        for (int r = 0; r < 16; ++r) red[r * 256 + threadIdx.x] = acc[t][r];
        __syncthreads();
        if (wv == 0 && ci < cin) {
            const int tap = NT == 3 ? (dy + 1) * 3 + t : 0;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float sum = red[r * 256 + lane] + red[r * 256 + 64 + lane] + red[r * 256 + 128 + lane] +
                                  red[r * 256 + 192 + lane];
                const int row = 8 * (r >> 2) + 4 * lh + (r & 3);
                atomicAdd(&dWt[((int64_t)tap * coutp + cob + row) * cin + ci], sum);
            }
        }
        __syncthreads();
    }
}

// bias gradient: db[co] += sum_p dZ[p][co]   (coutp divides the block size)
template <class T>
__global__ __launch_bounds__(256) void k_bgrad(const T* __restrict__ dZ, int64_t npix, int coutp, int cout,
                                               float* __restrict__ db) {
    const int per = (int)blockDim.x / coutp;
    const int c = (int)threadIdx.x % coutp, r = (int)threadIdx.x / coutp;
    float s = 0.f;
    if (r < per)
        for (int64_t p = (int64_t)blockIdx.x * per + r; p < npix; p += (int64_t)gridDim.x * per) s += tof(dZ[p * coutp + c]);
    __shared__ float red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    if ((int)threadIdx.x < coutp && (int)threadIdx.x < cout) {
        float t = 0.f;
        for (int k = 0; k < per; ++k) t += red[k * coutp + threadIdx.x];
        atomicAdd(&db[threadIdx.x], t);
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_act_grad(const float* __restrict__ G, const T* __restrict__ Y, int64_t n,
                                                  int relu, T* __restrict__ dZ) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float g = G[i];
        dZ[i] = fromf<T>((relu && !(tof(Y[i]) > 0.f)) ? 0.f : g);
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_pool(const T* __restrict__ X, int N, int H, int W, int C, T* __restrict__ Y) {
    const int Ho = H / 2, Wo = W / 2;
    const int64_t n_out = (int64_t)N * Ho * Wo * C;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_out; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        int64_t t = i / C;
        const int x = (int)(t % Wo);
        t /= Wo;
        const int y = (int)(t % Ho);
        const int n = (int)(t / Ho);
        const T* b = X + (((int64_t)n * H + 2 * y) * W + 2 * x) * C + c;
        const float s = tof(b[0]) + tof(b[C]) + tof(b[(int64_t)W * C]) + tof(b[(int64_t)W * C + C]);
        Y[i] = fromf<T>(0.25f * s);
    }
}

__global__ __launch_bounds__(256) void k_pool_grad(const float* __restrict__ dY, int N, int H, int W, int C,
                                                   float* __restrict__ dX) {
    const int64_t n_in = (int64_t)N * H * W * C;
    const int Ho = H / 2, Wo = W / 2;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_in; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        int64_t t = i / C;
        const int x = (int)(t % W);
        t /= W;
        const int y = (int)(t % H);
        const int n = (int)(t / H);
        dX[i] += 0.25f * dY[(((int64_t)n * Ho + y / 2) * Wo + x / 2) * C + c];
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_upcat(const T* __restrict__ coarse, const T* __restrict__ skip, int N, int H,
                                               int W, int c1, int c2, T* __restrict__ Y) {
    const int C = c1 + c2;
    const int64_t n_out = (int64_t)N * H * W * C;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_out; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const int64_t p = i / C;
        const int x = (int)(p % W);
        int64_t t = p / W;
        const int y = (int)(t % H);
        const int n = (int)(t / H);
        Y[i] = c < c1 ? coarse[(((int64_t)n * (H / 2) + y / 2) * (W / 2) + x / 2) * c1 + c] : skip[p * c2 + (c - c1)];
    }
}

__global__ __launch_bounds__(256) void k_upcat_grad(const float* __restrict__ dY, int N, int H, int W, int c1, int c2,
                                                    float* __restrict__ dcoarse, float* __restrict__ dskip) {
    const int C = c1 + c2, Ho = H / 2, Wo = W / 2;
    const int64_t n1 = (int64_t)N * Ho * Wo * c1, n2 = (int64_t)N * H * W * c2;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n1 + n2; i += (int64_t)gridDim.x * blockDim.x) {
        if (i < n1) {
            const int c = (int)(i % c1);
            int64_t t = i / c1;
            const int x = (int)(t % Wo);
            t /= Wo;
            const int y = (int)(t % Ho);
            const int n = (int)(t / Ho);
            const float* b = dY + (((int64_t)n * H + 2 * y) * W + 2 * x) * C + c;
            dcoarse[i] = b[0] + b[C] + b[(int64_t)W * C] + b[(int64_t)W * C + C];
        } else {
            const int64_t j = i - n1;
            const int c = (int)(j % c2);
            const int64_t p = j / c2;
            dskip[j] = dY[p * C + c1 + c];
        }
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_pack(const float* __restrict__ x, int64_t npix, int cin, int cinp,
                                              T* __restrict__ X) {
    const int64_t n = npix * cinp;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % cinp);
        const int64_t p = i / cinp;
        X[i] = fromf<T>(c < cin ? x[p * cin + c] : 0.f);
    }
}

__device__ __forceinline__ double wave_sum_d(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ y, const float* __restrict__ t,
                                              const float* __restrict__ w, int64_t npix, int cout, int coutp,
                                              float* __restrict__ G, double* __restrict__ loss) {
    double s = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += (int64_t)gridDim.x * blockDim.x) {
        const float wp = w[p];
        for (int c = 0; c < coutp; ++c) {
            float g = 0.f;
            if (c < cout) {
                const float d = y[p * cout + c] - t[p * cout + c];
                s += (double)wp * (double)d * (double)d;
                g = 2.f * wp * d / (float)cout;
            }
            G[p * coutp + c] = g;
        }
    }
    __shared__ double red[4];
    const double ws = wave_sum_d(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ws;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) b += red[k];
        atomicAdd(loss, b / (double)cout);
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_prep(const float* __restrict__ Wm, int cout, int cin, int coutp, int cinp,
                                              int taps, T* __restrict__ Wf, T* __restrict__ Wb) {
    const int64_t n = (int64_t)taps * coutp * cinp;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int ci = (int)(i % cinp);
        int64_t r = i / cinp;
        const int co = (int)(r % coutp);
        const int tap = (int)(r / coutp);
        const float v = (co < cout && ci < cin) ? Wm[((int64_t)co * cin + ci) * taps + tap] : 0.f;
        Wf[i] = fromf<T>(v);
        // backward: the transposed kernel with mirrored taps
        Wb[((int64_t)(taps - 1 - tap) * cinp + ci) * coutp + co] = fromf<T>(v);
    }
}

__global__ __launch_bounds__(256) void k_gather(const float* __restrict__ dWt, int cout, int cin, int coutp, int cinp,
                                                int taps, float* __restrict__ g) {
    const int64_t n = (int64_t)cout * cin * taps;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int tap = (int)(i % taps);
        const int64_t r = i / taps;
        const int ci = (int)(r % cin);
        const int co = (int)(r / cin);
        g[i] = dWt[((int64_t)tap * coutp + co) * cinp + ci];
    }
}

__global__ __launch_bounds__(256) void k_fill(float* __restrict__ p, int64_t n, float v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ __launch_bounds__(256) void k_fill_f64(double* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0.0;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                                              float bc1, float bc2) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
constexpr unsigned kMaxGrid = 65536;
inline unsigned grid_for(int64_t n) {
    const unsigned b = blocks_for(n);
    return b > kMaxGrid ? kMaxGrid : b;
}

template <class T>
struct L {
    static hipError_t conv(const void* X, const void* Wt, const float* bias, int N, int H, int W, int cin, int coutp,
                           int cstore, int taps, int relu, void* Y, float* yf, int accumulate, hipStream_t s) {
        const int64_t npix = (int64_t)N * H * W;
        const unsigned gx = blocks_for(npix, 128);
        if (coutp % 64 == 0)
            hipLaunchKernelGGL((k_conv<T, 2>), dim3(gx, coutp / 64), dim3(256), 0, s, (const T*)X, (const T*)Wt, bias,
                               N, H, W, cin, coutp, cstore, taps, relu, (T*)Y, yf, accumulate);
        else
            hipLaunchKernelGGL((k_conv<T, 1>), dim3(gx, coutp / 32), dim3(256), 0, s, (const T*)X, (const T*)Wt, bias,
                               N, H, W, cin, coutp, cstore, taps, relu, (T*)Y, yf, accumulate);
        return hipGetLastError();
    }
    static hipError_t wgrad(const void* X, const void* dZ, int N, int H, int W, int cin, int coutp, int taps,
                            float* dWt, hipStream_t s) {
        const int64_t npix = (int64_t)N * H * W;
        const int64_t nchunks = (npix + 15) / 16;
        const unsigned gy = (unsigned)(taps * (coutp / 32) * ((cin + 31) / 32));
        // about 2048 blocks in all, at least 16 chunks (4 per wave) per block
        int64_t want = 2048 / gy + 1;
        int64_t per = (nchunks + want - 1) / want;
        if (per < 16) per = 16;
        const unsigned gx = (unsigned)((nchunks + per - 1) / per);
        if (sizeof(T) == 2 && cin % 16 == 0 && coutp % 32 == 0 && (taps == 9 || taps == 1)) {
            // about 2048 blocks in all; a 3 x 3 kernel takes one block row per
            // row of taps (grid z)
            const unsigned gt = (unsigned)((coutp / 32) * ((cin + 31) / 32));
            const unsigned gz = taps == 9 ? 3u : 1u;
            int64_t want2 = 2048 / (gt * gz) + 1;
            int64_t per2 = (nchunks + want2 - 1) / want2;
            if (per2 < 16) per2 = 16;
            const unsigned gx2 = (unsigned)((nchunks + per2 - 1) / per2);
            if (taps == 9)
                hipLaunchKernelGGL((k_wgrad_lds<3>), dim3(gx2, gt, 3), dim3(256), 0, s, (const __bf16*)X,
                                   (const __bf16*)dZ, N, H, W, cin, coutp, per2, dWt);
            else
                hipLaunchKernelGGL((k_wgrad_lds<1>), dim3(gx2, gt, 1), dim3(256), 0, s, (const __bf16*)X,
                                   (const __bf16*)dZ, N, H, W, cin, coutp, per2, dWt);
        } else {
            hipLaunchKernelGGL((k_wgrad<T>), dim3(gx, gy), dim3(256), 0, s, (const T*)X, (const T*)dZ, N, H, W, cin,
                               coutp, taps, per, dWt);
        }
        return hipGetLastError();
    }
    static hipError_t bgrad(const void* dZ, int64_t npix, int coutp, int cout, float* db, hipStream_t s) {
        const int per = 256 / coutp;
        unsigned g = blocks_for(npix, per * 64);
        if (g > 1024) g = 1024;
        hipLaunchKernelGGL((k_bgrad<T>), dim3(g), dim3(256), 0, s, (const T*)dZ, npix, coutp, cout, db);
        return hipGetLastError();
    }
    static hipError_t act_grad(const float* G, const void* Y, int64_t n, int relu, void* dZ, hipStream_t s) {
        hipLaunchKernelGGL((k_act_grad<T>), dim3(grid_for(n)), dim3(256), 0, s, G, (const T*)Y, n, relu, (T*)dZ);
        return hipGetLastError();
    }
    static hipError_t pool(const void* X, int N, int H, int W, int C, void* Y, hipStream_t s) {
        hipLaunchKernelGGL((k_pool<T>), dim3(grid_for((int64_t)N * H * W * C / 4)), dim3(256), 0, s, (const T*)X, N, H,
                           W, C, (T*)Y);
        return hipGetLastError();
    }
    static hipError_t pool_grad(const float* dY, int N, int H, int W, int C, float* dX, hipStream_t s) {
        hipLaunchKernelGGL(k_pool_grad, dim3(grid_for((int64_t)N * H * W * C)), dim3(256), 0, s, dY, N, H, W, C, dX);
        return hipGetLastError();
    }
    static hipError_t upcat(const void* coarse, const void* skip, int N, int H, int W, int c1, int c2, void* Y,
                            hipStream_t s) {
        hipLaunchKernelGGL((k_upcat<T>), dim3(grid_for((int64_t)N * H * W * (c1 + c2))), dim3(256), 0, s,
                           (const T*)coarse, (const T*)skip, N, H, W, c1, c2, (T*)Y);
        return hipGetLastError();
    }
    static hipError_t upcat_grad(const float* dY, int N, int H, int W, int c1, int c2, float* dcoarse, float* dskip,
                                 hipStream_t s) {
        const int64_t n = (int64_t)N * (H / 2) * (W / 2) * c1 + (int64_t)N * H * W * c2;
        hipLaunchKernelGGL(k_upcat_grad, dim3(grid_for(n)), dim3(256), 0, s, dY, N, H, W, c1, c2, dcoarse, dskip);
        return hipGetLastError();
    }
    static hipError_t pack(const float* x, int64_t npix, int cin, int cinp, void* X, hipStream_t s) {
        hipLaunchKernelGGL((k_pack<T>), dim3(grid_for(npix * cinp)), dim3(256), 0, s, x, npix, cin, cinp, (T*)X);
        return hipGetLastError();
    }
    static hipError_t loss(const float* y, const float* t, const float* w, int64_t npix, int cout, int coutp, float* G,
                           double* lossp, hipStream_t s) {
        hipLaunchKernelGGL(k_loss, dim3(grid_for(npix)), dim3(256), 0, s, y, t, w, npix, cout, coutp, G, lossp);
        return hipGetLastError();
    }
    static hipError_t prep(const float* Wm, int cout, int cin, int coutp, int cinp, int taps, void* Wf, void* Wb,
                           hipStream_t s) {
        hipLaunchKernelGGL((k_prep<T>), dim3(grid_for((int64_t)taps * coutp * cinp)), dim3(256), 0, s, Wm, cout, cin,
                           coutp, cinp, taps, (T*)Wf, (T*)Wb);
        return hipGetLastError();
    }
    static hipError_t gather(const float* dWt, int cout, int cin, int coutp, int cinp, int taps, float* g,
                             hipStream_t s) {
        hipLaunchKernelGGL(k_gather, dim3(grid_for((int64_t)cout * cin * taps)), dim3(256), 0, s, dWt, cout, cin, coutp,
                           cinp, taps, g);
        return hipGetLastError();
    }
    static NnKernels set() {
        NnKernels k;
        k.conv = &conv;
        k.wgrad = &wgrad;
        k.bgrad = &bgrad;
        k.act_grad = &act_grad;
        k.pool = &pool;
        k.pool_grad = &pool_grad;
        k.upcat = &upcat;
        k.upcat_grad = &upcat_grad;
        k.pack = &pack;
        k.loss = &loss;
        k.prep = &prep;
        k.gather = &gather;
        k.elem_bytes = (int)sizeof(T);
        return k;
    }
};

}  // namespace

NnKernels nn_kernels_bf16() { return L<__bf16>::set(); }
NnKernels nn_kernels_f32() { return L<float>::set(); }

hipError_t nn_fill(float* p, int64_t n, float v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
hipError_t nn_fill_f64(double* p, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}
hipError_t nn_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                   float bc1, float bc2, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, s, w, g, m, v, n, lr, b1, b2, eps, bc1, bc2);
    return hipGetLastError();
}

}  // namespace nnk
