// Kernels of the learned closure: box filter, channel statistics, standardise,
// BF16-MFMA implicit-GEMM 3x3x3 periodic convolution (forward, backward-data,
// backward-weight), bias gradient, MSE, Adam, weight packing, guard.
//
// Activation layout: channel-last [batch][point][channel] (point = (z*n + y)*n + x),
// channel count padded to a multiple of 8 so 8 consecutive channels are one
// 16-byte load.  The contraction index of a convolution is kk = tap*Cpad + c with
// tap = (dz+1)*9 + (dy+1)*3 + (dx+1).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace sbli {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;

constexpr int kNetLayers = 3;

__device__ __forceinline__ float gelu_f(float v) { return 0.5f * v * (1.0f + erff(v * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float v) {
    return 0.5f * (1.0f + erff(v * 0.70710678118654752f)) + v * 0.39894228040143268f * expf(-0.5f * v * v);
}

__device__ __forceinline__ int wrapn(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// ---------------------------------------------------------------------------
// Box filter: separable centred trapezoid of width ratio*h (weights 1/(2 ratio)
// at +-ratio/2, 1/ratio in between), sampled at every ratio-th fine point.
// One thread per coarse output point and field.  With subtract != 0 the result
// is F(fine) - coarse (in place), e.g. F R_f - R_c for a closure target.
template <typename Tin>
__global__ void __launch_bounds__(256) box_filter_kernel(const Tin* __restrict__ fine, int nf, int nfields, int ratio,
                                                         float* __restrict__ coarse, int subtract) {
    const int nc = nf / ratio;
    const int64_t Pc = (int64_t)nc * nc * nc;
    const int64_t Pf = (int64_t)nf * nf * nf;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= Pc * nfields) return;
    const int f = (int)(id / Pc);
    const int64_t pc = id % Pc;
    const int xc = (int)(pc % nc), yc = (int)((pc / nc) % nc), zc = (int)(pc / ((int64_t)nc * nc));
    const int h = ratio / 2;
    const double wi = 1.0 / ratio, we = 0.5 / ratio;
    const Tin* src = fine + (int64_t)f * Pf;
    double acc = 0.0;
    for (int dz = -h; dz <= h; ++dz) {
        const double wz = (dz == -h || dz == h) ? we : wi;
        const int z = wrapn(zc * ratio + dz, nf);
        double accy = 0.0;
        for (int dy = -h; dy <= h; ++dy) {
            const double wy = (dy == -h || dy == h) ? we : wi;
            const int y = wrapn(yc * ratio + dy, nf);
            const Tin* row = src + ((int64_t)z * nf + y) * nf;
            double accx = 0.0;
            for (int dx = -h; dx <= h; ++dx) {
                const double wx = (dx == -h || dx == h) ? we : wi;
                accx += wx * (double)row[wrapn(xc * ratio + dx, nf)];
            }
            accy += wy * accx;
        }
        acc += wz * accy;
    }
    const int64_t o = (int64_t)f * Pc + pc;
    coarse[o] = subtract ? (float)(acc - (double)coarse[o]) : (float)acc;
}

// ---------------------------------------------------------------------------
// Per-channel mean, standard deviation (population statistics, FP64 sums) and
// largest magnitude of `count` planar [5][P] FP32 arrays.  One block per channel.
__global__ void __launch_bounds__(256) channel_stats_kernel(const float* __restrict__ data, int count, int64_t P,
                                                            float* __restrict__ mean_std /* [5] mean, [5] std */,
                                                            float* __restrict__ maxabs /* [5] */) {
    const int c = blockIdx.x;
    double s = 0.0, s2 = 0.0;
    float mx = 0.0f;
    for (int b = 0; b < count; ++b) {
        const float* src = data + ((int64_t)b * 5 + c) * P;
        for (int64_t i = threadIdx.x; i < P; i += blockDim.x) {
            const double v = src[i];
            s += v;
            s2 += v * v;
            mx = fmaxf(mx, fabsf(src[i]));
        }
    }
    __shared__ double ss[256], ss2[256];
    __shared__ float sm[256];
    ss[threadIdx.x] = s;
    ss2[threadIdx.x] = s2;
    sm[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            ss[threadIdx.x] += ss[threadIdx.x + w];
            ss2[threadIdx.x] += ss2[threadIdx.x + w];
            sm[threadIdx.x] = fmaxf(sm[threadIdx.x], sm[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double N = (double)count * (double)P;
        const double m = ss[0] / N;
        const double var = ss2[0] / N - m * m;
        mean_std[c] = (float)m;
        mean_std[5 + c] = (float)sqrt(var > 0.0 ? var : 0.0);
        maxabs[c] = sm[0];
    }
}

// Planar FP32 [B][5][P] -> standardised channel-last BF16 [B][P][8] (channels 5..7 zero).
__global__ void __launch_bounds__(256) standardize_kernel(const float* __restrict__ q, int64_t P, int B,
                                                          const float* __restrict__ mean_std,
                                                          __bf16* __restrict__ x) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)B * P) return;
    const int64_t b = id / P, p = id % P;
    bf16x8 v;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        float f = 0.0f;
        if (c < 5) f = (q[(b * 5 + c) * P + p] - mean_std[c]) / mean_std[5 + c];
        v[c] = (__bf16)f;
    }
    *(bf16x8*)(x + id * 8) = v;
}

// Network output y [B][P][8] (standardised) -> closure term planar [B][5][P].
__global__ void __launch_bounds__(256) destandardize_kernel(const float* __restrict__ y, int64_t P, int B,
                                                            const float* __restrict__ mean_std,
                                                            float* __restrict__ out) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)B * P) return;
    const int64_t b = id / P, p = id % P;
#pragma unroll
    for (int c = 0; c < 5; ++c) out[(b * 5 + c) * P + p] = y[id * 8 + c] * mean_std[5 + c] + mean_std[c];
}

// Box mean of every (sample, field) plane of a planar [B][5][P] array, removed
// in place: the closure term then adds nothing to the box totals of mass,
// momentum and energy, as the exact closure term does (both residuals are
// conservative and the filter keeps totals).  Three steps, each in a fixed
// order, so the result is deterministic: FP64 partial sums of kBoxMeanChunk
// points per workgroup, one mean per (sample, field), the subtraction.
constexpr int kBoxMeanChunk = 4096;
__global__ void __launch_bounds__(256) box_mean_partial_kernel(const float* __restrict__ a, int64_t P, int nchunks,
                                                               double* __restrict__ part) {
    // one workgroup per (sample * 5 + field, chunk), chunks fastest
    const int chunk = (int)(blockIdx.x % (unsigned)nchunks);
    const int64_t bf = blockIdx.x / (unsigned)nchunks;
    const float* src = a + bf * P;
    const int64_t lo = (int64_t)chunk * kBoxMeanChunk;
    const int64_t hi = lo + kBoxMeanChunk < P ? lo + kBoxMeanChunk : P;
    double s = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) s += (double)src[i];
    __shared__ double ss[256];
    ss[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) ss[threadIdx.x] += ss[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[bf * nchunks + chunk] = ss[0];
}
// one thread per (sample, field): the partials in chunk order
__global__ void __launch_bounds__(64) box_mean_final_kernel(const double* __restrict__ part, int nchunks, int nbf,
                                                            int64_t P, float* __restrict__ mean) {
    const int bf = blockIdx.x * blockDim.x + threadIdx.x;
    if (bf >= nbf) return;
    double s = 0.0;
    for (int k = 0; k < nchunks; ++k) s += part[(int64_t)bf * nchunks + k];
    mean[bf] = (float)(s / (double)P);
}
__global__ void __launch_bounds__(256) box_mean_subtract_kernel(float* __restrict__ a, int64_t P, int nbf,
                                                                const float* __restrict__ mean) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)nbf * P) return;
    a[id] -= mean[id / P];
}

// ---------------------------------------------------------------------------
// Implicit-GEMM convolution on MFMA (v_mfma_f32_32x32x16_bf16).
//   out[b][p][o] = sum_kk W[o][kk] * in[b][p + off(tap(kk))][c(kk)]
// A wave computes 2 tiles of 32 points x 32 output channels.  A operand
// (points x 16 kk): each lane reads 8 consecutive channels of one tap at one
// point (16 bytes); B operand (16 kk x 32 outputs): 8 consecutive kk of one
// output channel (16 bytes) from the packed weights Wp[32][Kpad].
// Epilogues:
//   kEpiGelu   : v = acc + bias; pre[..][o] = v (FP32, 32 ch); act[..][o] = bf16(gelu v)
//   kEpiLinear : v = acc + bias; y[..][o] = v (FP32, ostride ch) for o < ocount
//   kEpiDGelu  : v = acc * gelu'(pre[..][o]); act[..][o] = bf16(v) (32 ch)
//   kEpiData   : out[..][o] = acc (FP32, 32 ch)
enum { kEpiGelu = 0, kEpiLinear = 1, kEpiDGelu = 2, kEpiData = 3 };

// The input is staged in LDS (grids with n % 32 == 0).  A workgroup owns 32
// x-points x 8 y-rows of one z-plane of one sample (256 points; wave w takes
// rows 2w and 2w + 1 as its two 32-point M tiles).  The
// 34 x 10 x 3 input points it reads (periodic halo of one point) are loaded
// once into LDS and every one of the 27 taps reads its A operands from there,
// instead of from global memory 27 times.  LDS point stride: cpad + 8 channels
// for cpad = 32 (80 bytes: eight lanes' 16-byte reads fall in distinct banks),
// cpad for cpad = 8.
constexpr int kConvTx = 32, kConvTy = 8;
constexpr int kConvHx = kConvTx + 2, kConvHy = kConvTy + 2;

template <int EPI, int CPAD>
__global__ void __launch_bounds__(256) conv_mfma_lds_kernel(const __bf16* __restrict__ in, const __bf16* __restrict__ Wp,
                                                            int Kpad, const float* __restrict__ bias, int n,
                                                            float* __restrict__ fout, __bf16* __restrict__ bout,
                                                            const float* __restrict__ pre_in, int ocount, int ostride) {
    constexpr int LS = CPAD == 32 ? 40 : CPAD;                 // LDS point stride (elements)
    __shared__ __attribute__((aligned(16))) __bf16 sx[3 * kConvHy * kConvHx * LS];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int row = lane & 31, half = lane >> 5;
    const int64_t P = (int64_t)n * n * n;
    // tile -> (sample, z, y0, x0)
    const int tx = n / kConvTx, ty = n / kConvTy;
    int t = blockIdx.x;
    const int x0 = (t % tx) * kConvTx;
    t /= tx;
    const int y0 = (t % ty) * kConvTy;
    t /= ty;
    const int z = t % n;
    const int64_t b = t / n;
    const __bf16* inb = in + b * P * CPAD;
    // stage the halo box: 3 x 10 x 34 points, CPAD / 8 16-byte loads each.  A
    // thread issues all of its loads before its first LDS store, so their
    // latencies overlap instead of adding up.
    constexpr int G = CPAD / 8;
    constexpr int NS = 3 * kConvHy * kConvHx * G;
    constexpr int IT = (NS + 255) / 256;
    bf16x8 sv[IT];
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        const int i = threadIdx.x + 256 * k;
        if (i < NS) {
            const int g = i % G;
            const int pt = i / G;
            const int hx = pt % kConvHx, hy = (pt / kConvHx) % kConvHy, hz = pt / (kConvHx * kConvHy);
            const int gx = wrapn(x0 + hx - 1, n), gy = wrapn(y0 + hy - 1, n), gz = wrapn(z + hz - 1, n);
            sv[k] = *(const bf16x8*)(inb + (((int64_t)gz * n + gy) * n + gx) * CPAD + g * 8);
        }
    }
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        const int i = threadIdx.x + 256 * k;
        if (i < NS) *(bf16x8*)(&sx[(i / G) * LS + (i % G) * 8]) = sv[k];
    }
    __syncthreads();
    floatx16 acc0 = {0}, acc1 = {0};
    const __bf16* wrow = Wp + (int64_t)row * Kpad;
    const int ry0 = 2 * wave;                             // tile rows ry0, ry0 + 1 of the two M tiles
    const int lbase = ry0 * kConvHx + row;                // this lane's point in the halo box, tap (0, 0, 0)
    // halo-box offset of tap t (dz, dy, dx = t / 9, (t / 3) % 3, t % 3)
    auto tap_off = [](int t) { return ((t / 9) * kConvHy + (t / 3) % 3) * kConvHx + t % 3; };
    // The K loop runs over the packed width round_up(27 * CPAD, 16) (the value of
    // Kpad) and is unrolled completely, so every tap offset is a constant: a step
    // of 16 kk is one tap (channels c0 .. c0 + 15) for CPAD = 32, two taps (one
    // per half-wave) for CPAD = 8.
    constexpr int KP = (27 * CPAD + 15) / 16 * 16;
    // the backward-data epilogue's pre-activations are requested before the K
    // loop, so their latency is spent under the MFMAs
    float pre[2][16];
    if constexpr (EPI == kEpiDGelu) {
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            const int y = y0 + 2 * wave + tt;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int m = (j / 4) * 8 + half * 4 + (j & 3);
                const int64_t g = b * P + ((int64_t)z * n + y) * n + x0 + m;
                pre[tt][j] = pre_in[g * 32 + row];
            }
        }
    }
#pragma unroll
    for (int k0 = 0; k0 < KP; k0 += 16) {
        const bf16x8 bv = *(const bf16x8*)(wrow + k0 + half * 8);
        bf16x8 a0, a1;
        const bool valid = CPAD == 32 || k0 / CPAD + half < 27;
        if (valid) {
            int po, c;
            if constexpr (CPAD == 32) {
                po = tap_off(k0 / 32);
                c = k0 % 32 + half * 8;
            } else {
                po = half ? tap_off(k0 / CPAD + 1) : tap_off(k0 / CPAD);
                c = 0;
            }
            const int p0 = lbase + po;
            const int p1 = p0 + kConvHx;                  // next row
            a0 = *(const bf16x8*)(&sx[p0 * LS + c]);
            a1 = *(const bf16x8*)(&sx[p1 * LS + c]);
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) { a0[j] = (__bf16)0.0f; a1[j] = (__bf16)0.0f; }
        }
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, bv, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, bv, acc1, 0, 0, 0);
    }
    // D[m][o]: o = lane & 31, m = (j / 4) * 8 + (lane >> 5) * 4 + (j & 3); m = x within the row
    const int o = row;
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
        const floatx16 acc = tt == 0 ? acc0 : acc1;
        const int y = y0 + 2 * wave + tt;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int m = (j / 4) * 8 + half * 4 + (j & 3);
            const int64_t g = b * P + ((int64_t)z * n + y) * n + x0 + m;
            if (EPI == kEpiGelu) {
                const float v = acc[j] + bias[o];
                fout[g * 32 + o] = v;
                bout[g * 32 + o] = (__bf16)gelu_f(v);
            } else if (EPI == kEpiLinear) {
                if (o < ocount) fout[g * ostride + o] = acc[j] + bias[o];
            } else if (EPI == kEpiData) {
                fout[g * 32 + o] = acc[j];
            } else {
                bout[g * 32 + o] = (__bf16)(acc[j] * gelu_grad_f(pre[tt][j]));
            }
        }
    }
}

// Element-wise GELU backward: dx = bf16(g * gelu'(pre)), the arithmetic of the
// kEpiDGelu epilogue.
__global__ void __launch_bounds__(256) gelu_bwd_kernel(const float* __restrict__ g, const float* __restrict__ pre,
                                                       int64_t count, __bf16* __restrict__ dx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dx[i] = (__bf16)(g[i] * gelu_grad_f(pre[i]));
}

// ---------------------------------------------------------------------------
// Weight gradient on MFMA:  dW[o][kk] = sum_p dout[p][o] * in[p + off(tap)][c]
// (o < 32 rows, kk < Kpad32 columns).  A workgroup takes blocks of 32
// consecutive x-points of one (b, y, z) row (n % 32 == 0).  Per block it stages
// in LDS, transposed so the reduction over points is contiguous:
//   sd[o][32]                       dout of the block
//   si[tap][c][32]                  input shifted by each of the 27 taps
// then each wave accumulates its share of the Kpad32/32 column tiles.
// A staging thread loads 8 channels of 10 consecutive points of one (dz, dy)
// row (ten 16-byte loads: 8 points and one on each side), and for each of the
// three x-shifts transposes an 8 x 8 block in registers and stores 8 points of
// one channel per 16-byte LDS store; each input element is loaded once per
// (dz, dy) instead of once per tap.  LDS rows are padded to 40 elements (80 bytes)
// so that rows 8 or 32 apart, and the 32 rows one MFMA operand read spans, do
// not fall on the same banks.
// Results: per-workgroup partial sums part[wg][32][Kpad32] (FP32).
constexpr int kWgradMaxTiles = 28;   // Kpad32 / 32 <= 28 (27 * 32 = 864)
constexpr int kWgradRow = 40;        // LDS row length (elements) of sd and si

// o[j][k] = r[k][j]: the 8 x 8 block of 16-bit elements transposed.
__device__ __forceinline__ void transpose8x8(const bf16x8 (&r)[8], bf16x8 (&o)[8]) {
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int k = 0; k < 8; ++k) o[j][k] = r[k][j];
}

__global__ void __launch_bounds__(256) conv_wgrad_kernel(const __bf16* __restrict__ in, int cpad,
                                                         const __bf16* __restrict__ dout, int opad, int n,
                                                         int64_t nblocks, int Kpad32, float* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) __bf16 sd[32][kWgradRow];
    __shared__ __attribute__((aligned(16))) __bf16 si[27 * 32][kWgradRow];   // [(tap * cpad + c)][point]
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int row = lane & 31, half = lane >> 5;
    const int ntiles = Kpad32 / 32;
    const int nrows = n / 32;            // 32-point blocks per x-row
    const int64_t P = (int64_t)n * n * n;
    floatx16 acc[7];
#pragma unroll
    for (int i = 0; i < 7; ++i)
        for (int j = 0; j < 16; ++j) acc[i][j] = 0.0f;
    const int64_t per = (nblocks + gridDim.x - 1) / gridDim.x;
    const int64_t blk0 = (int64_t)blockIdx.x * per;
    const int64_t blk1 = blk0 + per < nblocks ? blk0 + per : nblocks;
    for (int64_t blk = blk0; blk < blk1; ++blk) {
        // decode block -> (b, z, y, x0)
        const int xb = (int)(blk % nrows);
        const int64_t r = blk / nrows;
        const int y = (int)(r % n);
        const int z = (int)((r / n) % n);
        const int64_t b = r / ((int64_t)n * n);
        const int x0 = xb * 32;
        __syncthreads();   // previous block's LDS reads are done
        // stage dout: 32 points x opad channels, 8 points x 8 channels per thread
        for (int t = threadIdx.x; t < 4 * (opad / 8); t += blockDim.x) {
            const int pg = t % 4, cg = t / 4;
            const int64_t g = b * P + ((int64_t)z * n + y) * n + x0 + pg * 8;
            bf16x8 r[8], o[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) r[k] = *(const bf16x8*)(dout + (g + k) * opad + cg * 8);
            transpose8x8(r, o);
#pragma unroll
            for (int j = 0; j < 8; ++j) *(bf16x8*)(&sd[cg * 8 + j][pg * 8]) = o[j];
        }
        for (int t = threadIdx.x; t < (32 - opad) * 4; t += blockDim.x) {
            bf16x8 zero;
#pragma unroll
            for (int j = 0; j < 8; ++j) zero[j] = (__bf16)0.0f;
            *(bf16x8*)(&sd[opad + t / 4][(t % 4) * 8]) = zero;
        }
        // stage the input for every tap: one (dz, dy) row segment per thread item
        for (int t = threadIdx.x; t < 9 * 4 * (cpad / 8); t += blockDim.x) {
            const int pg = t % 4;
            const int rest = t / 4;
            const int cg = rest % (cpad / 8);
            const int zy = rest / (cpad / 8);              // (dz + 1) * 3 + (dy + 1)
            const int dz = zy / 3 - 1, dy = zy % 3 - 1;
            const int64_t row = b * P + ((int64_t)wrapn(z + dz, n) * n + wrapn(y + dy, n)) * n;
            bf16x8 r[10];
#pragma unroll
            for (int k = 0; k < 10; ++k)
                r[k] = *(const bf16x8*)(in + (row + wrapn(x0 + pg * 8 + k - 1, n)) * cpad + cg * 8);
#pragma unroll
            for (int sx = 0; sx < 3; ++sx) {                // dx = sx - 1
                const int tap = zy * 3 + sx;
                bf16x8 blk[8], o[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) blk[k] = r[k + sx];
                transpose8x8(blk, o);
#pragma unroll
                for (int j = 0; j < 8; ++j) *(bf16x8*)(&si[tap * cpad + cg * 8 + j][pg * 8]) = o[j];
            }
        }
        __syncthreads();
        // A[o][pts] from sd, B[pts][kk] from si; two k-steps of 16 points
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const bf16x8 av = *(const bf16x8*)(&sd[row][ks * 16 + half * 8]);
#pragma unroll
            for (int i = 0; i < 7; ++i) {
                const int tile = wave + 4 * i;
                if (tile < ntiles) {
                    const int kk = tile * 32 + row;
                    bf16x8 bv;
                    if (kk < 27 * cpad) {
                        bv = *(const bf16x8*)(&si[kk][ks * 16 + half * 8]);
                    } else {
#pragma unroll
                        for (int j = 0; j < 8; ++j) bv[j] = (__bf16)0.0f;
                    }
                    acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[i], 0, 0, 0);
                }
            }
        }
    }
    // D[o][kk]: kk = tile*32 + (lane & 31), o = (j/4)*8 + half*4 + (j&3)
    float* dst = part + (int64_t)blockIdx.x * 32 * Kpad32;
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        const int tile = wave + 4 * i;
        if (tile >= ntiles) continue;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int o = (j / 4) * 8 + half * 4 + (j & 3);
            dst[(int64_t)o * Kpad32 + tile * 32 + row] = acc[i][j];
        }
    }
}

// Sums the per-workgroup partials in a fixed order and writes the gradient of
// a layer in the master layout dW[o][c][tap] (o < cout, c < cin).
__global__ void __launch_bounds__(256) wgrad_reduce_kernel(const float* __restrict__ part, int nwg, int Kpad32,
                                                           int cpad, int cin, int cout, float* __restrict__ dW) {
    // one thread per (o, kk), kk = tap * cpad + c fastest, so the partial rows
    // are read contiguously.  Four interleaved accumulators (partials w = 4i + j
    // into s_j) keep four loads in flight; they are combined in a fixed order,
    // so the result is deterministic.
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    const int kk = id % Kpad32;
    const int o = id / Kpad32;
    if (o >= cout) return;
    const int tap = kk / cpad, c = kk % cpad;
    if (tap >= 27 || c >= cin) return;
    const float* p = part + (int64_t)o * Kpad32 + kk;
    const int64_t stride = (int64_t)32 * Kpad32;
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
    int w = 0;
    // unrolled so that many partials are in flight; each s_j still adds its
    // partials in order of w
#pragma unroll 8
    for (; w + 4 <= nwg; w += 4) {
        s0 += p[(w + 0) * stride];
        s1 += p[(w + 1) * stride];
        s2 += p[(w + 2) * stride];
        s3 += p[(w + 3) * stride];
    }
    for (; w < nwg; ++w) s0 += p[w * stride];
    dW[(o * cin + c) * 27 + tap] = (s0 + s1) + (s2 + s3);
}

// Bias gradient db[o] = sum_p dout[p][o], in two deterministic passes.
// Pass 1: workgroup w sums points [w * chunk, (w + 1) * chunk) into
// part[w][32]; each thread reads 8 channels of a point with one 16-byte load
// (opad / 8 threads per point, 256 / (opad / 8) point lanes), and the point
// lanes are combined in LDS in a fixed order.
constexpr int kBiasWg = 512;
__global__ void __launch_bounds__(256) bias_grad_kernel(const __bf16* __restrict__ dout, int opad, int64_t npts,
                                                        float* __restrict__ part) {
    const int groups = opad / 8;                     // 1 or 4
    const int cg = threadIdx.x % groups, pl = threadIdx.x / groups;
    const int lanes = 256 / groups;
    const int64_t chunk = (npts + gridDim.x - 1) / gridDim.x;
    const int64_t p0 = (int64_t)blockIdx.x * chunk;
    const int64_t p1 = p0 + chunk < npts ? p0 + chunk : npts;
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t p = p0 + pl; p < p1; p += lanes) {
        const bf16x8 v = *(const bf16x8*)(dout + p * opad + cg * 8);
#pragma unroll
        for (int j = 0; j < 8; ++j) s[j] += (float)v[j];
    }
    __shared__ float ss[256][9];
#pragma unroll
    for (int j = 0; j < 8; ++j) ss[threadIdx.x][j] = s[j];
    __syncthreads();
    if ((int)threadIdx.x < opad) {
        const int c = threadIdx.x, g = c / 8, j = c % 8;
        float t = 0.0f;
        for (int l = 0; l < lanes; ++l) t += ss[l * groups + g][j];
        part[blockIdx.x * 32 + c] = t;
    }
}

// Pass 2: 256 threads = 32 channels x 8 slices; slice k sums partials
// w = k, k + 8, ...; the slices are combined in order.
__global__ void __launch_bounds__(256) bias_grad_final_kernel(const float* __restrict__ part, int nwg, int cout,
                                                              float* __restrict__ db) {
    const int o = threadIdx.x & 31, k = threadIdx.x >> 5;
    float s = 0.0f;
#pragma unroll 8
    for (int w = k; w < nwg; w += 8) s += part[w * 32 + o];   // in order of w
    __shared__ float ss[8][32];
    ss[k][o] = s;
    __syncthreads();
    if ((int)threadIdx.x < cout) {
        float t = 0.0f;
        for (int j = 0; j < 8; ++j) t += ss[j][threadIdx.x];
        db[threadIdx.x] = t;
    }
}

// MSE between the network output y [B][P][8] (5 used) and the standardised
// target (planar [B][5][P], standardised here): loss partial sums per block and
// the BF16 gradient dy = 2 (y - t) / (5 B P) into [B][P][8].
__global__ void __launch_bounds__(256) mse_grad_kernel(const float* __restrict__ y, const float* __restrict__ target,
                                                       int64_t P, int B, const float* __restrict__ mean_std,
                                                       __bf16* __restrict__ dy, double* __restrict__ loss_part) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double scale = 2.0 / (5.0 * (double)B * (double)P);
    double s = 0.0;
    if (id < (int64_t)B * P) {
        const int64_t b = id / P, p = id % P;
        bf16x8 g;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            float gv = 0.0f;
            if (c < 5) {
                const float t = (target[(b * 5 + c) * P + p] - mean_std[c]) / mean_std[5 + c];
                const float d = y[id * 8 + c] - t;
                s += (double)d * d;
                gv = (float)(scale * d);
            }
            g[c] = (__bf16)gv;
        }
        *(bf16x8*)(dy + id * 8) = g;
    }
    __shared__ double ss[256];
    ss[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) ss[threadIdx.x] += ss[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = ss[0];
}

__global__ void __launch_bounds__(256) sum_doubles_kernel(const double* __restrict__ part, int n, double scale,
                                                          double* __restrict__ out) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
    __shared__ double ss[256];
    ss[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) ss[threadIdx.x] += ss[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = ss[0] * scale;
}

// Adam (Kingma & Ba) on a flat FP32 parameter vector; step t >= 1.
__global__ void __launch_bounds__(256) adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v, int n, float lr,
                                                   float beta1, float beta2, float eps, int t) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.0f - powf(beta1, (float)t));
    const float vh = vi / (1.0f - powf(beta2, (float)t));
    p[i] -= lr * mh / (sqrtf(vh) + eps);
}

// Packs one layer's master weights W[o][c][tap] (FP32) into the MFMA layouts:
//   Wf[o][tap*cpad + c]  (32 x Kf, forward),  Wb[c][tap'*opad + o] (32 x Kb,
//   backward-data, tap' = 26 - tap mirrors the offset).  Padding entries are 0.
__global__ void __launch_bounds__(256) pack_weights_kernel(const float* __restrict__ W, int cin, int cout, int cpad,
                                                           int opad, int Kf, int Kb, __bf16* __restrict__ Wf,
                                                           __bf16* __restrict__ Wb) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (Wf != nullptr && id < 32 * Kf) {
        const int o = id / Kf, kk = id % Kf;
        const int tap = kk / cpad, c = kk % cpad;
        float v = 0.0f;
        if (o < cout && tap < 27 && c < cin) v = W[(o * cin + c) * 27 + tap];
        Wf[id] = (__bf16)v;
    }
    if (Wb != nullptr && id < 32 * Kb) {
        const int c = id / Kb, kk = id % Kb;
        const int tapm = kk / opad, o = kk % opad;
        float v = 0.0f;
        if (c < cin && tapm < 27 && o < cout) v = W[(o * cin + c) * 27 + (26 - tapm)];
        Wb[id] = (__bf16)v;
    }
}

// Closure guard: flag[0] = 1 if every closure value is finite and within
// +-limit[f] for its field, else 0; counters[0|1] count accepted / rejected.
__global__ void __launch_bounds__(1024) closure_guard_kernel(const float* __restrict__ C, int64_t P,
                                                             const float* __restrict__ limit, int* __restrict__ flag,
                                                             unsigned* __restrict__ counters) {
    int bad = 0;
    for (int f = 0; f < 5; ++f) {
        const float L = limit[f];
        for (int64_t i = threadIdx.x; i < P; i += blockDim.x) {
            const float v = C[(int64_t)f * P + i];
            bad |= !(fabsf(v) <= L);
        }
    }
    __shared__ int sb[1024];
    sb[threadIdx.x] = bad;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sb[threadIdx.x] |= sb[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        flag[0] = sb[0] ? 0 : 1;
        atomicAdd(&counters[sb[0] ? 1 : 0], 1u);
    }
}

}  // namespace sbli
