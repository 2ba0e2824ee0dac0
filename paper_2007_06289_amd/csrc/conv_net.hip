// Learned residual correction applied after the reconstruction: 3x3 convolutions (zero
// padding 1) with 1 or 16 channels, as implicit GEMMs on the matrix cores (BF16 operands, FP32
// accumulation, v_mfma_f32_16x16x32_bf16), plus FP32 weight gradients.
//
// Activations with 16 channels are stored BF16, NHWC ([b][y][x][c], 32 bytes per pixel);
// single-channel images are FP32 [b][y][x].  A wave computes 16 consecutive pixels of one row
// x 16 output channels: out[p][n] = sum_kk A[p][kk] Wg[kk][n], kk = tap * CIN + ci (tap =
// 3 (dy + 1) + dx + 1), in steps of 32 kk.  Operand layouts of the 16x16x32 instruction: lane l
// holds A[l % 16][8 (l / 16) .. + 7] and B[8 (l / 16) .. + 7][l % 16]; the result C[4 (l / 16) +
// i][l % 16] for i < 4.  The backward convolution with respect to the input is the same kernel
// with the weights transposed and the taps flipped (packed by cnn_pack_kernel), and its output
// multiplied by the ReLU mask of the layer below.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fhtfbp_internal.h"

namespace fhtfbp {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ uint16_t f2bf(float f) {   // round to nearest even
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16) | ((u & 0xffff) ? 0x40 : 0);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Packs FP32 weights w[cout][cin][9] into the B operand order of the kernel:
// packed[step][lane][j] = Wg[32 step + 8 (lane / 16) + j][lane % 16].  transpose_flip: pack the
// weights of the input-gradient convolution, Wg'[tap][co' = ci][ci' = co] = w[co][ci][8 - tap].
__global__ void cnn_pack_kernel(const float* __restrict__ w, uint16_t* __restrict__ packed,
                                int cin, int cout, int transpose_flip, int steps) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= steps * 64 * 8) return;
  const int j = e & 7, lane = (e >> 3) & 63, step = e >> 9;
  const int n = lane & 15, kk = step * 32 + (lane >> 4) * 8 + j;
  // geometry of the convolution being packed (after the transpose for the backward one)
  const int ci_n = transpose_flip ? cout : cin;    // its input channels
  const int co_n = transpose_flip ? cin : cout;    // its output channels
  float v = 0.f;
  if (kk < 9 * ci_n && n < co_n) {
    const int tap = kk / ci_n, c = kk % ci_n;
    if (!transpose_flip) v = w[(n * cin + c) * 9 + tap];
    else v = w[(c * cin + n) * 9 + (8 - tap)];
  }
  packed[e] = f2bf(v);
}

// CIN in {1, 16} input channels (FP32 image if 1, BF16 NHWC if 16); COUT in {1, 16}.
// COUT == 16: out16 (BF16 NHWC) = [relu](acc + bias) [* (mask > 0)].
// COUT == 1: out32 (FP32) = acc + bias [+ resid].
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) cnn_conv_kernel(const float* __restrict__ in32,
                                                       const uint16_t* __restrict__ in16,
                                                       const bf16x8* __restrict__ wop,
                                                       const float* __restrict__ bias,
                                                       const uint16_t* __restrict__ mask,
                                                       const float* __restrict__ resid,
                                                       uint16_t* __restrict__ out16,
                                                       float* __restrict__ out32, int relu, int H,
                                                       int W, long long groups) {
  constexpr int STEPS = (9 * CIN + 31) / 32;
  const int lane = threadIdx.x & 63;
  const long long gi = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);   // 16-pixel group
  if (gi >= groups) return;
  const int gpr = W >> 4;
  const int xg = (int)(gi % gpr);
  const long long by = gi / gpr;
  const int y = (int)(by % H);
  const int b = (int)(by / H);
  const int m = lane & 15, kg = lane >> 4;
  const int x = (xg << 4) + m;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int step = 0; step < STEPS; ++step) {
    bf16x8 a;
    if constexpr (CIN == 16) {
      const int kk0 = step * 32 + kg * 8;
      const int tap = kk0 >> 4, c0 = kk0 & 15;
      const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
      if (tap < 9 && yy >= 0 && yy < H && xx >= 0 && xx < W) {
        a = *reinterpret_cast<const bf16x8*>(in16 + (((size_t)b * H + yy) * W + xx) * 16 + c0);
      } else {
        a = bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
      }
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int tap = kg * 8 + j;
        const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
        float v = 0.f;
        if (tap < 9 && yy >= 0 && yy < H && xx >= 0 && xx < W) v = in32[((size_t)b * H + yy) * W + xx];
        a[j] = (short)f2bf(v);
      }
    }
    const bf16x8 bw = wop[step * 64 + lane];
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw, acc, 0, 0, 0);
  }
  const int n = lane & 15;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int px = (xg << 4) + 4 * kg + i;
    const size_t pix = ((size_t)b * H + y) * W + px;
    float v = acc[i] + (bias ? bias[n < COUT ? n : 0] : 0.f);
    if constexpr (COUT == 16) {
      if (relu) v = fmaxf(v, 0.f);
      if (mask && !(bf2f(mask[pix * 16 + n]) > 0.f)) v = 0.f;
      out16[pix * 16 + n] = f2bf(v);
    } else {
      if (n == 0) out32[pix] = v + (resid ? resid[pix] : 0.f);
    }
  }
}

// Weight and bias gradients of a convolution in the forward convention
// out[p][co] = sum_{ci, tap} w[co][ci][tap] in[p + off(tap)][ci]:
//   dw[co][ci][tap] = sum_p dz[p][co] in[p + off(tap)][ci],   db[co] = sum_p dz[p][co].
// dz has COUT channels (FP32 image if 1, BF16 NHWC if 16); in has CIN channels (same rule).
// Each block covers `rows` image rows x 64 columns of one slice and writes its sums to
// partial[block][COUT * CIN * 9 + COUT].
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) cnn_wgrad_kernel(const float* __restrict__ dz32,
                                                        const uint16_t* __restrict__ dz16,
                                                        const float* __restrict__ in32,
                                                        const uint16_t* __restrict__ in16,
                                                        float* __restrict__ partial, int H, int W,
                                                        int rows) {
  constexpr int NW = COUT * CIN * 9;
  constexpr int NOUT = NW + COUT;
  constexpr int XS = 64;
  __shared__ float sdz[XS][COUT];
  __shared__ float sin_[3][XS + 2][CIN];
  const int cols = W / XS;
  const int rb = blockIdx.x % ((H + rows - 1) / rows);
  const int rest = blockIdx.x / ((H + rows - 1) / rows);
  const int cb = rest % cols, b = rest / cols;
  const int x0 = cb * XS;
  float acc[(NOUT + 255) / 256];
#pragma unroll
  for (int k = 0; k < (NOUT + 255) / 256; ++k) acc[k] = 0.f;
  for (int y = rb * rows; y < min(H, (rb + 1) * rows); ++y) {
    __syncthreads();
    for (int e = threadIdx.x; e < XS * COUT; e += blockDim.x) {
      const int xx = e / COUT, c = e % COUT;
      const size_t pix = ((size_t)b * H + y) * W + x0 + xx;
      sdz[xx][c] = (COUT == 16) ? bf2f(dz16[pix * 16 + c]) : dz32[pix];
    }
    for (int e = threadIdx.x; e < 3 * (XS + 2) * CIN; e += blockDim.x) {
      const int r = e / ((XS + 2) * CIN), rem = e % ((XS + 2) * CIN);
      const int xx = rem / CIN, c = rem % CIN;
      const int yy = y + r - 1, gx = x0 + xx - 1;
      float v = 0.f;
      if (yy >= 0 && yy < H && gx >= 0 && gx < W) {
        const size_t pix = ((size_t)b * H + yy) * W + gx;
        v = (CIN == 16) ? bf2f(in16[pix * 16 + c]) : in32[pix];
      }
      sin_[r][xx][c] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < (NOUT + 255) / 256; ++k) {
      const int o = threadIdx.x + k * 256;
      if (o < NW) {
        const int co = o / (CIN * 9), ci = (o / 9) % CIN, tap = o % 9;
        const int dy = tap / 3, dx = tap % 3;
        float s = acc[k];
        for (int xx = 0; xx < XS; ++xx) s = fmaf(sdz[xx][co], sin_[dy][xx + dx][ci], s);
        acc[k] = s;
      } else if (o < NOUT) {
        const int co = o - NW;
        float s = acc[k];
        for (int xx = 0; xx < XS; ++xx) s += sdz[xx][co];
        acc[k] = s;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < (NOUT + 255) / 256; ++k) {
    const int o = threadIdx.x + k * 256;
    if (o < NOUT) partial[(size_t)blockIdx.x * NOUT + o] = acc[k];
  }
}

// out[o] = sum over blocks of partial[block][o], fixed order, accumulated in double.
__global__ void __launch_bounds__(256) cnn_reduce_kernel(const float* __restrict__ partial,
                                                         float* __restrict__ out, int blocks,
                                                         int nout) {
  __shared__ double sh[256];
  const int o = blockIdx.x;
  double s = 0.0;
  for (int blk = threadIdx.x; blk < blocks; blk += blockDim.x) s += partial[(size_t)blk * nout + o];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[o] = (float)sh[0];
}

}  // namespace

hipError_t launch_cnn_pack(const float* w, uint16_t* packed, int cin, int cout, int transpose_flip,
                           hipStream_t stream) {
  const int cin_n = transpose_flip ? cout : cin;
  const int steps = (9 * cin_n + 31) / 32;
  const int total = steps * 64 * 8;
  hipLaunchKernelGGL(cnn_pack_kernel, dim3((total + 255) / 256), dim3(256), 0, stream, w, packed,
                     cin, cout, transpose_flip, steps);
  return hipGetLastError();
}

hipError_t launch_cnn_conv(int cin, int cout, const float* in32, const uint16_t* in16,
                           const uint16_t* wop, const float* bias, const uint16_t* mask,
                           const float* resid, uint16_t* out16, float* out32, int relu, int batch,
                           int H, int W, hipStream_t stream) {
  const long long groups = (long long)batch * H * (W / 16);
  const dim3 grid((unsigned)((groups + 3) / 4));
  const bf16x8* w8 = reinterpret_cast<const bf16x8*>(wop);
  if (cin == 1 && cout == 16)
    hipLaunchKernelGGL((cnn_conv_kernel<1, 16>), grid, dim3(256), 0, stream, in32, in16, w8, bias,
                       mask, resid, out16, out32, relu, H, W, groups);
  else if (cin == 16 && cout == 16)
    hipLaunchKernelGGL((cnn_conv_kernel<16, 16>), grid, dim3(256), 0, stream, in32, in16, w8,
                       bias, mask, resid, out16, out32, relu, H, W, groups);
  else if (cin == 16 && cout == 1)
    hipLaunchKernelGGL((cnn_conv_kernel<16, 1>), grid, dim3(256), 0, stream, in32, in16, w8, bias,
                       mask, resid, out16, out32, relu, H, W, groups);
  else if (cin == 1 && cout == 1)
    hipLaunchKernelGGL((cnn_conv_kernel<1, 1>), grid, dim3(256), 0, stream, in32, in16, w8, bias,
                       mask, resid, out16, out32, relu, H, W, groups);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

int cnn_wgrad_rows() { return 16; }

hipError_t launch_cnn_wgrad(int cin, int cout, const float* dz32, const uint16_t* dz16,
                            const float* in32, const uint16_t* in16, float* partial, float* out,
                            int batch, int H, int W, hipStream_t stream) {
  const int rows = cnn_wgrad_rows();
  const int blocks = batch * (W / 64) * ((H + rows - 1) / rows);
  const int nout = cout * cin * 9 + cout;
  if (cin == 1 && cout == 16)
    hipLaunchKernelGGL((cnn_wgrad_kernel<1, 16>), dim3(blocks), dim3(256), 0, stream, dz32, dz16,
                       in32, in16, partial, H, W, rows);
  else if (cin == 16 && cout == 16)
    hipLaunchKernelGGL((cnn_wgrad_kernel<16, 16>), dim3(blocks), dim3(256), 0, stream, dz32, dz16,
                       in32, in16, partial, H, W, rows);
  else if (cin == 16 && cout == 1)
    hipLaunchKernelGGL((cnn_wgrad_kernel<16, 1>), dim3(blocks), dim3(256), 0, stream, dz32, dz16,
                       in32, in16, partial, H, W, rows);
  else
    return hipErrorInvalidValue;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(cnn_reduce_kernel, dim3(nout), dim3(256), 0, stream, partial, out, blocks,
                     nout);
  return hipGetLastError();
}

}  // namespace fhtfbp
