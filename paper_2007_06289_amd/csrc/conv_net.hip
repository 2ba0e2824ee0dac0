// Learned residual correction applied after the reconstruction: 3x3 convolutions (zero
// padding 1) with 1 or 16 channels, as implicit GEMMs on the matrix cores (BF16 operands, FP32
// accumulation, v_mfma_f32_16x16x32_bf16), plus FP32 weight gradients.
//
// Activations with 16 channels are stored BF16, NHWC ([b][y][x][c], 32 bytes per pixel);
// single-channel images are FP32 [b][y][x].  A wave computes 16 consecutive pixels of one row
// x 16 output channels: out[p][n] = sum_kk Act[p][kk] Wg[kk][n], kk = tap * CIN + ci (tap =
// 3 (dy + 1) + dx + 1), in steps of 32 kk.  Operand layouts of the 16x16x32 instruction: lane l
// holds A[l % 16][8 (l / 16) .. + 7] and B[8 (l / 16) .. + 7][l % 16]; the result C[4 (l / 16) +
// i][l % 16] for i < 4.  The weights go in as A (Wg transposed: A[n][kk]) and the activations as
// B (B[kk][p]), so the instruction yields out transposed: lane l holds channels 4 (l / 16) ..
// + 3 of pixel l % 16, which it stores as one 8-byte word.  BF16 rounding is the hardware's
// round-to-nearest-even conversion.  The backward convolution with respect to the input is the
// same kernel with the weights transposed and the taps flipped (packed by cnn_pack_kernel), and
// its output multiplied by the ReLU mask of the layer below.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fhtfbp_internal.h"

namespace fhtfbp {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ uint16_t f2bf(float f) {   // round to nearest even (hardware)
  return __builtin_bit_cast(uint16_t, (__bf16)f);
}
// Four channels of one pixel as BF16, packed for one 8-byte store.
__device__ __forceinline__ uint2 pack4_bf16(float a, float b, float c, float d) {
  return make_uint2((uint32_t)f2bf(a) | ((uint32_t)f2bf(b) << 16),
                    (uint32_t)f2bf(c) | ((uint32_t)f2bf(d) << 16));
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
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw, a, acc, 0, 0, 0);
  }
  // lane (m, kg): pixel x, channels 4 kg .. 4 kg + 3
  const size_t pix = ((size_t)b * H + y) * W + x;
  if constexpr (COUT == 16) {
    float v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      v[i] = acc[i] + (bias ? bias[4 * kg + i] : 0.f);
      if (relu) v[i] = fmaxf(v[i], 0.f);
      if (mask && !(bf2f(mask[pix * 16 + 4 * kg + i]) > 0.f)) v[i] = 0.f;
    }
    *reinterpret_cast<uint2*>(out16 + pix * 16 + 4 * kg) = pack4_bf16(v[0], v[1], v[2], v[3]);
  } else {
    if (kg == 0) out32[pix] = acc[0] + (bias ? bias[0] : 0.f) + (resid ? resid[pix] : 0.f);
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

// ---- the whole network in one launch (inference) ----------------------------------------------
// out = x + conv3(relu(conv2(relu(conv1(x) + b1)) + b2)) + b3 over tiles of TH x TW output
// pixels.  A block loads the x region the tile depends on (three pixels of halo on each
// side, zero outside the image) into LDS, computes h1 over the tile plus two pixels of halo
// and h2 over the tile plus one, both BF16 NHWC in LDS (zero outside the image: the zero
// padding of the next layer), and writes the tile.  Each layer issues the same matrix-core
// operations with the same operands as cnn_conv_kernel (same K order, same BF16 roundings,
// bias then ReLU, then the residual), so the image equals the three separate launches bit for
// bit; only h1 and h2 never go to HBM.  A group is 16 consecutive pixels of a region in
// row-major order; lane (m, kg) of a wave ends with channels 4 kg .. + 3 of pixel m.
constexpr int kFuseTH = 16, kFuseTW = 32;
constexpr int kXR = kFuseTH + 6, kXC = kFuseTW + 6;      // x region 22 x 38
constexpr int kH1R = kFuseTH + 4, kH1C = kFuseTW + 4;    // h1 region 20 x 36
constexpr int kH2R = kFuseTH + 2, kH2C = kFuseTW + 2;    // h2 region 18 x 34
constexpr int kH1Px = kH1R * kH1C, kH2Px = kH2R * kH2C;
constexpr int kH1Groups = (kH1Px + 15) / 16, kH2Groups = (kH2Px + 15) / 16;
// h2 is stored for whole groups of 16 pixels (the last group's extra pixels are never read)
constexpr int kH2Store = kH2Groups * 16;
static_assert(kH1Px % 16 == 0, "h1 region in whole groups of 16 pixels");

__global__ void __launch_bounds__(256) cnn_fused_kernel(const float* __restrict__ in,
                                                        const bf16x8* __restrict__ w1,
                                                        const float* __restrict__ b1,
                                                        const bf16x8* __restrict__ w2,
                                                        const float* __restrict__ b2,
                                                        const bf16x8* __restrict__ w3,
                                                        const float* __restrict__ b3,
                                                        float* __restrict__ out, int H, int W,
                                                        int tiles_x, int tiles_per_img) {
  __shared__ float sx[kXR * kXC];
  __shared__ __align__(16) uint16_t sh1[kH1Px * 16];
  __shared__ __align__(16) uint16_t sh2[kH2Store * 16];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int m = lane & 15, kg = lane >> 4;
  const int b = blockIdx.x / tiles_per_img;
  const int t = blockIdx.x - b * tiles_per_img;
  const int Y0 = (t / tiles_x) * kFuseTH, X0 = (t % tiles_x) * kFuseTW;
  const float* img = in + (size_t)b * H * W;
  for (int e = tid; e < kXR * kXC; e += 256) {
    const int r = e / kXC, c = e - r * kXC;
    const int gy = Y0 - 3 + r, gx = X0 - 3 + c;
    sx[e] = (gy >= 0 && gy < H && gx >= 0 && gx < W) ? img[(size_t)gy * W + gx] : 0.f;
  }
  const bf16x8 w1op = w1[lane];
  bf16x8 w2op[5], w3op[5];
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    w2op[s] = w2[s * 64 + lane];
    w3op[s] = w3[s * 64 + lane];
  }
  float bias1[4], bias2[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    bias1[i] = b1[4 * kg + i];
    bias2[i] = b2[4 * kg + i];
  }
  const float bias3 = b3[0];
  __syncthreads();

  // Bias, ReLU and BF16 of a lane's four channels of region pixel px (zero outside the image),
  // stored as one 8-byte word.
  auto store4 = [&](uint16_t* dst, const f32x4& acc, const float* bias, int px, int cols,
                    int oy, int ox) {
    const int rr = px / cols, cc = px - rr * cols;
    const int gy = Y0 + oy + rr, gx = X0 + ox + cc;
    const bool inside = gy >= 0 && gy < H && gx >= 0 && gx < W;
    uint2 w = pack4_bf16(fmaxf(acc[0] + bias[0], 0.f), fmaxf(acc[1] + bias[1], 0.f),
                         fmaxf(acc[2] + bias[2], 0.f), fmaxf(acc[3] + bias[3], 0.f));
    if (!inside) w = make_uint2(0u, 0u);
    *reinterpret_cast<uint2*>(dst + px * 16 + 4 * kg) = w;
  };

  // layer 1: x (1 channel) -> h1 (16).  Lane group kg holds taps 8 kg .. 8 kg + 7: kg = 0
  // taps 0..7, kg = 1 tap 8, the rest zero; every lane reads and selects (no branch).
  for (int g = wave; g < kH1Groups; g += 4) {
    const int p = g * 16 + m;
    const int r = p / kH1C, c = p - r * kH1C;
    const float* xp = sx + r * kXC + c;
    float v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float v0 = xp[(j / 3) * kXC + j % 3];
      const float v8 = xp[2 * kXC + 2];
      v[j] = kg == 0 ? v0 : ((kg == 1 && j == 0) ? v8 : 0.f);
    }
    bf16x8 a;
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = (short)f2bf(v[j]);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1op, a, acc, 0, 0, 0);
    store4(sh1, acc, bias1, p, kH1C, -2, -2);
  }
  __syncthreads();

  // The activation operand of step s for the pixel at (r, c) of a 16-channel region of `cols`
  // columns: K = tap * 16 + channel, lane group kg holds 8 channels of tap 2 s + kg / 2 (zero
  // past the ninth tap).
  auto a16 = [&](const uint16_t* src, int cols, int r, int c, int s) -> bf16x8 {
    const int kk0 = s * 32 + kg * 8;
    const int tap = kk0 >> 4, c0 = kk0 & 15;
    bf16x8 a = bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
    if (tap < 9)
      a = *reinterpret_cast<const bf16x8*>(src + ((r + tap / 3) * cols + c + tap % 3) * 16 + c0);
    return a;
  };

  // layer 2: h1 (16) -> h2 (16).  A wave takes two groups at a time (its groups g and g + 4;
  // the second repeats the first when there is none): their operands load together and the
  // two accumulation chains interleave on the matrix core.
  for (int g = wave; g < kH2Groups; g += 8) {
    const int gb = g + 4 < kH2Groups ? g + 4 : g;
    const int pa = g * 16 + m, pb = gb * 16 + m;           // < kH2Store
    const int qa = min(pa, kH2Px - 1), qb = min(pb, kH2Px - 1);
    const int ra = qa / kH2C, ca = qa - ra * kH2C, rb = qb / kH2C, cb = qb - rb * kH2C;
    bf16x8 aa[5], ab[5];
#pragma unroll
    for (int s = 0; s < 5; ++s) {
      aa[s] = a16(sh1, kH1C, ra, ca, s);
      ab[s] = a16(sh1, kH1C, rb, cb, s);
    }
    f32x4 acca = {0.f, 0.f, 0.f, 0.f}, accb = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 5; ++s) {
      acca = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2op[s], aa[s], acca, 0, 0, 0);
      accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2op[s], ab[s], accb, 0, 0, 0);
    }
    store4(sh2, acca, bias2, pa, kH2C, -1, -1);
    store4(sh2, accb, bias2, pb, kH2C, -1, -1);
  }
  __syncthreads();

  // layer 3: h2 (16) -> 1 channel (channel 0: lanes kg = 0, first element), plus bias and the
  // residual; a group is 16 pixels of a tile row, two groups (g, g + 4) per wave at a time
  float* dst = out + (size_t)b * H * W;
  constexpr int kOutGroups = kFuseTH * (kFuseTW / 16);
  static_assert(kOutGroups % 8 == 0, "output groups pair up");
  for (int g = wave; g < kOutGroups; g += 8) {
    bf16x8 aa[5], ab[5];
    const int ra = g / (kFuseTW / 16), ca = (g % (kFuseTW / 16)) * 16 + m;
    const int rb = (g + 4) / (kFuseTW / 16), cb = ((g + 4) % (kFuseTW / 16)) * 16 + m;
#pragma unroll
    for (int s = 0; s < 5; ++s) {
      aa[s] = a16(sh2, kH2C, ra, ca, s);
      ab[s] = a16(sh2, kH2C, rb, cb, s);
    }
    f32x4 acca = {0.f, 0.f, 0.f, 0.f}, accb = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 5; ++s) {
      acca = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3op[s], aa[s], acca, 0, 0, 0);
      accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3op[s], ab[s], accb, 0, 0, 0);
    }
    if (kg == 0) {
      const int gya = Y0 + ra, gxa = X0 + ca, gyb = Y0 + rb, gxb = X0 + cb;
      if (gya < H && gxa < W)
        dst[(size_t)gya * W + gxa] = acca[0] + bias3 + sx[(ra + 3) * kXC + ca + 3];
      if (gyb < H && gxb < W)
        dst[(size_t)gyb * W + gxb] = accb[0] + bias3 + sx[(rb + 3) * kXC + cb + 3];
    }
  }
}

}  // namespace

hipError_t launch_cnn_fused(const float* in, const uint16_t* w1, const float* b1,
                            const uint16_t* w2, const float* b2, const uint16_t* w3,
                            const float* b3, float* out, int batch, int H, int W,
                            hipStream_t stream) {
  const int tiles_x = (W + kFuseTW - 1) / kFuseTW, tiles_y = (H + kFuseTH - 1) / kFuseTH;
  const long long blocks = (long long)batch * tiles_x * tiles_y;
  if (blocks > 0x7fffffffll) return hipErrorInvalidValue;
  hipLaunchKernelGGL(cnn_fused_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, in,
                     reinterpret_cast<const bf16x8*>(w1), b1, reinterpret_cast<const bf16x8*>(w2),
                     b2, reinterpret_cast<const bf16x8*>(w3), b3, out, H, W, tiles_x,
                     tiles_x * tiles_y);
  return hipGetLastError();
}

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
