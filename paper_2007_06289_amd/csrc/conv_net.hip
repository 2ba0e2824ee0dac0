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

#include <algorithm>

#include "fhtfbp_internal.h"

namespace fhtfbp {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ uint16_t f2bf(float f) {   // round to nearest even (hardware)
  return __builtin_bit_cast(uint16_t, (__bf16)f);
}
typedef float float2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
// Two floats as BF16 in one word (a in the low half): one hardware conversion.
__device__ __forceinline__ uint32_t pack2_bf16(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((float2v){a, b}, bf16x2v));
}
// Four channels of one pixel as BF16, packed for one 8-byte store.
__device__ __forceinline__ uint2 pack4_bf16(float a, float b, float c, float d) {
  return make_uint2(pack2_bf16(a, b), pack2_bf16(c, d));
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
// and h2 over the tile plus one, both BF16 in LDS (zero outside the image: the zero padding
// of the next layer), and writes the tile.  Each layer issues the same matrix-core operations
// with the same operands as cnn_conv_kernel (same K order, same BF16 roundings, bias then
// ReLU, then the residual), so the image equals the three separate launches bit for bit;
// only h1 and h2 never go to HBM.  A group is 16 consecutive pixels of a region in row-major
// order; lane (m, kg) of a wave ends with channels 4 kg .. + 3 of pixel m.  In LDS the 16
// channels of a pixel are split in two planes of 8 (16 bytes per pixel and plane): the 16
// lanes that read one operand half then read 256 consecutive bytes.
template <int TH, int TW>
struct FusedTile {
  static constexpr int XR = TH + 6, XC = TW + 6;         // x region
  static constexpr int H1R = TH + 4, H1C = TW + 4;       // h1 region
  static constexpr int H2R = TH + 2, H2C = TW + 2;       // h2 region
  static constexpr int H1Px = H1R * H1C, H2Px = H2R * H2C;
  static constexpr int H1Groups = H1Px / 16, H2Groups = (H2Px + 15) / 16;
  // h2 is stored for whole groups of 16 pixels (the last group's extra pixels are never read)
  static constexpr int H2Store = H2Groups * 16;
  static constexpr int OutGroups = TH * (TW / 16);
  static_assert(H1Px % 16 == 0, "h1 region in whole groups of 16 pixels");
  static_assert(TW % 16 == 0 && OutGroups % 8 == 0, "output groups pair up");
};

template <int TH, int TW>
__global__ void __launch_bounds__(256) cnn_fused_kernel(const float* __restrict__ in,
                                                        const bf16x8* __restrict__ w1,
                                                        const float* __restrict__ b1,
                                                        const bf16x8* __restrict__ w2,
                                                        const float* __restrict__ b2,
                                                        const bf16x8* __restrict__ w3,
                                                        const float* __restrict__ b3,
                                                        float* __restrict__ out, int H, int W,
                                                        int tiles_x, int tiles_per_img,
                                                        int total_tiles) {
  using T = FusedTile<TH, TW>;
  constexpr int XPX = T::XR * T::XC;
  constexpr int XPT = (XPX + 255) / 256;             // x values per thread and tile
  __shared__ float sx[2][XPX];                       // this tile's x region and the next one's
  __shared__ __align__(16) uint16_t sh1[2 * T::H1Px * 8];
  __shared__ __align__(16) uint16_t sh2[2 * T::H2Store * 8];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int m = lane & 15, kg = lane >> 4;
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
  // Operand addressing of layers 2 and 3, fixed per lane: step s reads tap 2 s + kg / 2, i.e.
  // the pixel (tap / 3) rows and (tap % 3) columns from the lane's base pixel, in channel
  // plane kg % 2.  Tap 9 (step 4, kg >= 2) does not exist: those lanes read their base pixel
  // and zero it.
  int o1[5], o2[5];
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    const int tap = 2 * s + (kg >> 1);
    o1[s] = tap < 9 ? (tap / 3) * T::H1C + tap % 3 : 0;
    o2[s] = tap < 9 ? (tap / 3) * T::H2C + tap % 3 : 0;
  }
  const bool tap9 = (kg >> 1) != 0;
  // layer 1's operand words: lane group 0 keeps taps 0..7, group 1 tap 8 (first word)
  const uint32_t lmask0 = kg == 0 ? 0xffffffffu : 0u, lmask8 = kg == 1 ? 0xffffffffu : 0u;
  // The weights and biases are waited for here, before the tile loop: an empty asm that reads
  // them makes the compiler complete their loads once, so that inside the loop no wait for
  // them also waits for the next tile's x loads, which are issued later.
  asm volatile("" ::"v"(w1op), "v"(w2op[0]), "v"(w2op[1]), "v"(w2op[2]), "v"(w2op[3]),
               "v"(w2op[4]));
  asm volatile("" ::"v"(w3op[0]), "v"(w3op[1]), "v"(w3op[2]), "v"(w3op[3]), "v"(w3op[4]));
  asm volatile("" ::"v"(bias1[0]), "v"(bias1[1]), "v"(bias1[2]), "v"(bias1[3]), "v"(bias2[0]),
               "v"(bias2[1]), "v"(bias2[2]), "v"(bias2[3]), "v"(bias3));
  const uint16_t* sh1l = sh1 + (kg & 1) * T::H1Px * 8;
  const uint16_t* sh2l = sh2 + (kg & 1) * T::H2Store * 8;

  // The x region of tile tl (three pixels of halo, zero outside the image): loaded into
  // registers, later stored into one of the two LDS buffers.
  float xr[XPT];
  auto load_x = [&](int tl) {
    const int b = tl / tiles_per_img, t = tl - b * tiles_per_img;
    const int Y0 = (t / tiles_x) * TH, X0 = (t % tiles_x) * TW;
    const float* img = in + (size_t)b * H * W;
#pragma unroll
    for (int k = 0; k < XPT; ++k) {
      const int e = tid + k * 256;
      const int r = e / T::XC, c = e - r * T::XC;
      const int gy = Y0 - 3 + r, gx = X0 - 3 + c;
      xr[k] = (e < XPX && gy >= 0 && gy < H && gx >= 0 && gx < W) ? img[(size_t)gy * W + gx]
                                                                  : 0.f;
    }
  };
  auto store_x = [&](float* dst) {
#pragma unroll
    for (int k = 0; k < XPT; ++k)
      if (tid + k * 256 < XPX) dst[tid + k * 256] = xr[k];
  };

  int tl = blockIdx.x;
  if (tl >= total_tiles) return;
  load_x(tl);
  store_x(sx[0]);
  __syncthreads();
  for (int buf = 0; tl < total_tiles; tl += gridDim.x, buf ^= 1) {
    const int b = tl / tiles_per_img;
    const int t = tl - b * tiles_per_img;
    const int Y0 = (t / tiles_x) * TH, X0 = (t % tiles_x) * TW;
    const float* sxc = sx[buf];
    // the next tile's x goes out now and lands while this tile's layers run
    const int tn = tl + (int)gridDim.x;
    if (tn < total_tiles) load_x(tn);
    // every region pixel of an interior tile lies in the image: no zeroing to decide
    const bool interior = Y0 >= 3 && X0 >= 3 && Y0 + TH + 3 <= H && X0 + TW + 3 <= W;

    // Bias, ReLU and BF16 of a lane's four channels of region pixel px (zero outside the
    // image), stored as one 8-byte word into plane kg / 2 of a region of `px_total` pixels.
    auto store4 = [&](uint16_t* dst, int px_total, const f32x4& acc, const float* bias, int px,
                      int cols, int oy, int ox) {
      uint2 w = pack4_bf16(fmaxf(acc[0] + bias[0], 0.f), fmaxf(acc[1] + bias[1], 0.f),
                           fmaxf(acc[2] + bias[2], 0.f), fmaxf(acc[3] + bias[3], 0.f));
      if (!interior) {
        const int rr = px / cols, cc = px - rr * cols;
        const int gy = Y0 + oy + rr, gx = X0 + ox + cc;
        if (!(gy >= 0 && gy < H && gx >= 0 && gx < W)) w = make_uint2(0u, 0u);
      }
      *reinterpret_cast<uint2*>(dst + ((kg >> 1) * px_total + px) * 8 + (kg & 1) * 4) = w;
    };

    // layer 1: x (1 channel) -> h1 (16).  Lane group kg holds taps 8 kg .. 8 kg + 7: kg = 0
    // taps 0..7, kg = 1 tap 8, the rest zero; every lane reads and selects (no branch).
    // all nine taps are read by every lane (immediate offsets, no branch), converted in pairs,
    // and each lane keeps its own words: kg = 0 taps 0..7, kg = 1 tap 8, else zero
    auto a1 = [&](int p) -> bf16x8 {
      const int r = p / T::H1C, c = p - r * T::H1C;
      const float* xp = sxc + r * T::XC + c;
      float tv[9];
#pragma unroll
      for (int j = 0; j < 9; ++j) tv[j] = xp[(j / 3) * T::XC + j % 3];
      uint32_t w[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) w[k] = pack2_bf16(tv[2 * k], tv[2 * k + 1]) & lmask0;
      w[0] |= pack2_bf16(tv[8], 0.f) & lmask8;
      return __builtin_bit_cast(bf16x8, make_uint4(w[0], w[1], w[2], w[3]));
    };
    // two groups (g, g + 4) at a time, as in the layers below
    for (int g = wave; g < T::H1Groups; g += 8) {
      const int gb = g + 4 < T::H1Groups ? g + 4 : g;
      const int pa = g * 16 + m, pb = gb * 16 + m;
      const bf16x8 aa = a1(pa), ab = a1(pb);
      f32x4 acca = {0.f, 0.f, 0.f, 0.f}, accb = {0.f, 0.f, 0.f, 0.f};
      acca = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1op, aa, acca, 0, 0, 0);
      accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1op, ab, accb, 0, 0, 0);
      store4(sh1, T::H1Px, acca, bias1, pa, T::H1C, -2, -2);
      store4(sh1, T::H1Px, accb, bias1, pb, T::H1C, -2, -2);
    }
    __syncthreads();   // h1 complete; the previous tile's layer 3 is done with h2

    // The activation operand of step s for base pixel index q of a 16-channel region (lane
    // plane `src`, per-lane tap offsets `o`): K = tap * 16 + channel; zero past the ninth tap.
    auto a16 = [&](const uint16_t* src, const int* o, int q, int s) -> bf16x8 {
      bf16x8 a = *reinterpret_cast<const bf16x8*>(src + (q + o[s]) * 8);
      if (s == 4 && tap9) a = bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
      return a;
    };

    // layer 2: h1 (16) -> h2 (16).  A wave takes two groups at a time (its groups g and g + 4;
    // the second repeats the first when there is none): their operands load together and the
    // two accumulation chains interleave on the matrix core.
    for (int g = wave; g < T::H2Groups; g += 8) {
      const int gb = g + 4 < T::H2Groups ? g + 4 : g;
      const int pa = g * 16 + m, pb = gb * 16 + m;           // < H2Store
      const int qa = min(pa, T::H2Px - 1), qb = min(pb, T::H2Px - 1);
      const int ra = qa / T::H2C, ca = qa - ra * T::H2C, rb = qb / T::H2C, cb = qb - rb * T::H2C;
      const int ba = ra * T::H1C + ca, bb = rb * T::H1C + cb;   // base pixels in the h1 region
      bf16x8 aa[5], ab[5];
#pragma unroll
      for (int s = 0; s < 5; ++s) {
        aa[s] = a16(sh1l, o1, ba, s);
        ab[s] = a16(sh1l, o1, bb, s);
      }
      f32x4 acca = {0.f, 0.f, 0.f, 0.f}, accb = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 5; ++s) {
        acca = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2op[s], aa[s], acca, 0, 0, 0);
        accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2op[s], ab[s], accb, 0, 0, 0);
      }
      store4(sh2, T::H2Store, acca, bias2, pa, T::H2C, -1, -1);
      store4(sh2, T::H2Store, accb, bias2, pb, T::H2C, -1, -1);
    }
    if (tn < total_tiles) store_x(sx[buf ^ 1]);
    __syncthreads();   // h2 and the next tile's x region complete

    // layer 3: h2 (16) -> 1 channel (channel 0: lanes kg = 0, first element), plus bias and
    // the residual; a group is 16 pixels of a tile row, two groups (g, g + 4) per wave at a time
    float* dst = out + (size_t)b * H * W;
    for (int g = wave; g < T::OutGroups; g += 8) {
      bf16x8 aa[5], ab[5];
      const int ra = g / (TW / 16), ca = (g % (TW / 16)) * 16 + m;
      const int rb = (g + 4) / (TW / 16), cb = ((g + 4) % (TW / 16)) * 16 + m;
#pragma unroll
      for (int s = 0; s < 5; ++s) {
        aa[s] = a16(sh2l, o2, ra * T::H2C + ca, s);
        ab[s] = a16(sh2l, o2, rb * T::H2C + cb, s);
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
          dst[(size_t)gya * W + gxa] = acca[0] + bias3 + sxc[(ra + 3) * T::XC + ca + 3];
        if (gyb < H && gxb < W)
          dst[(size_t)gyb * W + gxb] = accb[0] + bias3 + sxc[(rb + 3) * T::XC + cb + 3];
      }
    }
  }
}

}  // namespace

// Output tile of the fused network: 16 x 32 pixels (50 KB of LDS per block).  The launch is
// persistent: as many blocks as the device holds at once, each looping over tiles.
constexpr int kFuseTH = 16, kFuseTW = 32;

hipError_t launch_cnn_fused(const float* in, const uint16_t* w1, const float* b1,
                            const uint16_t* w2, const float* b2, const uint16_t* w3,
                            const float* b3, float* out, int batch, int H, int W,
                            hipStream_t stream) {
  const int tiles_x = (W + kFuseTW - 1) / kFuseTW, tiles_y = (H + kFuseTH - 1) / kFuseTH;
  const long long tiles = (long long)batch * tiles_x * tiles_y;
  if (tiles > 0x7fffffffll) return hipErrorInvalidValue;
  auto kern = cnn_fused_kernel<kFuseTH, kFuseTW>;
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0);
  if (e != hipSuccess) return e;
  const long long grid = std::min<long long>(tiles, (long long)cus * std::max(per_cu, 1));
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), 0, stream, in,
                     reinterpret_cast<const bf16x8*>(w1), b1, reinterpret_cast<const bf16x8*>(w2),
                     b2, reinterpret_cast<const bf16x8*>(w3), b3, out, H, W, tiles_x,
                     tiles_x * tiles_y, (int)tiles);
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
