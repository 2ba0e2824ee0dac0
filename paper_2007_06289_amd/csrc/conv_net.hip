// Learned residual correction applied after the reconstruction: 3x3 convolutions (zero
// padding 1) with 1 or 16 channels, as implicit GEMMs on the matrix cores (BF16 operands, FP32
// accumulation), plus their weight gradients, also on the matrix cores (FP32 sums; BF16
// operands for 16 -> 16, FP32 operands for the single-channel layers).
//
// Activations with 16 channels are stored BF16, NHWC ([b][y][x][c], 32 bytes per pixel);
// single-channel images are FP32 [b][y][x].  A wave computes 16 consecutive pixels of one row
// x 16 output channels: out[p][n] = sum_kk Act[p][kk] Wg[kk][n].  The weights go in as the A
// operand (Wg transposed: A[n][kk]) and the activations as B (B[kk][p]), so the instruction
// yields out transposed: lane l holds channels 4 (l / 16) .. + 3 of pixel l % 16 (C[4 (l / 16) +
// i][l % 16], i < 4), which it stores as one 8-byte word.  Operand layouts: in a 16x16x32 step
// lane l holds A[l % 16][8 (l / 16) .. + 7] and B[8 (l / 16) .. + 7][l % 16]; in a 16x16x16 step
// A[l % 16][4 (l / 16) .. + 3] and B[4 (l / 16) .. + 3][l % 16].
//
// K order (taps t = 3 dy + dx, dy, dx in 0..2 for the offsets -1..1), chosen so that the
// operands of one window row serve every output row that uses it, with no padding taps:
//   16 input channels: three 16x16x32 steps s = 0..2 for window row dy = s, lane group g
//     holding column dx = g / 2 and channels 8 (g % 2) .. + 7; then three 16x16x16 steps for
//     column dx = 2 of rows dy = 0..2, lane group g holding channels 4 g .. + 3.
//   1 input channel: one 16x16x16 step, lane group g < 3 holding taps 3 g .. 3 g + 2 (row dy =
//     g) and a zero, group 3 zeros.
// A convolution from 16 channels to one turns the roles around: one 16x16x16 step per pixel
// group with the taps as the rows of A (A[t][c] = w[c][t], rows 9..15 zero) and the pixel's
// channels as B (lane group g: channels 4 g .. + 3, the layout a 16-channel layer's result
// already has) gives the nine per-tap partial sums of each pixel; an output pixel is then the
// sum of its nine neighbours' partials in tap order, in FP32.
// BF16 rounding is the hardware's round-to-nearest-even conversion.  The backward convolution
// with respect to the input is the same kernel with the weights transposed and the taps
// flipped (packed by cnn_pack_kernel), and its output multiplied by the ReLU mask of the layer
// below.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "fhtfbp_internal.h"

namespace fhtfbp {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(short)))) short bf16x4;
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
// ReLU of two packed BF16 values: as 16-bit integers the negative ones (sign bit set) are the
// negative ones, so a packed integer max with 0 clears them (the same values as the FP32 max
// before rounding: rounding keeps the sign and maps no positive value to a negative one).
typedef short short2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t w) {
  return __builtin_bit_cast(uint32_t,
                            __builtin_elementwise_max(__builtin_bit_cast(short2v, w), short2v{0, 0}));
}


__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// A block's copy of ITEMS values into LDS, item e = thread + 256 j: each thread issues all of
// its loads before its first store, so their memory latencies overlap instead of adding up.
template <int ITEMS, typename Load, typename Store>
__device__ __forceinline__ void stage_block(int tid, Load load, Store store) {
  constexpr int PER = (ITEMS + 255) / 256;
  decltype(load(0)) v[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int e = tid + 256 * j;
    if (e < ITEMS) v[j] = load(e);
  }
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int e = tid + 256 * j;
    if (e < ITEMS) store(e, v[j]);
  }
}

// Packs FP32 weights w[cout][cin][9] into the A operand order of the kernel (the K order in
// the header), 512 values per step (16x16x32: packed[step][lane][j] = Wg[kk(step, lane, j)]
// [lane % 16], j < 8; a 16x16x16 step uses the first 256, j < 4).  transpose_flip: pack the
// weights of the input-gradient convolution, Wg'[tap][co' = ci][ci' = co] = w[co][ci][8 - tap].
__global__ void cnn_pack_kernel(const float* __restrict__ w, uint16_t* __restrict__ packed,
                                int cin, int cout, int transpose_flip, int steps) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= steps * 64 * 8) return;
  // geometry of the convolution being packed (after the transpose for the backward one)
  const int ci_n = transpose_flip ? cout : cin;    // its input channels
  const int co_n = transpose_flip ? cin : cout;    // its output channels
  const int step = e >> 9, r = e & 511;
  int tap = -1, c = 0, n = 0;
  if (ci_n == 16 && co_n == 1) {         // taps x channels: A[t][c] at lane t + 16 (c / 4), c % 4
    if (step == 0 && r < 256) {
      const int lane = r >> 2, t = lane & 15;
      if (t < 9) {
        tap = t;
        c = 4 * (lane >> 4) + (r & 3);
      }
    }
  } else if (ci_n == 16) {               // 16 -> 16: the 16x16x32 steps, then the 16x16x16 ones
    if (e < 3 * 512) {                   // row dy = step, lane l: column (l / 16) / 2
      const int lane = r >> 3, j = r & 7, g = lane >> 4;
      n = lane & 15;
      tap = 3 * step + (g >> 1);
      c = (g & 1) * 8 + j;
    } else if (e < 3 * 512 + 3 * 256) {  // row dy = (e - 1536) / 256, column 2
      const int r4 = e - 3 * 512, lane = (r4 & 255) >> 2, j = r4 & 3, g = lane >> 4;
      n = lane & 15;
      tap = 3 * (r4 >> 8) + 2;
      c = 4 * g + j;
    }
  } else if (r < 256) {                  // 1 input channel: one 16x16x16 step
    const int lane = r >> 2, j = r & 3, g = lane >> 4;
    n = lane & 15;
    if (g < 3 && j < 3) tap = 3 * g + j;
  }
  float v = 0.f;
  if (tap >= 0 && n < co_n && c < ci_n) {
    if (!transpose_flip) v = w[(n * cin + c) * 9 + tap];
    else v = w[(c * cin + n) * 9 + (8 - tap)];
  }
  packed[e] = f2bf(v);
}

// The epilogue of a 16-channel output, shared by the per-layer kernels: lane (m, kg) holds
// channels 4 kg .. + 3 of pixel pix; bias, then the mask (kept where > 0: the ReLU derivative
// of the layer below, in the backward pass), BF16, then the optional ReLU, one 8-byte store.
// The mask word (the lane's 4 channels of the pixel) is loaded by the caller, ahead of time.
__device__ __forceinline__ void store_c16(const f32x4& acc, const float (&bs)[4], bool masked,
                                          uint2 mw, int relu, uint16_t* __restrict__ out16,
                                          size_t pix, int kg) {
  float v[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) v[j] = acc[j] + bs[j];
  if (masked) {
    const uint16_t mh[4] = {(uint16_t)mw.x, (uint16_t)(mw.x >> 16), (uint16_t)mw.y,
                            (uint16_t)(mw.y >> 16)};
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (!(bf2f(mh[j]) > 0.f)) v[j] = 0.f;
  }
  uint2 w = pack4_bf16(v[0], v[1], v[2], v[3]);
  if (relu) w = make_uint2(relu_bf16x2(w.x), relu_bf16x2(w.y));
  *reinterpret_cast<uint2*>(out16 + pix * 16 + 4 * kg) = w;
}

// 1 -> 16 convolution (FP32 image in, BF16 NHWC out) over tiles of 32 x 32 output pixels: the
// 34 x 34 input pixels a tile needs (zero outside the image) are staged once in LDS, and each
// wave walks one 16-column segment down 16 rows, one 16x16x16 step per output row with the
// operands of the K order in the header (lane group g < 3: window row g, columns 0..2 and a
// zero; group 3 zeros).
constexpr int kC1TH = 32, kC1TW = 32;
__global__ void __launch_bounds__(256) cnn_conv1_tile_kernel(const float* __restrict__ in32,
                                                             const bf16x8* __restrict__ wop,
                                                             const float* __restrict__ bias,
                                                             const uint16_t* __restrict__ mask,
                                                             uint16_t* __restrict__ out16,
                                                             int relu, int H, int W, int tiles_x,
                                                             int tiles_per_img) {
  constexpr int RR = kC1TH + 2, RC = kC1TW + 2;
  __shared__ float sx[RR * RC];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int m = lane & 15, kg = lane >> 4;
  const int b = blockIdx.x / tiles_per_img, t = blockIdx.x - b * tiles_per_img;
  const int Y0 = (t / tiles_x) * kC1TH, X0 = (t % tiles_x) * kC1TW;
  // the mask words of this lane's output pixels, loaded before the staging
  uint2 mw[kC1TH / 2];
  {
    const int gx = X0 + (wave & 1) * 16 + m, r0 = (wave >> 1) * (kC1TH / 2);
#pragma unroll
    for (int i = 0; i < kC1TH / 2; ++i) {
      const int gy = Y0 + r0 + i;
      mw[i] = (mask && gx < W && gy < H)
                  ? *reinterpret_cast<const uint2*>(mask + (((size_t)b * H + gy) * W + gx) * 16 +
                                                    4 * kg)
                  : make_uint2(0u, 0u);
    }
  }
  stage_block<RR * RC>(
      tid,
      [&](int e) {
        const int r = e / RC, c = e - r * RC;
        const int gy = Y0 - 1 + r, gx = X0 - 1 + c;
        return (gy >= 0 && gy < H && gx >= 0 && gx < W) ? in32[((size_t)b * H + gy) * W + gx]
                                                         : 0.f;
      },
      [&](int e, float v) { sx[e] = v; });
  const bf16x4 wa = reinterpret_cast<const bf16x4*>(wop)[lane];
  float bs[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) bs[i] = bias ? bias[4 * kg + i] : 0.f;
  __syncthreads();
  const int x = (wave & 1) * 16 + m, r0 = (wave >> 1) * (kC1TH / 2);
  const int gx = X0 + x;
  if (gx >= W) return;   // W is a multiple of 16: whole segments are in or out
  const float* q = sx + (r0 + (kg < 3 ? kg : 0)) * RC + x;
#pragma unroll
  for (int i = 0; i < kC1TH / 2; ++i) {
    const int gy = Y0 + r0 + i;
    if (gy >= H) break;
    bf16x4 a = __builtin_bit_cast(bf16x4, make_uint2(pack2_bf16(q[i * RC], q[i * RC + 1]),
                                                       pack2_bf16(q[i * RC + 2], 0.f)));
    if (kg == 3) a = bf16x4{0, 0, 0, 0};
    const f32x4 acc = mfma16(wa, a, f32x4{0.f, 0.f, 0.f, 0.f});
    store_c16(acc, bs, mask != nullptr, mw[i], relu, out16, ((size_t)b * H + gy) * W + gx, kg);
  }
}

// 16 -> 1 convolution (BF16 NHWC in, FP32 out) over tiles of 32 rows x 30 columns: the nine
// per-tap partial sums (K order of the header) of each input pixel of the tile's 34 x 32
// neighbourhood, two 16-pixel groups per row, go to LDS as nine FP32 planes; an output pixel
// is the sum of its nine neighbours' partials in tap order, then the bias and the residual.
constexpr int kC3TH = 32, kC3TW = 30;
__global__ void __launch_bounds__(256) cnn_conv16to1_tile_kernel(const uint16_t* __restrict__ in16,
                                                                 const bf16x8* __restrict__ wop,
                                                                 const float* __restrict__ bias,
                                                                 const float* __restrict__ resid,
                                                                 float* __restrict__ out32, int H,
                                                                 int W, int tiles_x,
                                                                 int tiles_per_img) {
  constexpr int PR = kC3TH + 2, PC = kC3TW + 2;
  static_assert(PC == 32 && (2 * PR) % 4 == 0, "two groups per row, whole rounds of 4 waves");
  constexpr int PS = PR * PC + 4;   // plane stride: lane groups 0..2 land in different banks
  __shared__ float sp[9 * PS];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int m = lane & 15, kg = lane >> 4;
  const int b = blockIdx.x / tiles_per_img, t = blockIdx.x - b * tiles_per_img;
  const int Y0 = (t / tiles_x) * kC3TH, X0 = (t % tiles_x) * kC3TW;
  // the residual of this thread's output pixels, loaded while the partials are formed
  constexpr int OUT_PER = (kC3TH * kC3TW + 255) / 256;
  float rv[OUT_PER];
#pragma unroll
  for (int j = 0; j < OUT_PER; ++j) {
    const int e = tid + 256 * j, r = e / kC3TW, c = e - r * kC3TW;
    const int gy = Y0 + r, gx = X0 + c;
    rv[j] = (resid && e < kC3TH * kC3TW && gy < H && gx < W)
                ? resid[((size_t)b * H + gy) * W + gx] : 0.f;
  }
  const bf16x4 at = reinterpret_cast<const bf16x4*>(wop)[lane];
  constexpr int PER_WAVE = 2 * PR / 4;
  bf16x4 bv[PER_WAVE];
#pragma unroll
  for (int k = 0; k < PER_WAVE; ++k) {   // group wave + 4 k: row q / 2, columns 16 (q % 2) + m
    const int q = wave + 4 * k, r = q >> 1, col = ((q & 1) << 4) + m;
    const int gy = Y0 - 1 + r, gx = X0 - 1 + col;
    bv[k] = bf16x4{0, 0, 0, 0};
    if (gy >= 0 && gy < H && gx >= 0 && gx < W)
      bv[k] = *reinterpret_cast<const bf16x4*>(in16 + (((size_t)b * H + gy) * W + gx) * 16 +
                                               4 * kg);
  }
#pragma unroll
  for (int k = 0; k < PER_WAVE; ++k) {
    const int q = wave + 4 * k, r = q >> 1, col = ((q & 1) << 4) + m;
    const f32x4 pt = mfma16(at, bv[k], f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (4 * kg + i < 9) sp[(4 * kg + i) * PS + r * PC + col] = pt[i];
  }
  __syncthreads();
  const float b0 = bias ? bias[0] : 0.f;
#pragma unroll
  for (int j = 0; j < OUT_PER; ++j) {
    const int e = tid + 256 * j, r = e / kC3TW, c = e - r * kC3TW;
    const int gy = Y0 + r, gx = X0 + c;
    if (e >= kC3TH * kC3TW || gy >= H || gx >= W) continue;
    const float* q = sp + r * PC + c;
    float sum = q[0];
#pragma unroll
    for (int tp = 1; tp < 9; ++tp) sum += q[tp * PS + (tp / 3) * PC + tp % 3];
    out32[((size_t)b * H + gy) * W + gx] = sum + b0 + rv[j];
  }
}

// 16 -> 16 convolution over tiles of 16 output rows x 32 columns: the input pixels the tile
// needs (18 x 34, zero outside the image) are staged once in LDS, in two planes of 8 channels,
// and each wave walks one 16-column segment down 8 output rows as the fused kernel's layer 2
// does, with the same operands and matrix-core steps (the K order of the header), so the two
// give the same h2 bit for bit; each input pixel is read from memory once per tile.  The
// epilogue: bias, then the mask (the ReLU derivative of the layer below, in the backward
// pass), BF16, then the optional ReLU.
constexpr int kC16TH = 16, kC16TW = 32;
__global__ void __launch_bounds__(256) cnn_conv16_tile_kernel(const uint16_t* __restrict__ in16,
                                                              const bf16x8* __restrict__ wop,
                                                              const float* __restrict__ bias,
                                                              const uint16_t* __restrict__ mask,
                                                              uint16_t* __restrict__ out16,
                                                              int relu, int H, int W, int tiles_x,
                                                              int tiles_per_img) {
  constexpr int RR = kC16TH + 2, RC = kC16TW + 2, RP = RR * RC;
  __shared__ __align__(16) uint16_t sin16[2 * RP * 8];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int m = lane & 15, kg = lane >> 4;
  const int b = blockIdx.x / tiles_per_img, t = blockIdx.x - b * tiles_per_img;
  const int Y0 = (t / tiles_x) * kC16TH, X0 = (t % tiles_x) * kC16TW;
  // the mask words of this lane's output pixels, loaded before the staging
  uint2 mw[kC16TH / 2];
  {
    const int gx = X0 + (wave & 1) * 16 + m, r0 = (wave >> 1) * (kC16TH / 2);
#pragma unroll
    for (int i = 0; i < kC16TH / 2; ++i) {
      const int gy = Y0 + r0 + i;
      mw[i] = (mask && gx < W && gy < H)
                  ? *reinterpret_cast<const uint2*>(mask + (((size_t)b * H + gy) * W + gx) * 16 +
                                                    4 * kg)
                  : make_uint2(0u, 0u);
    }
  }
  // 16 bytes (8 channels of plane h) of one region pixel per step
  stage_block<2 * RP>(
      tid,
      [&](int e) {
        const int q = e >> 1, h = e & 1;
        const int r = q / RC, c = q - r * RC;
        const int gy = Y0 - 1 + r, gx = X0 - 1 + c;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (gy >= 0 && gy < H && gx >= 0 && gx < W)
          v = *reinterpret_cast<const uint4*>(in16 + (((size_t)b * H + gy) * W + gx) * 16 + 8 * h);
        return v;
      },
      [&](int e, const uint4& v) {
        *reinterpret_cast<uint4*>(sin16 + ((e & 1) * RP + (e >> 1)) * 8) = v;
      });
  bf16x8 wr[3];
  bf16x4 wd[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    wr[s] = wop[s * 64 + lane];
    wd[s] = reinterpret_cast<const bf16x4*>(wop)[3 * 128 + s * 64 + lane];
  }
  float bs[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) bs[i] = bias ? bias[4 * kg + i] : 0.f;
  __syncthreads();
  const int x = (wave & 1) * 16 + m, r0 = (wave >> 1) * (kC16TH / 2);
  auto ldR = [&](int r) -> bf16x8 {
    return *reinterpret_cast<const bf16x8*>(sin16 + ((kg & 1) * RP + r * RC + x + (kg >> 1)) * 8);
  };
  auto ldD = [&](int r) -> bf16x4 {
    return *reinterpret_cast<const bf16x4*>(sin16 + ((kg >> 1) * RP + r * RC + x + 2) * 8 +
                                            (kg & 1) * 4);
  };
  bf16x8 R0 = ldR(r0), R1 = ldR(r0 + 1);
  bf16x4 D0 = ldD(r0), D1 = ldD(r0 + 1);
  const int gx = X0 + x;
#pragma unroll
  for (int i = 0; i < kC16TH / 2; ++i) {
    const bf16x8 R2 = ldR(r0 + i + 2);
    const bf16x4 D2 = ldD(r0 + i + 2);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma32(wr[0], R0, acc);
    acc = mfma32(wr[1], R1, acc);
    acc = mfma32(wr[2], R2, acc);
    asm volatile("s_nop 7\n\ts_nop 7" : "+v"(acc));   // as in the fused kernel's layer 2
    acc = mfma16(wd[0], D0, acc);
    acc = mfma16(wd[1], D1, acc);
    acc = mfma16(wd[2], D2, acc);
    const int gy = Y0 + r0 + i;
    if (gy < H && gx < W)
      store_c16(acc, bs, mask != nullptr, mw[i], relu, out16, ((size_t)b * H + gy) * W + gx, kg);
    R0 = R1;
    R1 = R2;
    D0 = D1;
    D1 = D2;
  }
}

// Weight and bias gradients of a convolution in the forward convention
// out[p][co] = sum_{ci, tap} w[co][ci][tap] in[p + off(tap)][ci]:
//   dw[co][ci][tap] = sum_p dz[p][co] in[p + off(tap)][ci],   db[co] = sum_p dz[p][co].
// dz has COUT channels (FP32 image if 1, BF16 NHWC if 16); in has CIN channels (same rule).
// Each block of the weight-gradient kernels below covers 16 image rows x 64 columns of one
// slice and writes its sums to partial[block][COUT * CIN * 9 + COUT] (index (co CIN + ci) 9 +
// tap, then the bias gradients); the blocks' sums are then added in a fixed order.

// out[o] = sum over blocks of partial[block][o], fixed order, accumulated in double.
// Weight and bias gradients of the 16 -> 16 convolution on the matrix cores, for the blocks
// and partial layout above: dw[co][ci][tap] = sum_p dz[p][co] in[p + off(tap)][ci]
// as 16x16x32 BF16 products with A[co][k] = dz at 32 consecutive pixels of a row and B[k][ci] =
// the input at the same pixels moved by the tap (products of BF16 values are exact, sums are
// FP32), and db[co] = sum_p dz[p][co] as one more product against B = 1.  A block covers 16 rows
// x 64 columns of one slice in two stages of 8 rows: the stage's dz rows and input rows (one
// above and one below, columns -2 .. 65, zero outside the image) go to LDS channel-major, one
// row of pixels per channel, so that a lane's 8 pixels of one channel are one 16-byte read;
// the input one column left or right (dx = 0, 2) comes from that read and a neighbouring word
// by funnel shifts.  Wave w takes rows w and w + 4 of each stage; the four waves' sums are
// added in wave order at the end.
constexpr int kWgStage = 8;
constexpr int kWgXP = 88;   // input plane row: element 8 + xx for column xx (16-byte aligned reads)
constexpr int kWgDP = 72;   // dz plane row: element xx
__global__ void __launch_bounds__(256) cnn_wgrad16_kernel(const uint16_t* __restrict__ dz16,
                                                          const uint16_t* __restrict__ in16,
                                                          float* __restrict__ partial, int H,
                                                          int W, int rows) {
  constexpr int XS = 64, XR = kWgStage + 2, NW = 16 * 16 * 9, NOUT = NW + 16;
  constexpr int XWORDS = XR * 16 * kWgXP / 2, DWORDS = kWgStage * 16 * kWgDP / 2;
  static_assert(XWORDS + DWORDS >= 4 * 10 * 64 * 4, "the wave sums fit in the staging area");
  __shared__ __align__(16) uint32_t sxd[XWORDS + DWORDS];
  uint32_t* sx = sxd;
  uint32_t* sd = sxd + XWORDS;
  const int cols = W / XS;
  const int nrb = (H + rows - 1) / rows;
  const int rb = blockIdx.x % nrb, rest = blockIdx.x / nrb;
  const int cb = rest % cols, b = rest / cols;
  const int x0 = cb * XS;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int m = lane & 15, kg = lane >> 4;
  // channel 8 h + j of two pixels as one word (the left pixel in the low half)
  auto put8 = [](uint32_t* dst, int stride_words, const uint4& v0, const uint4& v1) {
    const uint32_t a[4] = {v0.x, v0.y, v0.z, v0.w}, c[4] = {v1.x, v1.y, v1.z, v1.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      dst[(2 * k) * stride_words] = (a[k] & 0xffffu) | (c[k] << 16);
      dst[(2 * k + 1) * stride_words] = (a[k] >> 16) | (c[k] & 0xffff0000u);
    }
  };
  f32x4 acc[9], accb = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};
  const short one = 0x3f80;   // BF16 1.0
  const bf16x8 ones = {one, one, one, one, one, one, one, one};
  const int y0 = rb * rows, y1 = min(H, y0 + rows);
  for (int ys = y0; ys < y1; ys += kWgStage) {
    const int ny = min(kWgStage, y1 - ys);
    __syncthreads();   // the previous stage's reads are done
    // input rows ys - 1 .. ys + 8, column pairs (xx, xx + 1) for xx = -2, 0, .., 64
    struct Pair {
      uint4 a, c;
    };
    stage_block<XR * 34 * 2>(
        tid,
        [&](int e) {
          const int h = e & 1, q = e >> 1, r = q / 34, xx = 2 * (q - r * 34) - 2;
          const int gy = ys - 1 + r, gx = x0 + xx;
          Pair v = {make_uint4(0u, 0u, 0u, 0u), make_uint4(0u, 0u, 0u, 0u)};
          if (gy >= 0 && gy < H) {
            const uint16_t* src = in16 + (((size_t)b * H + gy) * W + gx) * 16 + 8 * h;
            if (gx >= 0 && gx < W) v.a = *reinterpret_cast<const uint4*>(src);
            if (gx + 1 >= 0 && gx + 1 < W) v.c = *reinterpret_cast<const uint4*>(src + 16);
          }
          return v;
        },
        [&](int e, const Pair& v) {
          const int h = e & 1, q = e >> 1, r = q / 34, xx = 2 * (q - r * 34) - 2;
          put8(sx + ((r * 16 + 8 * h) * kWgXP + 8 + xx) / 2, kWgXP / 2, v.a, v.c);
        });
    // dz rows ys .. ys + ny - 1, column pairs (xx, xx + 1) for xx = 0, 2, .., 62
    stage_block<kWgStage * 32 * 2>(
        tid,
        [&](int e) {
          const int h = e & 1, q = e >> 1, r = q >> 5, xx = 2 * (q & 31);
          Pair v = {make_uint4(0u, 0u, 0u, 0u), make_uint4(0u, 0u, 0u, 0u)};
          if (r < ny) {
            const uint16_t* src = dz16 + (((size_t)b * H + ys + r) * W + x0 + xx) * 16 + 8 * h;
            v.a = *reinterpret_cast<const uint4*>(src);
            v.c = *reinterpret_cast<const uint4*>(src + 16);
          }
          return v;
        },
        [&](int e, const Pair& v) {
          const int h = e & 1, q = e >> 1, r = q >> 5, xx = 2 * (q & 31);
          put8(sd + ((r * 16 + 8 * h) * kWgDP + xx) / 2, kWgDP / 2, v.a, v.c);
        });
    __syncthreads();
    for (int rr = wave; rr < ny; rr += 4) {
#pragma unroll
      for (int ch = 0; ch < 2; ++ch) {
        const int p0 = 8 * kg + 32 * ch;   // this lane's 8 pixels: p0 .. p0 + 7
        const bf16x8 A = *reinterpret_cast<const bf16x8*>(sd + ((rr * 16 + m) * kWgDP + p0) / 2);
        accb = mfma32(A, ones, accb);
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
          const uint32_t* xr = sx + ((rr + dy) * 16 + m) * (kWgXP / 2) + 4 + p0 / 2;
          const uint4 V = *reinterpret_cast<const uint4*>(xr);
          const uint32_t prev = xr[-1], next = xr[4];   // pixels p0 - 2, p0 - 1 and p0 + 8, + 9
          const uint32_t s01 = __builtin_amdgcn_alignbit(V.y, V.x, 16);
          const uint32_t s12 = __builtin_amdgcn_alignbit(V.z, V.y, 16);
          const uint32_t s23 = __builtin_amdgcn_alignbit(V.w, V.z, 16);
          const uint4 L = make_uint4(__builtin_amdgcn_alignbit(V.x, prev, 16), s01, s12, s23);
          const uint4 R = make_uint4(s01, s12, s23, __builtin_amdgcn_alignbit(next, V.w, 16));
          acc[3 * dy + 0] = mfma32(A, __builtin_bit_cast(bf16x8, L), acc[3 * dy + 0]);
          acc[3 * dy + 1] = mfma32(A, __builtin_bit_cast(bf16x8, V), acc[3 * dy + 1]);
          acc[3 * dy + 2] = mfma32(A, __builtin_bit_cast(bf16x8, R), acc[3 * dy + 2]);
        }
      }
    }
  }
  // lane (m, kg) holds co = 4 kg + i, ci = m of each sum; add the waves' sums in wave order
  __syncthreads();
  float4* red = reinterpret_cast<float4*>(sxd);
#pragma unroll
  for (int k = 0; k < 9; ++k)
    red[(wave * 10 + k) * 64 + lane] = make_float4(acc[k][0], acc[k][1], acc[k][2], acc[k][3]);
  red[(wave * 10 + 9) * 64 + lane] = make_float4(accb[0], accb[1], accb[2], accb[3]);
  __syncthreads();
  const float* redf = reinterpret_cast<const float*>(sxd);
  const int co = tid >> 4, ci = tid & 15, src_lane = 16 * (co >> 2) + ci, i = co & 3;
  float* dst = partial + (size_t)blockIdx.x * NOUT;
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    if (k == 9 && ci != 0) break;
    float v = 0.f;
#pragma unroll
    for (int w = 0; w < 4; ++w) v += redf[((w * 10 + k) * 64 + src_lane) * 4 + i];
    if (k < 9) dst[(co * 16 + ci) * 9 + k] = v;
    else dst[NW + co] = v;
  }
}

// Weight and bias gradients of the single-channel layers on the FP32 matrix cores
// (16x16x4 steps, FP32 operands: the FP32 output gradient and image stay unrounded), for the
// blocks and partial layout above (16 rows x 64 columns of one slice).  A step
// takes 4 consecutive pixels of a row as K; lane (m, kg) holds A[m][kg] and B[kg][m].
//   1 -> 16: A[co][k] = dz[p_k][co], B[k][t] = in[p_k + off(t)] for taps t < 9 and B[k][9] = 1,
//     so D[co][t] accumulates dw[co][0][t] and D[co][9] the bias gradient.
//   16 -> 1: with q = p + off(t), dw[0][ci][t] = sum_q dz[q - off(t)] in[q][ci]: A[t][k] =
//     dz[q_k - off(t)] (dz zero outside the block's pixels), B[k][ci] = in[q_k][ci] over the
//     block's pixels and their one-pixel border, so D[t][ci] accumulates dw[0][ci][t]; the
//     centre tap's lanes (A = dz[q]) also add up the bias gradient.
// The whole block is staged in LDS at once; wave w takes every fourth row from its w-th, and
// the four waves' sums are added in wave order.
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) cnn_wgrad1_kernel(const float* __restrict__ dz32,
                                                         const uint16_t* __restrict__ dz16,
                                                         const float* __restrict__ in32,
                                                         const uint16_t* __restrict__ in16,
                                                         float* __restrict__ partial, int H,
                                                         int W) {
  static_assert((CIN == 1 && COUT == 16) || (CIN == 16 && COUT == 1), "single-channel layers");
  constexpr int XS = 64, RB = 16, NW = COUT * CIN * 9, NOUT = NW + COUT;
  constexpr bool kIn1 = CIN == 1;
  // 1 -> 16: input FP32 [RB + 2][68] (rows y0 - 1 .., columns x0 - 1 ..), dz BF16 [RB][64][16]
  // 16 -> 1: input BF16 [RB + 2][68][16] (rows y0 - 1 .., columns x0 - 1 ..), dz FP32
  //          [RB + 4][72] (rows y0 - 2 .., columns x0 - 2 ..)
  constexpr int XC = 68;
  constexpr int IN_BYTES = kIn1 ? (RB + 2) * XC * 4 : (RB + 2) * XC * 16 * 2;
  constexpr int DZ_BYTES = kIn1 ? RB * XS * 16 * 2 : (RB + 4) * 72 * 4;
  static_assert(IN_BYTES % 16 == 0 && IN_BYTES + DZ_BYTES >= (4 * 64 * 4 + 16) * 4,
                "aligned areas; the wave sums fit");
  __shared__ __align__(16) unsigned char smem[IN_BYTES + DZ_BYTES];
  const int nrb = (H + RB - 1) / RB, cols = W / XS;
  const int rb = blockIdx.x % nrb, rest = blockIdx.x / nrb;
  const int cb = rest % cols, b = rest / cols;
  const int x0 = cb * XS, y0 = rb * RB, ny = min(RB, H - y0);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int m = lane & 15, kg = lane >> 4;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;
  if constexpr (kIn1) {
    float* sx = reinterpret_cast<float*>(smem);
    uint16_t* sdz = reinterpret_cast<uint16_t*>(smem + IN_BYTES);
    stage_block<(RB + 2) * XC>(
        tid,
        [&](int e) {
          const int r = e / XC, c = e - r * XC, gy = y0 - 1 + r, gx = x0 - 1 + c;
          return (c < XS + 2 && gy >= 0 && gy < H && gx >= 0 && gx < W)
                     ? in32[((size_t)b * H + gy) * W + gx] : 0.f;
        },
        [&](int e, float v) { sx[e] = v; });
    stage_block<RB * XS * 2>(
        tid,
        [&](int e) {
          const int r = e >> 7, px = (e >> 1) & 63, h = e & 1;
          uint4 v = make_uint4(0u, 0u, 0u, 0u);
          if (r < ny)
            v = *reinterpret_cast<const uint4*>(
                dz16 + (((size_t)b * H + y0 + r) * W + x0 + px) * 16 + 8 * h);
          return v;
        },
        [&](int e, const uint4& v) {
          const int r = e >> 7, px = (e >> 1) & 63, h = e & 1;
          *reinterpret_cast<uint4*>(sdz + (r * XS + px) * 16 + 8 * h) = v;
        });
    __syncthreads();
    const int dy = m / 3, dx = m % 3;
    for (int rr = wave; rr < ny; rr += 4) {
#pragma unroll 4
      for (int g = 0; g < XS / 4; ++g) {
        const int p = 4 * g + kg;
        const float a = bf2f(sdz[(rr * XS + p) * 16 + m]);
        const float bv = m < 9 ? sx[(rr + dy) * XC + p + dx] : (m == 9 ? 1.f : 0.f);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv, acc, 0, 0, 0);
      }
    }
  } else {
    uint16_t* sx = reinterpret_cast<uint16_t*>(smem);
    float* sdz = reinterpret_cast<float*>(smem + IN_BYTES);
    stage_block<(RB + 2) * XC * 2>(
        tid,
        [&](int e) {
          const int q = e >> 1, h = e & 1, r = q / XC, c = q - r * XC;
          const int gy = y0 - 1 + r, gx = x0 - 1 + c;
          uint4 v = make_uint4(0u, 0u, 0u, 0u);
          if (gy >= 0 && gy < H && gx >= 0 && gx < W)
            v = *reinterpret_cast<const uint4*>(in16 + (((size_t)b * H + gy) * W + gx) * 16 +
                                                8 * h);
          return v;
        },
        [&](int e, const uint4& v) { *reinterpret_cast<uint4*>(sx + e * 8) = v; });
    // the block's own pixels only: rows y0 .. y0 + ny - 1, columns x0 .. x0 + 63
    stage_block<(RB + 4) * 72>(
        tid,
        [&](int e) {
          const int r = e / 72, c = e - r * 72;
          return (r >= 2 && r < 2 + ny && c >= 2 && c < 2 + XS)
                     ? dz32[((size_t)b * H + y0 - 2 + r) * W + x0 - 2 + c] : 0.f;
        },
        [&](int e, float v) { sdz[e] = v; });
    __syncthreads();
    const int dy = m / 3, dx = m % 3;
    // input rows rr = 0 .. ny + 1 (image rows y0 - 1 ..), 17 groups of 4 columns (x0 - 1 ..)
    for (int rr = wave; rr < ny + 2; rr += 4) {
#pragma unroll 4
      for (int g = 0; g < XC / 4; ++g) {
        const int qc = 4 * g + kg;
        const float bv = bf2f(sx[(rr * XC + qc) * 16 + m]);
        const float a = m < 9 ? sdz[(rr - dy + 2) * 72 + qc - dx + 2] : 0.f;
        if (m == 4) bsum += a;
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv, acc, 0, 0, 0);
      }
    }
  }
  // the waves' sums, added in wave order (lane (m, kg) holds D[4 kg + i][m])
  __syncthreads();
  float* red = reinterpret_cast<float*>(smem);
  *reinterpret_cast<float4*>(red + (wave * 64 + lane) * 4) = make_float4(acc[0], acc[1], acc[2],
                                                                         acc[3]);
  if (!kIn1 && m == 4) red[4 * 64 * 4 + wave * 4 + kg] = bsum;
  __syncthreads();
  if (tid < NOUT) {
    int row, col;   // of D
    if constexpr (kIn1) {
      row = tid < NW ? tid / 9 : tid - NW;   // co
      col = tid < NW ? tid % 9 : 9;          // tap, or the ones column
    } else {
      row = tid % 9;                         // tap
      col = tid / 9;                         // ci
    }
    float v = 0.f;
    if (kIn1 || tid < NW) {
      const int src = 16 * (row >> 2) + col, i = row & 3;
#pragma unroll
      for (int w = 0; w < 4; ++w) v += red[(w * 64 + src) * 4 + i];
    } else {
#pragma unroll
      for (int k = 0; k < 16; ++k) v += red[4 * 64 * 4 + k];
    }
    partial[(size_t)blockIdx.x * NOUT + tid] = v;
  }
}

// The blocks' sums added per output in a fixed order, in two steps.  First, block (g, c) takes
// outputs 64 g .. + 63 and the chunk c of kWgChunk blocks: wave w adds blocks w, w + 4, .. of
// the chunk (a wave reads 64 consecutive outputs of a block, 256 bytes; all its loads issued
// before the sums), in FP64, and the four waves' sums are added in wave order.  Then each
// output adds its chunks' sums in chunk order (loaded 32 at a time) and is rounded to FP32 once.
constexpr int kWgChunk = 32;
__global__ void __launch_bounds__(256) cnn_reduce_blocks_kernel(const float* __restrict__ partial,
                                                                double* __restrict__ chunk_sums,
                                                                int blocks, int nout) {
  __shared__ double sh[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int o = blockIdx.x * 64 + lane, c = blockIdx.y;
  const int b0 = c * kWgChunk;
  float v[kWgChunk / 4];
#pragma unroll
  for (int j = 0; j < kWgChunk / 4; ++j) {
    const int blk = b0 + w + 4 * j;
    v[j] = (o < nout && blk < blocks) ? partial[(size_t)blk * nout + o] : 0.f;
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < kWgChunk / 4; ++j) s += (double)v[j];
  sh[w][lane] = s;
  __syncthreads();
  if (w == 0 && o < nout)
    chunk_sums[(size_t)c * nout + o] = ((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane];
}

__global__ void __launch_bounds__(256) cnn_reduce_chunks_kernel(const double* __restrict__ chunk_sums,
                                                                float* __restrict__ out, int chunks,
                                                                int nout) {
  const int o = blockIdx.x * 256 + threadIdx.x;
  if (o >= nout) return;
  double s = 0.0;
  for (int c0 = 0; c0 < chunks; c0 += 32) {
    double v[32];
#pragma unroll
    for (int j = 0; j < 32; ++j)
      v[j] = c0 + j < chunks ? chunk_sums[(size_t)(c0 + j) * nout + o] : 0.0;
#pragma unroll
    for (int j = 0; j < 32; ++j) s += v[j];
  }
  out[o] = (float)s;
}

// ---- the whole network in one launch (inference) ----------------------------------------------
// out = x + conv3(relu(conv2(relu(conv1(x) + b1)) + b2)) + b3 over tiles of TH x TW output
// pixels.  A block loads the x region the tile depends on (three pixels of halo on each
// side, zero outside the image) into LDS, computes h1 over the tile plus two pixels of halo
// (BF16 in LDS, zero outside the image: the zero padding of the next layer) and h2 over the
// tile plus one, whose per-tap partials for layer 3 go to LDS instead of h2 itself, and writes
// the tile.  Each layer issues the same matrix-core operations with the same operands as the
// per-layer kernels (same K order, same BF16 roundings, bias then ReLU, the partials summed in
// the same order, then the residual), so the image equals the three separate launches bit for
// bit; only h1 and h2 never go to HBM.  A group is 16 pixels (layer 1: consecutive in the
// region's row-major order; layer 2: 16 columns of one row); lane (m, kg) of a wave ends with
// channels 4 kg .. + 3 of pixel m.  In LDS the 16 channels of a pixel are split in two planes
// of 8 (16 bytes per pixel and plane): the 16 lanes that read one operand part then read
// consecutive words.  The tile is 30 columns wide so that h2's rows are 32: two segments of
// 16 columns, down which layer 2's waves walk (the header's K order makes one window row's
// operands serve the three output rows that use it).
template <int TH, int TW>
struct FusedTile {
  static constexpr int XR = TH + 6, XC = TW + 6;         // x region
  static constexpr int H1R = TH + 4, H1C = TW + 4;       // h1 region
  static constexpr int H2R = TH + 2, H2C = TW + 2;       // h2 region
  static constexpr int H1Px = H1R * H1C, H2Px = H2R * H2C;
  // h1 is computed in whole groups of 16 pixels (the last group's extra pixels are never read)
  static constexpr int H1Groups = (H1Px + 15) / 16, H1Store = H1Groups * 16;
  static constexpr int H2Store = H2Px;
  static_assert(H2C == 32 && H2R % 2 == 0, "h2 rows of two 16-column segments, rows split in two");
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
  __shared__ __align__(16) uint16_t sh1[2 * T::H1Store * 8];
  __shared__ float sp3[9 * T::H2Store];              // layer 3's per-tap partials of h2
  __shared__ float sdrop[256];                       // where lanes without a tap write
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int m = lane & 15, kg = lane >> 4;
  const bf16x4 w1op = reinterpret_cast<const bf16x4*>(w1)[lane];
  bf16x8 w2r[3];
  bf16x4 w2d[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    w2r[s] = w2[s * 64 + lane];
    w2d[s] = reinterpret_cast<const bf16x4*>(w2)[3 * 128 + s * 64 + lane];
  }
  const bf16x4 w3t = reinterpret_cast<const bf16x4*>(w3)[lane];   // taps x channels
  float bias1[4], bias2[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    bias1[i] = b1[4 * kg + i];
    bias2[i] = b2[4 * kg + i];
  }
  const float bias3 = b3[0];
  // layer 1: lane group kg < 3 reads row kg of the 3 x 3 window; group 3 reads row 2 again,
  // which adds nothing: its packed weights (and every fourth one) are zero, and the x region
  // holds finite values
  const int x_row = min(kg, 2) * T::XC;
  // The weights and biases are waited for here, before the tile loop: an empty asm that reads
  // them makes the compiler complete their loads once, so that inside the loop no wait for
  // them also waits for the next tile's x loads, which are issued later.
  asm volatile("" ::"v"(w1op), "v"(w2r[0]), "v"(w2r[1]), "v"(w2r[2]), "v"(w2d[0]), "v"(w2d[1]),
               "v"(w2d[2]));
  asm volatile("" ::"v"(w3t));
  asm volatile("" ::"v"(bias1[0]), "v"(bias1[1]), "v"(bias1[2]), "v"(bias1[3]), "v"(bias2[0]),
               "v"(bias2[1]), "v"(bias2[2]), "v"(bias2[3]), "v"(bias3));

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

    // Bias, BF16, ReLU of a lane's four channels of region pixel px (zero outside the image).
    auto hword = [&](const f32x4& acc, const float* bias, int px, int cols, int oy,
                     int ox) -> uint2 {
      uint2 w = pack4_bf16(acc[0] + bias[0], acc[1] + bias[1], acc[2] + bias[2],
                           acc[3] + bias[3]);
      w = make_uint2(relu_bf16x2(w.x), relu_bf16x2(w.y));
      if (!interior) {
        const int rr = px / cols, cc = px - rr * cols;
        const int gy = Y0 + oy + rr, gx = X0 + ox + cc;
        if (!(gy >= 0 && gy < H && gx >= 0 && gx < W)) w = make_uint2(0u, 0u);
      }
      return w;
    };
    // ... stored as one 8-byte word into plane kg / 2 of a region of `px_total` pixels
    auto store4 = [&](uint16_t* dst, int px_total, const f32x4& acc, const float* bias, int px,
                      int cols, int oy, int ox) {
      const uint2 w = hword(acc, bias, px, cols, oy, ox);
      *reinterpret_cast<uint2*>(dst + ((kg >> 1) * px_total + px) * 8 + (kg & 1) * 4) = w;
    };
    // h2 of pixel px is layer 3's B operand as it stands (lane group kg: channels 4 kg .. + 3):
    // one 16x16x16 step against the taps gives its nine per-tap partials, kept in LDS
    auto partials3 = [&](const f32x4& acc, int px) {
      const uint2 w = hword(acc, bias2, px, T::H2C, -1, -1);
      const f32x4 pt = mfma16(w3t, __builtin_bit_cast(bf16x4, w), f32x4{0.f, 0.f, 0.f, 0.f});
      // rows 9 .. 15 hold no tap: their lanes write into a slot of their own instead of
      // branching around the store
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float* d = 4 * kg + i < 9 ? &sp3[(4 * kg + i) * T::H2Store + px] : &sdrop[tid];
        *d = pt[i];
      }
    };

    // layer 1: x (1 channel) -> h1 (16), one 16x16x16 step per group: lane group kg holds the
    // three taps of window row min(kg, 2) (converted in pairs) and a zero
    auto a1 = [&](int p) -> bf16x4 {
      const int pc = min(p, T::H1Px - 1);   // the last group's extra pixels read the last one
      const int r = pc / T::H1C, c = pc - r * T::H1C;
      const float* xp = sxc + r * T::XC + c + x_row;
      const uint32_t w0 = pack2_bf16(xp[0], xp[1]);
      const uint32_t w1 = pack2_bf16(xp[2], 0.f);
      return __builtin_bit_cast(bf16x4, make_uint2(w0, w1));
    };
    // two groups (g, g + 4) at a time, as in layer 2
    for (int g = wave; g < T::H1Groups; g += 8) {
      const int gb = g + 4 < T::H1Groups ? g + 4 : g;
      const int pa = g * 16 + m, pb = gb * 16 + m;
      const bf16x4 aa = a1(pa), ab = a1(pb);
      f32x4 acca = {0.f, 0.f, 0.f, 0.f}, accb = {0.f, 0.f, 0.f, 0.f};
      acca = mfma16(w1op, aa, acca);
      accb = mfma16(w1op, ab, accb);
      store4(sh1, T::H1Store, acca, bias1, pa, T::H1C, -2, -2);
      store4(sh1, T::H1Store, accb, bias1, pb, T::H1C, -2, -2);
    }
    __syncthreads();   // h1 complete; the previous tile's layer 3 is done with the partials

    // layer 2: h1 (16) -> h2 (16).  The h2 region is two segments of 16 columns; wave w walks
    // segment w % 2 down half of its rows.  Output row y takes window rows y .. y + 2 of h1,
    // each as one 16x16x32 step (lane groups kg < 2: column x, kg >= 2: column x + 1, channels
    // 8 (kg % 2) ..) and one 16x16x16 step (column x + 2, channels 4 kg ..): a window row's
    // operands serve three output rows, so each row loads only its last window row.
    {
      constexpr int RPW = T::H2R / 2;
      const int x = (wave & 1) * 16 + m, y0 = (wave >> 1) * RPW;
      auto ldR = [&](int r) -> bf16x8 {
        return *reinterpret_cast<const bf16x8*>(
            sh1 + ((kg & 1) * T::H1Store + r * T::H1C + x + (kg >> 1)) * 8);
      };
      auto ldD = [&](int r) -> bf16x4 {
        return *reinterpret_cast<const bf16x4*>(
            sh1 + ((kg >> 1) * T::H1Store + r * T::H1C + x + 2) * 8 + (kg & 1) * 4);
      };
      bf16x8 R0 = ldR(y0), R1 = ldR(y0 + 1);
      bf16x4 D0 = ldD(y0), D1 = ldD(y0 + 1);
#pragma unroll
      for (int i = 0; i < RPW; ++i) {
        const bf16x8 R2 = ldR(y0 + i + 2);
        const bf16x4 D2 = ldD(y0 + i + 2);
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        __builtin_amdgcn_s_setprio(1);
        acc = mfma32(w2r[0], R0, acc);
        acc = mfma32(w2r[1], R1, acc);
        acc = mfma32(w2r[2], R2, acc);
        // a 16x16x16 step that accumulates onto a 16x16x32 step's result needs wait states
        // the compiler does not insert when the two are back to back (found by the bit-exact
        // comparison with the layer-by-layer kernel): 16 are given explicitly
        asm volatile("s_nop 7\n\ts_nop 7" : "+v"(acc));
        acc = mfma16(w2d[0], D0, acc);
        acc = mfma16(w2d[1], D1, acc);
        acc = mfma16(w2d[2], D2, acc);
        __builtin_amdgcn_s_setprio(0);
        partials3(acc, (y0 + i) * T::H2C + x);
        R0 = R1;
        R1 = R2;
        D0 = D1;
        D1 = D2;
      }
    }
    if (tn < total_tiles) store_x(sx[buf ^ 1]);
    __syncthreads();   // the partials and the next tile's x region complete

    // layer 3: each output pixel sums the partials of its nine h2 neighbours in tap order,
    // then adds the bias and the residual (two pixels per thread, a row of 32 per half wave)
    float* dst = out + (size_t)b * H * W;
#pragma unroll
    for (int k = 0; k < (TH * TW + 255) / 256; ++k) {
      const int e = tid + 256 * k;
      if (e >= TH * TW) break;
      const int r = e / TW, c = e - r * TW;
      const float* q = sp3 + r * T::H2C + c;
      float sum = q[0];
#pragma unroll
      for (int t = 1; t < 9; ++t) sum += q[t * T::H2Store + (t / 3) * T::H2C + t % 3];
      const int gy = Y0 + r, gx = X0 + c;
      if (gy < H && gx < W) dst[(size_t)gy * W + gx] = sum + bias3 + sxc[(r + 3) * T::XC + c + 3];
    }
  }
}

}  // namespace

// Output tile of the fused network: 16 x 30 pixels (49 KB of LDS per block, three per CU).  The launch is
// persistent: as many blocks as the device holds at once, each looping over tiles.
constexpr int kFuseTH = 16, kFuseTW = 30;

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
  const bf16x8* w8 = reinterpret_cast<const bf16x8*>(wop);
  int th, tw;
  if (cin == 1 && cout == 16) th = kC1TH, tw = kC1TW;
  else if (cin == 16 && cout == 16) th = kC16TH, tw = kC16TW;
  else if (cin == 16 && cout == 1) th = kC3TH, tw = kC3TW;
  else return hipErrorInvalidValue;
  const int tiles_x = (W + tw - 1) / tw, tiles_y = (H + th - 1) / th;
  const long long tiles = (long long)batch * tiles_x * tiles_y;
  if (tiles > 0x7fffffffll) return hipErrorInvalidValue;
  const dim3 grid((unsigned)tiles);
  if (cin == 1)
    hipLaunchKernelGGL(cnn_conv1_tile_kernel, grid, dim3(256), 0, stream, in32, w8, bias, mask,
                       out16, relu, H, W, tiles_x, tiles_x * tiles_y);
  else if (cout == 16)
    hipLaunchKernelGGL(cnn_conv16_tile_kernel, grid, dim3(256), 0, stream, in16, w8, bias, mask,
                       out16, relu, H, W, tiles_x, tiles_x * tiles_y);
  else
    hipLaunchKernelGGL(cnn_conv16to1_tile_kernel, grid, dim3(256), 0, stream, in16, w8, bias,
                       resid, out32, H, W, tiles_x, tiles_x * tiles_y);
  return hipGetLastError();
}

int cnn_wgrad_rows() { return 16; }

namespace {
// the partial buffer: the blocks' sums (blocks x nout floats), then from the next even float
// one FP64 sum per chunk of kWgChunk blocks and output
int64_t wgrad_block_floats(int64_t blocks, int64_t nout) { return (blocks * nout + 1) & ~1ll; }
}  // namespace

int64_t cnn_wgrad_partial_floats(int cin, int cout, int batch, int H, int W) {
  const int64_t rows = cnn_wgrad_rows();
  const int64_t blocks = (int64_t)batch * (W / 64) * ((H + rows - 1) / rows);
  const int64_t nout = cout * cin * 9 + cout;
  const int64_t chunks = (blocks + kWgChunk - 1) / kWgChunk;
  return wgrad_block_floats(blocks, nout) + 2 * chunks * nout;
}

hipError_t launch_cnn_wgrad(int cin, int cout, const float* dz32, const uint16_t* dz16,
                            const float* in32, const uint16_t* in16, float* partial, float* out,
                            int batch, int H, int W, hipStream_t stream) {
  const int rows = cnn_wgrad_rows();
  const int blocks = batch * (W / 64) * ((H + rows - 1) / rows);
  const int nout = cout * cin * 9 + cout;
  if (rows != 16) return hipErrorInvalidValue;   // the kernels' row blocks
  if (cin == 1 && cout == 16)
    hipLaunchKernelGGL((cnn_wgrad1_kernel<1, 16>), dim3(blocks), dim3(256), 0, stream, dz32, dz16,
                       in32, in16, partial, H, W);
  else if (cin == 16 && cout == 16)
    hipLaunchKernelGGL(cnn_wgrad16_kernel, dim3(blocks), dim3(256), 0, stream, dz16, in16, partial,
                       H, W, rows);
  else if (cin == 16 && cout == 1)
    hipLaunchKernelGGL((cnn_wgrad1_kernel<16, 1>), dim3(blocks), dim3(256), 0, stream, dz32, dz16,
                       in32, in16, partial, H, W);
  else
    return hipErrorInvalidValue;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int chunks = (blocks + kWgChunk - 1) / kWgChunk;
  if (chunks > 65535) return hipErrorInvalidValue;   // grid y
  double* chunk_sums = reinterpret_cast<double*>(partial + wgrad_block_floats(blocks, nout));
  hipLaunchKernelGGL(cnn_reduce_blocks_kernel, dim3((nout + 63) / 64, chunks), dim3(256), 0,
                     stream, partial, chunk_sums, blocks, nout);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(cnn_reduce_chunks_kernel, dim3((nout + 255) / 256), dim3(256), 0, stream,
                     chunk_sums, out, chunks, nout);
  return hipGetLastError();
}

}  // namespace fhtfbp
