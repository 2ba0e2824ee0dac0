// One LDS-resident pass of the transposed dyadic Fast Hough Transform (Sec. 4.4-4.5), with the
// recursive ramp-filter pair (Sec. 3, eq 9-13) fused into the first pass and the class sum
// (eq 22) fused into the last.
//
// Buffer levels.  Between passes a class is stored as N rows of N floats; at level k (strip
// height h = 2^k) row j*h + t holds pattern t of strip j.  Level n is the linogram (one strip,
// N patterns = slope indices), level 0 the class-frame image (N strips of height 1).  Going
// down one level, pattern pair (2t, 2t+1) of a strip feeds pattern t of its lower half
// unshifted and pattern t of its upper half shifted back by t and t + 1 columns.
//
// Tiles.  A pass runs F levels from k_hi down to k_lo = k_hi - F.  The 2^F patterns
// t = v 2^F + r (r < 2^F) of strip j only mix among themselves, so they form one tile: 2^F
// consecutive rows in, 2^F rows (j 2^F + i) 2^k_lo + v out.  A tile lives in LDS as full
// rows, skewed by one word every L columns so both row-parallel and chunk-parallel accesses
// avoid bank conflicts.
//
// Lazy shifts.  Rather than shifting the upper half by t, every row keeps a pending rotation
// o (stored[x] = logical[x + o]).  With the rotation of the lower half inherited and that of
// the upper half increased by t, the row of sub-strip i and pattern t carries o = t * i, so
// inside the tile the two inputs of a butterfly differ only by the parent sub-strip index J:
//     lower[x] = S[2t][x] + S[2t+1][x - J],   upper[x] = S[2t][x] + S[2t+1][x - J - 1].
// The rotations are applied when the tile is written (o = v * i; zero in the last pass).
// The butterflies are done in place (lower into the row of pattern 2t, upper into 2t+1), so
// after F levels sub-strip i sits in physical row bitreverse_F(i).
#pragma once
#include "fhtfbp_internal.h"

namespace fhtfbp {
namespace {

__device__ __forceinline__ int lds_at(int r, int c, int rs, int log2l) {
  return r * rs + c + (c >> log2l);
}

__device__ __forceinline__ int brev_bits(int v, int bits) {
  return bits == 0 ? 0 : (int)(__brev((unsigned)v) >> (32 - bits));
}

// ---- load a tile --------------------------------------------------------------------------
template <int L>
__device__ void load_tile(const PassArgs& A, float* S, int b, int q, int row0) {
  const int T = blockDim.x, tid = threadIdx.x;
  const int N = 1 << A.log2n, mask = N - 1;
  const int R = 1 << A.log2r;
  if (A.in_mode == IN_ROWS) {
    const float* src = A.in + ((size_t)(b * 4 + q) * N + row0) * N;
    // R rows of N floats are contiguous in the source only when the rows are consecutive,
    // which holds for every pass (tile rows are v 2^F + r of strip j).
    const int nvec = (R * N) >> 2;
    const float4* s4 = reinterpret_cast<const float4*>(src);
    for (int e = tid; e < nvec; e += T) {
      float4 v = s4[e];
      const int r = (e << 2) >> A.log2n, x = (e << 2) & mask;
      float* d = S + r * A.rs;
      d[x + (x >> A.log2l)] = v.x;
      d[x + 1 + ((x + 1) >> A.log2l)] = v.y;
      d[x + 2 + ((x + 2) >> A.log2l)] = v.z;
      d[x + 3 + ((x + 3) >> A.log2l)] = v.w;
    }
  } else {
    // forward transform: tile row r is frame row yf = row0 + r; tile column x is frame
    // column c = -x mod N (the mirror that turns the transposed FHT into the forward one)
    const float* img = A.in + (size_t)b * N * N;
    if (q < 2) {
      for (int e = tid; e < R * N; e += T) {
        const int r = e >> A.log2n, x = e & mask;
        const int c = (-x) & mask;
        const int col = (q == 0) ? c : (N - 1 - c);
        S[lds_at(r, x, A.rs, A.log2l)] = img[(size_t)(row0 + r) * N + col];
      }
    } else {
      for (int e = tid; e < R * N; e += T) {
        const int r = e & (R - 1), x = e >> A.log2r;
        const int c = (-x) & mask;
        const int irow = (q == 2) ? c : (N - 1 - c);
        S[lds_at(r, x, A.rs, A.log2l)] = img[(size_t)irow * N + row0 + r];
      }
    }
  }
}

// ---- recursive ramp-filter pair over every tile row (rows are linogram rows row0 + r) --------
// Work item (r, c): chunk c = positions c L .. c L + L - 1 of row r's window.  Each chunk runs
// the recursion from zero state, the true entering states come from a scan over the chunks of
// the row (lanes of one wave) with the transition matrices Phi^(L 2^j), and the response of
// the recursion to that entering state is added.  The anticausal pass is the same recursion
// run from the end of the window.
template <int L, int K>
__device__ void filter_tile(const PassArgs& A, float* S, int q, int row0) {
  const int tid = threadIdx.x;
  const int C = 1 << A.log2c;
  const int r = tid >> A.log2c, c = tid & (C - 1);
  const int N = 1 << A.log2n, mask = N - 1;
  const int t = row0 + r;
  const int g = ((q * N + t) * A.groups) / (4 * N);
  const float* cf = A.coef + (size_t)g * A.coef_stride;
  float bk[K], ak[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    bk[k] = cf[k];
    ak[k] = cf[K + k];
  }
  const float* phi = cf + 2 * K;
  const int sig = A.sigma[t];
  const float ct = A.scale[t];
  const int base = c * L;
  float* row = S + r * A.rs;
  auto at = [&](int i) -> float {   // window position i -> LDS value
    const int s = (sig + i) & mask;
    return row[s + (s >> A.log2l)];
  };
  float x[L];
#pragma unroll
  for (int i = 0; i < L; ++i) x[i] = at(base + i);
  float xp[K], xn[K];   // window samples before / after the chunk (zero outside the window)
#pragma unroll
  for (int k = 1; k < K; ++k) {
    xp[k] = (base - k >= 0) ? at(base - k) : 0.f;
    xn[k] = (base + L - 1 + k < N) ? at(base + L - 1 + k) : 0.f;
  }
  xp[0] = 0.f;
  xn[0] = 0.f;

  float y[L];
  float st[K];
  // causal pass, zero entering state
#pragma unroll
  for (int k = 0; k < K; ++k) st[k] = 0.f;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) acc = fmaf(bk[k], (i - k >= 0) ? x[i - k] : xp[k - i], acc);
#pragma unroll
    for (int k = 0; k < K; ++k) acc = fmaf(-ak[k], st[k], acc);
    y[i] = acc;
#pragma unroll
    for (int k = K - 1; k > 0; --k) st[k] = st[k - 1];
    st[0] = acc;
  }
  // inclusive scan of the end states over the chunks to the left
  {
    float tv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) tv[k] = st[k];
    for (int j = 0; (1 << j) < C; ++j) {
      const int d = 1 << j;
      float u[K];
#pragma unroll
      for (int k = 0; k < K; ++k) u[k] = __shfl_up(tv[k], d, C);
      if (c >= d) {
        const float* P = phi + j * K * K;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          float acc = tv[k];
#pragma unroll
          for (int m = 0; m < K; ++m) acc = fmaf(P[k * K + m], u[m], acc);
          tv[k] = acc;
        }
      }
    }
    float sin_[K];
#pragma unroll
    for (int k = 0; k < K; ++k) sin_[k] = (C > 1) ? __shfl_up(tv[k], 1, C) : 0.f;
    if (c == 0) {
#pragma unroll
      for (int k = 0; k < K; ++k) sin_[k] = 0.f;
    }
    // response of the recursion to the entering state
#pragma unroll
    for (int i = 0; i < L; ++i) {
      float z = 0.f;
#pragma unroll
      for (int k = 0; k < K; ++k) z = fmaf(-ak[k], sin_[k], z);
      y[i] += z;
#pragma unroll
      for (int k = K - 1; k > 0; --k) sin_[k] = sin_[k - 1];
      sin_[0] = z;
    }
  }
  // anticausal pass, zero entering state, added into y as it goes
#pragma unroll
  for (int k = 0; k < K; ++k) st[k] = 0.f;
#pragma unroll
  for (int i = L - 1; i >= 0; --i) {
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) acc = fmaf(bk[k], (i + k < L) ? x[i + k] : xn[i + k - L + 1], acc);
#pragma unroll
    for (int k = 0; k < K; ++k) acc = fmaf(-ak[k], st[k], acc);
    y[i] += acc;
#pragma unroll
    for (int k = K - 1; k > 0; --k) st[k] = st[k - 1];
    st[0] = acc;
  }
  {
    float tv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) tv[k] = st[k];
    for (int j = 0; (1 << j) < C; ++j) {
      const int d = 1 << j;
      float u[K];
#pragma unroll
      for (int k = 0; k < K; ++k) u[k] = __shfl_down(tv[k], d, C);
      if (c + d < C) {
        const float* P = phi + j * K * K;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          float acc = tv[k];
#pragma unroll
          for (int m = 0; m < K; ++m) acc = fmaf(P[k * K + m], u[m], acc);
          tv[k] = acc;
        }
      }
    }
    float sin_[K];
#pragma unroll
    for (int k = 0; k < K; ++k) sin_[k] = (C > 1) ? __shfl_down(tv[k], 1, C) : 0.f;
    if (c == C - 1) {
#pragma unroll
      for (int k = 0; k < K; ++k) sin_[k] = 0.f;
    }
#pragma unroll
    for (int i = L - 1; i >= 0; --i) {
      float z = 0.f;
#pragma unroll
      for (int k = 0; k < K; ++k) z = fmaf(-ak[k], sin_[k], z);
      y[i] += z;
#pragma unroll
      for (int k = K - 1; k > 0; --k) sin_[k] = sin_[k - 1];
      sin_[0] = z;
    }
  }
  __syncthreads();   // every chunk has read its samples and its neighbours' halo
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const int s = (sig + base + i) & mask;
    row[s + (s >> A.log2l)] = ct * y[i];
  }
  __syncthreads();
}

// ---- F in-place transposed butterfly levels with lazy shifts ---------------------------------
// Streaming form (N >= 64): the work of a level is split into units (row pair, column segment
// of W = N / S columns), S = max(1, waves / pairs), and every wave walks its units from the top
// 64-column block of the segment down.  A shifted read (x - J or x - J - 1, J < 64) then lands
// in a block of the segment not yet overwritten, except at the lowest block, where it reaches
// into the 64 columns below the segment (cyclically); those are copied to registers before a
// barrier, ahead of any write.  Two barriers per level, a handful of registers.
__device__ __forceinline__ void level_stream(const PassArgs& A, float* S, float* below, int l) {
  const int N = 1 << A.log2n, mask = N - 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int waves = blockDim.x >> 6;
  const int log2p = A.log2r - 1;                       // pairs = 2^log2p
  const int segs = waves > (1 << log2p) ? waves >> log2p : 1;
  const int W = N / segs;
  const int units = ((1 << log2p) * segs) / waves;     // units per wave
  for (int u = 0; u < units; ++u) {
    const int unit = wave + u * waves;                   // unit = pair * segs + seg
    const int pair = unit / segs, seg = unit - pair * segs;
    const int ib = pair & ((1 << l) - 1), pp = pair >> l;
    const int r1 = ((pp << (l + 1)) | ib) | (1 << l);
    const int xb = (seg * W - 64 + lane) & mask;
    below[unit * 64 + lane] = S[lds_at(r1, xb, A.rs, A.log2l)];
  }
  __syncthreads();
  for (int u = 0; u < units; ++u) {
    const int unit = wave + u * waves;
    const int pair = unit / segs, seg = unit - pair * segs;
    const int ib = pair & ((1 << l) - 1), pp = pair >> l;
    const int r0 = (pp << (l + 1)) | ib, r1 = r0 | (1 << l);
    const int J = brev_bits(ib, l);
    float* row0 = S + r0 * A.rs;
    float* row1 = S + r1 * A.rs;
    const int x0 = seg * W;
    for (int blk = (W >> 6) - 1; blk >= 0; --blk) {
      const int x = x0 + (blk << 6) + lane;
      const int x1 = x - J, x2 = x - J - 1;
      const float v0 = row0[x + (x >> A.log2l)];
      float v1, v2;
      if (blk > 0) {
        v1 = row1[x1 + (x1 >> A.log2l)];
        v2 = row1[x2 + (x2 >> A.log2l)];
      } else {
        // columns below x0 come from the copy (entry k holds column x0 - 64 + k)
        const int m1 = x1 & mask, m2 = x2 & mask;
        v1 = (x1 >= x0) ? row1[m1 + (m1 >> A.log2l)] : below[unit * 64 + ((x1 - x0 + 64) & 63)];
        v2 = (x2 >= x0) ? row1[m2 + (m2 >> A.log2l)] : below[unit * 64 + ((x2 - x0 + 64) & 63)];
      }
      row0[x + (x >> A.log2l)] = v0 + v1;
      row1[x + (x >> A.log2l)] = v0 + v2;
    }
  }
}

// Two-phase form for rows shorter than 64 columns: every thread reads all its butterfly inputs,
// then writes.
template <int L>
__device__ void level_two_phase(const PassArgs& A, float* S, int l) {
  const int T = blockDim.x, tid = threadIdx.x;
  const int N = 1 << A.log2n, mask = N - 1;
  constexpr int NB = (L / 2 > 0) ? L / 2 : 1;
  float va[NB], vb[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const int e = tid + k * T;
    const int pair = e >> A.log2n, x = e & mask;
    const int ib = pair & ((1 << l) - 1), pp = pair >> l;
    const int r0 = (pp << (l + 1)) | ib, r1 = r0 | (1 << l);
    const int J = brev_bits(ib, l);
    const float v0 = S[lds_at(r0, x, A.rs, A.log2l)];
    const float v1 = S[lds_at(r1, (x - J) & mask, A.rs, A.log2l)];
    const float v2 = S[lds_at(r1, (x - J - 1) & mask, A.rs, A.log2l)];
    va[k] = v0 + v1;
    vb[k] = v0 + v2;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const int e = tid + k * T;
    const int pair = e >> A.log2n, x = e & mask;
    const int ib = pair & ((1 << l) - 1), pp = pair >> l;
    const int r0 = (pp << (l + 1)) | ib, r1 = r0 | (1 << l);
    S[lds_at(r0, x, A.rs, A.log2l)] = va[k];
    S[lds_at(r1, x, A.rs, A.log2l)] = vb[k];
  }
}

// STREAM: streaming form (rows of 64 columns or more), else two-phase.  `below` is the LDS area
// after the tile (64 floats per streaming unit).
template <int L, bool STREAM>
__device__ void run_levels(const PassArgs& A, float* S) {
  float* below = S + (1 << A.log2r) * A.rs;
  for (int l = 0; l < A.levels; ++l) {
    if constexpr (STREAM) level_stream(A, S, below, l);
    else level_two_phase<L>(A, S, l);
    __syncthreads();
  }
}

template <int L, int K, bool STREAM>
__device__ void process_class(const PassArgs& A, float* S, int b, int q, int row0) {
  load_tile<L>(A, S, b, q, row0);
  __syncthreads();
  if constexpr (K > 0) filter_tile<L, K>(A, S, q, row0);
  run_levels<L, STREAM>(A, S);
}

// Passes that keep the four classes apart: the first and middle passes of the back projection,
// every pass of the forward transform, and the filter alone (OUT_SAME).
template <int L, int K, bool STREAM>
__global__ void __launch_bounds__(1024) fht_rows_kernel(PassArgs A) {
  extern __shared__ float S[];
  const int T = blockDim.x, tid = threadIdx.x;
  const int N = 1 << A.log2n, mask = N - 1;
  const int R = 1 << A.log2r;
  const int F = A.levels;
  const int tiles = N >> A.log2r;          // tiles per class
  const int k_lo = A.k_hi - F;
  const int vbits = A.k_hi - F;            // tile index = j * 2^vbits + v
  const int tile = blockIdx.x % tiles;
  const int bq = blockIdx.x / tiles;
  const int b = bq >> 2, q = bq & 3;
  int row0, j = 0, v = 0;
  if (A.out_mode == OUT_SAME) {
    row0 = tile * R;
  } else {
    j = tile >> vbits;
    v = tile & ((1 << vbits) - 1);
    row0 = (j << A.k_hi) + (v << F);
  }
  process_class<L, K, STREAM>(A, S, b, q, row0);

  float* dst = A.out + (size_t)(b * 4 + q) * N * N;
  if (A.out_mode == OUT_SAME) {
    for (int e = tid; e < (R * N) >> 2; e += T) {
      const int rho = (e << 2) >> A.log2n, x = (e << 2) & mask;
      float4 w;
      w.x = S[lds_at(rho, x, A.rs, A.log2l)];
      w.y = S[lds_at(rho, x + 1, A.rs, A.log2l)];
      w.z = S[lds_at(rho, x + 2, A.rs, A.log2l)];
      w.w = S[lds_at(rho, x + 3, A.rs, A.log2l)];
      *reinterpret_cast<float4*>(dst + (size_t)(row0 + rho) * N + x) = w;
    }
  } else if (A.out_mode == OUT_ROWS) {
    for (int e = tid; e < (R * N) >> 2; e += T) {
      const int rho = (e << 2) >> A.log2n, x = (e << 2) & mask;
      const int i = brev_bits(rho, F);
      const int orow = (((j << F) + i) << k_lo) + v;
      const int o = (v * i) & mask;
      float4 w;
      w.x = S[lds_at(rho, (x - o) & mask, A.rs, A.log2l)];
      w.y = S[lds_at(rho, (x + 1 - o) & mask, A.rs, A.log2l)];
      w.z = S[lds_at(rho, (x + 2 - o) & mask, A.rs, A.log2l)];
      w.w = S[lds_at(rho, (x + 3 - o) & mask, A.rs, A.log2l)];
      *reinterpret_cast<float4*>(dst + (size_t)orow * N + x) = w;
    }
  } else {  // OUT_LINO_MIRROR: last forward pass, row t = j R + i, lino[t][s] = tile[t][-s]
    for (int e = tid; e < (R * N) >> 2; e += T) {
      const int rho = (e << 2) >> A.log2n, x = (e << 2) & mask;
      const int t = row0 + brev_bits(rho, F);
      float4 w;
      w.x = S[lds_at(rho, (-x) & mask, A.rs, A.log2l)];
      w.y = S[lds_at(rho, (-x - 1) & mask, A.rs, A.log2l)];
      w.z = S[lds_at(rho, (-x - 2) & mask, A.rs, A.log2l)];
      w.w = S[lds_at(rho, (-x - 3) & mask, A.rs, A.log2l)];
      *reinterpret_cast<float4*>(dst + (size_t)t * N + x) = w;
    }
  }
}

// Last back-projection pass (k_lo = 0): one block handles tile j of a class pair and sums the
// pair in the image frame (eq 20-22).  OUT_IMG_V: classes 0 and 1 give image rows j R .. j R +
// R - 1, image[y][x] = c0[y][x] + c1[y][N-1-x].  OUT_IMG_H: classes 2 and 3 give image columns
// j R .. j R + R - 1, image[y][x] += c2[x][y] + c3[x][N-1-y] (launched after OUT_IMG_V).
template <int L, int K, bool STREAM>
__global__ void __launch_bounds__(1024) fht_combine_kernel(PassArgs A) {
  extern __shared__ float S[];
  const int T = blockDim.x, tid = threadIdx.x;
  const int N = 1 << A.log2n, mask = N - 1;
  const int R = 1 << A.log2r;
  const int F = A.levels;
  const int tiles = N >> A.log2r;
  const int b = blockIdx.x / tiles, j = blockIdx.x % tiles;
  const bool vpair = A.out_mode == OUT_IMG_V;
  const int qa = vpair ? 0 : 2;
  const int row0 = j * R;
  float keep[L];
  process_class<L, K, STREAM>(A, S, b, qa, row0);
#pragma unroll
  for (int k = 0; k < L; ++k) {
    const int e = tid + k * T;
    const int i = vpair ? (e >> A.log2n) : (e & (R - 1));
    const int c = vpair ? (e & mask) : (e >> A.log2r);
    keep[k] = S[lds_at(brev_bits(i, F), c, A.rs, A.log2l)];
  }
  __syncthreads();
  process_class<L, K, STREAM>(A, S, b, qa + 1, row0);
  float* img = A.out + (size_t)b * N * N;
  if (vpair) {
#pragma unroll
    for (int k = 0; k < L; ++k) {
      const int e = tid + k * T;
      const int i = e >> A.log2n, x = e & mask;
      img[(size_t)(row0 + i) * N + x] = keep[k] + S[lds_at(brev_bits(i, F), N - 1 - x, A.rs, A.log2l)];
    }
  } else {
#pragma unroll
    for (int k = 0; k < L; ++k) {
      const int e = tid + k * T;
      const int i = e & (R - 1), y = e >> A.log2r;
      const float v = keep[k] + S[lds_at(brev_bits(i, F), N - 1 - y, A.rs, A.log2l)];
      float* p = img + (size_t)y * N + row0 + i;
      *p = *p + v;
    }
  }
}

template <typename Kern>
hipError_t launch_kernel(Kern kern, const PassArgs& a, int blocks, int threads, size_t lds,
                         hipStream_t stream) {
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), lds, stream, a);
  return hipGetLastError();
}

template <int L, int K, bool STREAM>
hipError_t launch_lks(const PassArgs& a, int batch, hipStream_t stream) {
  const int N = 1 << a.log2n;
  const int R = 1 << a.log2r;
  const int threads = R << a.log2c;
  const size_t lds = pass_lds_bytes(a);
  const int tiles = N >> a.log2r;
  if (a.out_mode == OUT_IMG_V || a.out_mode == OUT_IMG_H) {
    if constexpr (L <= 32 || K == 0)
      return launch_kernel(fht_combine_kernel<L, K, STREAM>, a, batch * tiles, threads, lds,
                           stream);
    else
      return hipErrorInvalidValue;   // the filter runs in a combining pass only when N <= 128
  }
  return launch_kernel(fht_rows_kernel<L, K, STREAM>, a, batch * 4 * tiles, threads, lds, stream);
}

template <int L, int K>
hipError_t launch_lk(const PassArgs& a, int batch, hipStream_t stream) {
  const bool stream_form = pass_streams(a);
  if constexpr (L < 32) return launch_lks<L, K, false>(a, batch, stream);   // N < 32
  else if constexpr (L > 32) return launch_lks<L, K, true>(a, batch, stream);
  else
    return stream_form ? launch_lks<L, K, true>(a, batch, stream)
                       : launch_lks<L, K, false>(a, batch, stream);
}

}  // namespace

// Orders 5..7 run on the order-8 kernels with zero-padded coefficients (bit-identical: the
// padded taps add exact zeros).
template <int L>
hipError_t launch_pass_l(const PassArgs& a, int batch, hipStream_t stream) {
  switch (a.order) {
    case 0: return launch_lk<L, 0>(a, batch, stream);
    case 1: return launch_lk<L, 1>(a, batch, stream);
    case 2: return launch_lk<L, 2>(a, batch, stream);
    case 3: return launch_lk<L, 3>(a, batch, stream);
    case 4: return launch_lk<L, 4>(a, batch, stream);
    case 8: return launch_lk<L, 8>(a, batch, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fhtfbp
