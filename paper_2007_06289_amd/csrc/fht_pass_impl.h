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
#include <type_traits>

#include "fhtfbp_internal.h"

namespace fhtfbp {

// Index of the calling wave in its block, as a wave-uniform (scalar) value: everything derived
// from it (unit, row pair, relative shift) is then computed once per wave on the scalar unit
// instead of once per lane.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }
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

// ---- first-difference numerator (orders K >= 2) -----------------------------------------------
// On entry xc[k] = x[base - 1 - k] and xa[k] = x[base + L + k] for k < K - 1 (zero outside the
// window).  Rearranged into the difference history: xc[k] = d[base - 1 - k] for k < K - 2 (the
// slot K - 2 is shifted out before it is read) and xc[K - 1] = x[base - 1], the sample the next
// difference is taken against; likewise for the anticausal half, mirrored.
template <int K>
__device__ __forceinline__ void diff_history(float* xc, float* xa) {
  const float pc = xc[0], pa = xa[0];
#pragma unroll
  for (int k = 0; k < K - 2; ++k) {
    xc[k] = xc[k] - xc[k + 1];
    xa[k] = xa[k] - xa[k + 1];
  }
  if constexpr (K >= 2) {
    xc[K - 2] = 0.f;
    xa[K - 2] = 0.f;
  }
  xc[K - 1] = pc;
  xa[K - 1] = pa;
}

// One sample of both halves: shift the differences, take the new one against the previous
// sample (xi - x[i-1] causal, xj - x[j+1] anticausal) and keep xi, xj for the next step.
template <int K>
__device__ __forceinline__ void diff_step(float* xc, float* xa, float xi, float xj) {
#pragma unroll
  for (int k = K - 2; k > 0; --k) {
    xc[k] = xc[k - 1];
    xa[k] = xa[k - 1];
  }
  xc[0] = xi - xc[K - 1];
  xa[0] = xj - xa[K - 1];
  xc[K - 1] = xi;
  xa[K - 1] = xj;
}

// ---- recursive ramp-filter pair over every tile row (rows are linogram rows row0 + r) --------
// Work item (r, c): chunk c = positions c L .. c L + L - 1 of row r's window.  Each chunk runs
// the recursion from zero state, the true entering states come from a scan over the chunks of
// the row (lanes of one wave) with the transition matrices Phi^(L 2^j), and the response of
// the recursion to that entering state is added.  The anticausal pass is the same recursion
// run from the end of the window.  Inputs are re-read from LDS in each sweep (only a K-sample
// sliding window is held), the output of the chunk is accumulated in registers.
//
// Orders K >= 2 take the numerator in first-difference form, B(z) = (1 - z^-1) C(z) + s with
// taps c_k = -(b_{k+1} + ... + b_{K-1}) (k < K - 1) and s = sum(b): each recursion filters
// d[i] = x[i] - x[i-1] (anticausal: x[i] - x[i+1]) by C and, when REM, adds s x[i].  For a
// balanced numerator (sum(b) = 0) there is no remainder, and the float32 filter keeps the
// exactly zero response at zero frequency that the ramp has (eq 6); otherwise that response is
// s c_t rounded once.  Rounding b_k c_t to float32 one tap at a time would leave sum_k b_k c_t
// a few ulps off its value, an offset per row that the back projection sums over ~N rows.
template <int L, int K, bool REM = false>
__device__ void filter_tile(const PassArgs& A, float* S, int q, int row0) {
  constexpr bool DIFF = K >= 2;
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));   // recomputed per call (keeps loop-invariant addresses out of
                                  // registers in the persistent kernel)
  const int C = 1 << A.log2c;
  const int r = tid >> A.log2c, c = tid & (C - 1);
  const int N = 1 << A.log2n, mask = N - 1;
  const int t = row0 + r;
  const int g = ((q * N + t) * A.groups) / (4 * N);
  const float* cf = A.coef + (size_t)g * A.coef_stride;
  const float* cb = DIFF ? cf + A.coef_stride - K : cf;   // C's taps and s at the table's end
  int sig = A.sigma[t];
  const float ct = A.scale[t];
  // the row factor c_t scales the numerator: the recursion then yields c_t y directly
  float bk[K], ak[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    bk[k] = ct * cb[k];
    ak[k] = cf[K + k];
  }
  const float* phi = cf + 2 * K;
  const float* hom = phi + kScanLevels * K * K;
  const int base = c * L;
  float* row = S + r * A.rs;
  const int log2l = A.log2l;
  auto in = [&](int i) -> float {   // window position i (inside the window) -> LDS value
    const int s = (sig + i) & mask;
    return row[s + (s >> log2l)];
  };
  auto at = [&](int i) -> float {   // halo sample: zero outside the window
    const int s = (sig + ((i < 0 || i >= N) ? 0 : i)) & mask;
    const float v = row[s + (s >> log2l)];
    return (i >= 0 && i < N) ? v : 0.f;
  };

  // Same arithmetic, in the same order, as filter_tile_aligned: one step of the causal and one
  // of the anticausal half per iteration (two independent dependency chains), then both carry
  // scans, then both carry corrections.  Step s handles causal sample s and anticausal sample
  // L - 1 - s; a sample's first contribution assigns y, the second adds.
  float y[L];
  float stc[K], sta[K], xc[K], xa[K];
  asm volatile("" : "+v"(sig));
#pragma unroll
  for (int k = 0; k < K; ++k) {
    stc[k] = 0.f;
    sta[k] = 0.f;
    xc[k] = (k < K - 1) ? at(base - 1 - k) : 0.f;
    xa[k] = (k < K - 1) ? at(base + L + k) : 0.f;
  }
  if constexpr (DIFF) diff_history<K>(xc, xa);
#pragma unroll
  for (int s = 0; s < L; ++s) {
    const int i = s, j = L - 1 - s;
    float ac = 0.f, aa = 0.f;
    if constexpr (DIFF) {
      diff_step<K>(xc, xa, in(base + i), in(base + j));
      if constexpr (REM) {       // the remainder s x[i] first
        ac = bk[K - 1] * xc[K - 1];
        aa = bk[K - 1] * xa[K - 1];
      }
#pragma unroll
      for (int k = 0; k < K - 1; ++k) {
        ac = fmaf(bk[k], xc[k], ac);
        aa = fmaf(bk[k], xa[k], aa);
      }
    } else {
#pragma unroll
      for (int k = K - 1; k > 0; --k) {
        xc[k] = xc[k - 1];
        xa[k] = xa[k - 1];
      }
      xc[0] = in(base + i);
      xa[0] = in(base + j);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        ac = fmaf(bk[k], xc[k], ac);
        aa = fmaf(bk[k], xa[k], aa);
      }
    }
    // oldest state first: the previous output enters last, one FMA per step on the chain
#pragma unroll
    for (int k = K - 1; k >= 0; --k) {
      ac = fmaf(-ak[k], stc[k], ac);
      aa = fmaf(-ak[k], sta[k], aa);
    }
    if (s < L / 2) {
      y[i] = ac;
      y[j] = aa;
    } else {
      y[i] += ac;
      y[j] += aa;
    }
#pragma unroll
    for (int k = K - 1; k > 0; --k) {
      stc[k] = stc[k - 1];
      sta[k] = sta[k - 1];
    }
    stc[0] = ac;
    sta[0] = aa;
  }
  {
    float tc[K], ta[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      tc[k] = stc[k];
      ta[k] = sta[k];
    }
    for (int jj = 0; (1 << jj) < C && jj < A.scan_levels; ++jj) {
      const int d = 1 << jj;
      float uc[K], ua[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        uc[k] = __shfl_up(tc[k], d, C);
        ua[k] = __shfl_down(ta[k], d, C);
      }
      const float* P = phi + jj * K * K;
      float nc[K], na[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        float accc = tc[k], acca = ta[k];
#pragma unroll
        for (int m = 0; m < K; ++m) {
          accc = fmaf(P[k * K + m], uc[m], accc);
          acca = fmaf(P[k * K + m], ua[m], acca);
        }
        nc[k] = accc;
        na[k] = acca;
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        tc[k] = (c >= d) ? nc[k] : tc[k];
        ta[k] = (c + d < C) ? na[k] : ta[k];
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const float pc = (C > 1) ? __shfl_up(tc[k], 1, C) : 0.f;
      const float pa = (C > 1) ? __shfl_down(ta[k], 1, C) : 0.f;
      stc[k] = (c == 0) ? 0.f : pc;
      sta[k] = (c == C - 1) ? 0.f : pa;
    }
    // carry correction: the carried-in state through the homogeneous response, oldest first
#pragma unroll
    for (int s = 0; s < L; ++s) {
      const int i = s, j = L - 1 - s;
      float yc = y[i], ya = y[j];
#pragma unroll
      for (int k = K - 1; k >= 0; --k) {
        yc = fmaf(hom[k * L + s], stc[k], yc);
        ya = fmaf(hom[k * L + s], sta[k], ya);
      }
      y[i] = yc;
      y[j] = ya;
    }
  }
  __syncthreads();   // every chunk has read its samples and its neighbours' halo
  asm volatile("" : "+v"(sig));
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const int s = (sig + base + i) & mask;
    row[s + (s >> log2l)] = y[i];
  }
  __syncthreads();
}

// The same filter for rows stored window-aligned (window position p at LDS column p, skew period
// 32): every in-chunk access is the chunk's base pointer plus an immediate offset.  The caller
// passes the row factor c_t, and guarantees that all rows of a wave lie in one coefficient
// group (first_pass_supported): the group's coefficients are then read with scalar loads,
// which do not wait behind the vector loads of the next tile that are already in flight.
// `step_hook(s)` runs at the top of recursion step s (the caller uses it to issue the next
// tile's loads a few at a time, so the texture unit takes them while the ALUs work).
// WIDE: rows of 128 chunks over two waves (the row length 4096); otherwise C <= 64.
// The numerator forms of filter_tile (first difference for K >= 2, remainder when REM).
template <int K, bool WIDE, bool REM, typename Hook>
__device__ bool filter_tile_aligned(const PassArgs& A, float* S, float* xs, int q, int row0,
                                    float ct, Hook&& step_hook) {
  constexpr int L = 32;
  constexpr bool DIFF = K >= 2;
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int C = 1 << A.log2c;
  const int lane = tid & 63;
  // Rows of 32 chunks (ILV): the wave's two rows interleave by 16 chunks, lanes 0-15 holding
  // row 2w's chunks 0-15, lanes 16-31 row 2w + 1's, lanes 32-47 and 48-63 their chunks 16-31,
  // so that level 0's partner (the same chunk of the other row) is lane ^ 16, as for rows of
  // 16 chunks.  Otherwise a row's chunks are consecutive lanes.
  const bool ilv = A.log2c == 5;
  const int r = ilv ? (((tid >> 6) << 1) | ((lane >> 4) & 1)) : tid >> A.log2c;
  const int c = ilv ? ((lane & 15) | ((lane >> 5) << 4)) : tid & (C - 1);
  // the lane of chunk cc of this lane's row (rows within one wave)
  auto chunk_lane = [&](int cc) -> int {
    return ilv ? ((cc & 15) | (lane & 16) | ((cc >> 4) << 5)) : (lane & ~(C - 1)) | cc;
  };
  const int N = 1 << A.log2n;
  const int t = row0 + r;
  const int g = __builtin_amdgcn_readfirstlane(((q * N + t) * A.groups) / (4 * N));
  cfloat* cf = as_constant(A.coef + (size_t)g * A.coef_stride);
  cfloat* cb = DIFF ? cf + (A.coef_stride - K) : cf;   // C's taps and s at the table's end
  // the row factor c_t scales the numerator (per lane: a wave holds 64 / C rows)
  float bk[K], ak[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    bk[k] = ct * cb[k];
    ak[k] = cf[K + k];
  }
  cfloat* phi = cf + 2 * K;
  cfloat* hom = phi + kScanLevels * K * K;
  const int base = c * L;
  float* row = S + r * A.rs;
  float* rp = row + base + (base >> 5);       // window positions base .. base + 31
  auto at = [&](int p) -> float {             // halo sample, zero outside the window
    const int pc = (p < 0 || p >= N) ? 0 : p;
    const float v = row[pc + (pc >> 5)];
    return (p >= 0 && p < N) ? v : 0.f;
  };
  // The causal and the anticausal halves are independent until their sum, and so are their
  // carry scans and carry corrections: each loop below runs one step of both, two independent
  // dependency chains.  Step s handles causal sample s and anticausal sample L - 1 - s; a
  // sample's first contribution assigns y, the second adds.
  float y[L];
  float stc[K], sta[K], xc[K], xa[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    stc[k] = 0.f;
    sta[k] = 0.f;
    xc[k] = (k < K - 1) ? at(base - 1 - k) : 0.f;
    xa[k] = (k < K - 1) ? at(base + L + k) : 0.f;
  }
  if constexpr (DIFF) diff_history<K>(xc, xa);
#pragma unroll
  for (int s = 0; s < L; ++s) {
    const int i = s, j = L - 1 - s;
    if constexpr (!DIFF) {
#pragma unroll
      for (int k = K - 1; k > 0; --k) {
        xc[k] = xc[k - 1];
        xa[k] = xa[k - 1];
      }
    }
    if ((s & 3) == 0) asm volatile("" ::: "memory");   // keeps at most 8 LDS reads in flight
    step_hook(s);
    if ((s & 7) == 0) __builtin_amdgcn_sched_barrier(0);   // the hook's work stays at step s
    float ac = 0.f, aa = 0.f;
    if constexpr (DIFF) {
      diff_step<K>(xc, xa, rp[i], rp[j]);
      if constexpr (REM) {       // the remainder s x[i] first
        ac = bk[K - 1] * xc[K - 1];
        aa = bk[K - 1] * xa[K - 1];
      }
#pragma unroll
      for (int k = 0; k < K - 1; ++k) {
        ac = fmaf(bk[k], xc[k], ac);
        aa = fmaf(bk[k], xa[k], aa);
      }
    } else {
      xc[0] = rp[i];
      xa[0] = rp[j];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        ac = fmaf(bk[k], xc[k], ac);
        aa = fmaf(bk[k], xa[k], aa);
      }
    }
    // oldest state first: the previous output enters last, one FMA per step on the chain
#pragma unroll
    for (int k = K - 1; k >= 0; --k) {
      ac = fmaf(-ak[k], stc[k], ac);
      aa = fmaf(-ak[k], sta[k], aa);
    }
    if (s < L / 2) {
      y[i] = ac;
      y[j] = aa;
    } else {
      y[i] += ac;
      y[j] += aa;
    }
#pragma unroll
    for (int k = K - 1; k > 0; --k) {
      stc[k] = stc[k - 1];
      sta[k] = sta[k - 1];
    }
    stc[0] = ac;
    sta[0] = aa;
  }
  {
    // chunk end states through Phi_j: causal from the chunks on the left, anticausal from the
    // right (Hillis-Steele; every lane takes part in every shuffle)
    float tc[K], ta[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      tc[k] = stc[k];
      ta[k] = sta[k];
    }
    // a row's chunks span W = min(C, 64) lanes of one wave (C = 128: two waves, the last scan
    // level below goes across them)
    const int W = WIDE ? 64 : C;
    const int cw = c & (W - 1);
    for (int jj = 0; (1 << jj) < W && jj < A.scan_levels; ++jj) {
      const int d = 1 << jj;
      float uc[K], ua[K];
      // the states of chunks cw - d and cw + d (masked below where they do not exist)
      const int lu = WIDE ? lane - (cw >= d ? d : 0) : chunk_lane(cw >= d ? cw - d : cw);
      const int ld = WIDE ? lane + (cw + d < W ? d : 0) : chunk_lane(cw + d < W ? cw + d : cw);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        uc[k] = __shfl(tc[k], lu);
        ua[k] = __shfl(ta[k], ld);
      }
      cfloat* P = phi + jj * K * K;
      float nc[K], na[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        float accc = tc[k], acca = ta[k];
#pragma unroll
        for (int m = 0; m < K; ++m) {
          accc = fmaf(P[k * K + m], uc[m], accc);
          acca = fmaf(P[k * K + m], ua[m], acca);
        }
        nc[k] = accc;
        na[k] = acca;
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        tc[k] = (cw >= d) ? nc[k] : tc[k];
        ta[k] = (cw + d < W) ? na[k] : ta[k];
      }
    }
    // C = 128: the row's two waves join through LDS.  After the levels above, lane i of the
    // second wave holds the causal state of its chunks 64 .. 64 + i alone, and lane i of the
    // first the anticausal state of its chunks i .. 63 alone.  The first wave's causal state at
    // chunk 63 (S) and the second's anticausal state at chunk 64 (T) are complete; each wave
    // publishes its own, and every lane adds the other's carried over its distance m in
    // chunks: Phi^(32 m) S with m = i + 1 in the second wave, Phi^(32 m) T with m = 64 - i in
    // the first, the power taken from the table's Phi^(32 2^j) by the bits of m.  S and T are
    // also the carries across the wave boundary in the shift by one chunk below.
    float ec[K], ea[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      ec[k] = 0.f;
      ea[k] = 0.f;
    }
    if constexpr (WIDE) {
      const int half = c >> 6, lane = c & 63;
      float* mine = xs + ((r * 2 + half) * K) * 64;
      const float* other = xs + ((r * 2 + (half ^ 1)) * K) * 64;
#pragma unroll
      for (int k = 0; k < K; ++k) mine[k * 64 + lane] = half == 0 ? tc[k] : ta[k];
      __syncthreads();
#pragma unroll
      for (int k = 0; k < K; ++k) {
        ec[k] = other[k * 64 + 63];     // S, read by the second wave
        ea[k] = other[k * 64];          // T, read by the first wave
      }
      const int m = half == 0 ? 64 - lane : lane + 1;     // 1 .. 64
      float v[K];
#pragma unroll
      for (int k = 0; k < K; ++k) v[k] = half == 0 ? ea[k] : ec[k];
#pragma unroll
      for (int j = 0; j < 7; ++j) {
        cfloat* P = phi + j * K * K;
        float nv[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          float acc = 0.f;
#pragma unroll
          for (int q2 = 0; q2 < K; ++q2) acc = fmaf(P[k * K + q2], v[q2], acc);
          nv[k] = acc;
        }
        const bool use = (m >> j) & 1;
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = use ? nv[k] : v[k];
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (half == 0) ta[k] += v[k];
        else tc[k] += v[k];
      }
    }
    const int l1u = WIDE ? lane - (cw >= 1 ? 1 : 0) : chunk_lane(cw >= 1 ? cw - 1 : cw);
    const int l1d = WIDE ? lane + (cw + 1 < W ? 1 : 0) : chunk_lane(cw + 1 < W ? cw + 1 : cw);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const float pc = (W > 1) ? __shfl(tc[k], l1u) : 0.f;
      const float pa = (W > 1) ? __shfl(ta[k], l1d) : 0.f;
      stc[k] = (c == 0) ? 0.f : (cw == 0 ? ec[k] : pc);
      sta[k] = (c == C - 1) ? 0.f : (cw == W - 1 ? ea[k] : pa);
    }
    // carry correction: the carried-in state through the homogeneous response, oldest first
    // (the table goes through scalar registers 8 steps at a time, 4 from order 4 on: the
    // barriers keep the compiler from loading all of it at once and spilling scalar registers
    // elsewhere)
#pragma unroll
    for (int s = 0; s < L; ++s) {
      if ((s & (K >= 4 ? 3 : 7)) == 0) asm volatile("" ::: "memory");
      const int i = s, j = L - 1 - s;
      float yc = y[i], ya = y[j];
#pragma unroll
      for (int k = K - 1; k >= 0; --k) {
        yc = fmaf(hom[k * L + s], stc[k], yc);
        ya = fmaf(hom[k * L + s], sta[k], ya);
      }
      y[i] = yc;
      y[j] = ya;
    }
  }
  __syncthreads();   // every chunk has read its samples and its neighbours' halo
  // With C <= 32 the two rows that level 0 of the transposed transform pairs (tile rows 2k and
  // 2k + 1) sit in lanes c and c + C of one wave.  Their window starts are equal (row0 is
  // even), so in window coordinates the butterfly is lower[x] = r0[x] + r1[x] and upper[x] =
  // r0[x] + r1[x - 1], cyclically: it is done here, on the scaled filter output in registers,
  // and the rows are stored after level 0 (the same additions as the LDS level would do).
  const bool level0 = A.log2c <= 5;
  if (level0) {
    const bool upper = (r & 1) != 0;
    float v[L];
#pragma unroll
    for (int i = 0; i < L; ++i) v[i] = y[i];
    // r1[x - 1] at the start of the chunk: the last value of the previous chunk of this row
    const float prev = __shfl(v[L - 1], chunk_lane((c - 1) & (C - 1)));
    // the partner lane is lane ^ 16 for C = 32 (interleaved rows) and 16, lane ^ C otherwise.
    // For C = 32 and 16 one permlane swap of rows of 16 lanes per sample does it: swapping
    // X = v[i] with Y = (upper ? r1[x - 1] : v[i]) leaves r0[x] in the first output of every
    // lane and, in the second, r1[x] for the lower row and r1[x - 1] for the upper one, so each
    // lane's level-0 value is the sum of the two (no LDS traffic, no select after the swap).
    // (The 32-lane swap, for rows of consecutive lanes, costs two register copies per sample.)
    // Other C use a shuffle.
    if (A.log2c == 4 || ilv) {
#pragma unroll
      for (int i = 0; i < L; ++i) {
        const float yv = upper ? (i == 0 ? prev : v[i - 1]) : v[i];
        const auto sw = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i]),
                                                         __float_as_uint(yv), false, false);
        rp[i] = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
      }
    } else {
#pragma unroll
      for (int i = 0; i < L; ++i) {
        const float p = __shfl_xor(v[i], C);
        rp[i] = upper ? p + (i == 0 ? prev : v[i - 1]) : v[i] + p;
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < L; ++i) rp[i] = y[i];
  }
  __syncthreads();
  return level0;
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
  const int lane = threadIdx.x & 63, wave = wave_id();
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
    // blocks from the top; the reads of a lower block never touch columns a higher block of
    // the same batch writes, so four blocks are read before any is written
    for (int top = (W >> 6) - 1; top >= 0; top -= 4) {
      float va[4], vb[4];
#pragma unroll
      for (int u2 = 0; u2 < 4; ++u2) {
        const int blk = top - u2;
        if (blk < 0) break;
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
        va[u2] = v0 + v1;
        vb[u2] = v0 + v2;
      }
#pragma unroll
      for (int u2 = 0; u2 < 4; ++u2) {
        const int blk = top - u2;
        if (blk < 0) break;
        const int x = x0 + (blk << 6) + lane;
        row0[x + (x >> A.log2l)] = va[u2];
        row1[x + (x >> A.log2l)] = vb[u2];
      }
    }
  }
}

// Streaming level with a compile-time number of 64-column blocks per unit and the 32-column
// skew: the five LDS addresses of a butterfly are per-unit base pointers plus immediate offsets
// (66 words per block), so the walk costs two adds per 64 butterflies besides the LDS accesses.
template <int NBLK>
__device__ __forceinline__ void level_stream_fast(const PassArgs& A, float* S, float* below,
                                                  int l) {
  const int N = 1 << A.log2n, mask = N - 1;
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int waves = blockDim.x >> 6;
  const int log2p = A.log2r - 1;
  const int segs = waves > (1 << log2p) ? waves >> log2p : 1;
  constexpr int W = NBLK * 64;
  const int units = ((1 << log2p) * segs) / waves;
  for (int u = 0; u < units; ++u) {
    const int unit = wave + u * waves;
    const int pair = unit / segs, seg = unit - pair * segs;
    const int ib = pair & ((1 << l) - 1), pp = pair >> l;
    const int r1 = ((pp << (l + 1)) | ib) | (1 << l);
    const int xb = (seg * W - 64 + lane) & mask;
    below[unit * 64 + lane] = S[r1 * A.rs + xb + (xb >> 5)];
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
    const int xb = x0 + 64 + lane;              // column of block 1
    const int x1 = xb - J, x2 = xb - J - 1;     // >= 0 since J < 64
    float* a0 = row0 + xb + (xb >> 5);
    float* w1 = row1 + xb + (xb >> 5);
    const float* a1 = row1 + x1 + (x1 >> 5);
    const float* a2 = row1 + x2 + (x2 >> 5);
#pragma unroll
    for (int top = NBLK - 1; top >= 1; top -= 4) {
      float va[4], vb[4];
#pragma unroll
      for (int u2 = 0; u2 < 4; ++u2) {
        const int k = top - u2;
        if (k >= 1) {
          const int off = 66 * (k - 1);
          const float v0 = a0[off];
          va[u2] = v0 + a1[off];
          vb[u2] = v0 + a2[off];
        }
      }
#pragma unroll
      for (int u2 = 0; u2 < 4; ++u2) {
        const int k = top - u2;
        if (k >= 1) {
          const int off = 66 * (k - 1);
          a0[off] = va[u2];
          w1[off] = vb[u2];
        }
      }
    }
    {   // block 0: reads below x0 come from the copy
      const int x = x0 + lane;
      const int y1 = x - J, y2 = x - J - 1;
      const int m1 = y1 & mask, m2 = y2 & mask;
      const float v0 = row0[x + (x >> 5)];
      const float t1 = row1[m1 + (m1 >> 5)];
      const float t2 = row1[m2 + (m2 >> 5)];
      const float v1 = (y1 >= x0) ? t1 : below[unit * 64 + ((y1 - x0 + 64) & 63)];
      const float v2 = (y2 >= x0) ? t2 : below[unit * 64 + ((y2 - x0 + 64) & 63)];
      row0[x + (x >> 5)] = v0 + v1;
      row1[x + (x >> 5)] = v0 + v2;
    }
  }
}

// Lane L receives v from lane L - 1 and lane 0 receives `first` (DPP wave shift right by one).
__device__ __forceinline__ float lanes_shift_up(float v, float first) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(first), __float_as_int(v),
                                                    0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ float lane63(float v) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ float uniform_float(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Streaming level for a tile whose rows start with the rotations sigma of their filtering
// windows (ROT): the butterfly inputs then differ by d = (sigma_a - sigma_b) - J, which can be
// positive.  Units with d <= 0 walk down from the top block with a copy of the 64 columns below
// the segment; units with d >= 1 walk up from the bottom block with a copy of the 64 columns
// above it.  Without ROT, d = -J (the plain lazy-shift form).
template <int NBLK, bool ROT>
__device__ __forceinline__ void level_stream_rot(const PassArgs& A, float* S, float* copy, int l,
                                                 int row0) {
  const int N = 1 << A.log2n, mask = N - 1;
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int waves = blockDim.x >> 6;
  const int log2p = A.log2r - 1;
  const int log2wv = 31 - __clz(waves);
  const int log2s = log2wv > log2p ? log2wv - log2p : 0;    // segments per row pair
  constexpr int W = NBLK * 64;
  const int units = 1 << (log2p + log2s - log2wv);
  auto rel = [&](int pp, int J) -> int {
    int d = -J;
    if constexpr (ROT) {
      const int sa = window_start_of(row0 + (pp << (l + 1)), A.log2n, A.windowed);
      const int sb = window_start_of(row0 + (pp << (l + 1)) + (1 << l), A.log2n, A.windowed);
      int delta = (sa - sb) & mask;
      if (delta > (N >> 1)) delta -= N;
      d += delta;
    }
    return d;
  };
  for (int u = 0; u < units; ++u) {
    const int unit = wave + u * waves;
    const int pair = unit >> log2s, seg = unit & ((1 << log2s) - 1);
    const int ib = pair & ((1 << l) - 1), pp = pair >> l;
    const int r1 = ((pp << (l + 1)) | ib) | (1 << l);
    const int d = rel(pp, brev_bits(ib, l));
    const int xc = ((d <= 0) ? (seg * W - 64) : (seg * W + W)) + lane;
    const int xm = xc & mask;
    copy[unit * 64 + lane] = S[r1 * A.rs + xm + (xm >> 5)];
  }
  // with one segment per row pair, a unit's copy is written and read by the same wave (LDS
  // accesses of a wave complete in order): only split rows need the block to wait here
  if (log2s > 0) __syncthreads();
  for (int u = 0; u < units; ++u) {
    const int unit = wave + u * waves;
    const int pair = unit >> log2s, seg = unit & ((1 << log2s) - 1);
    const int ib = pair & ((1 << l) - 1), pp = pair >> l;
    const int r0 = (pp << (l + 1)) | ib, r1 = r0 | (1 << l);
    const int d = rel(pp, brev_bits(ib, l));
    float* row0p = S + r0 * A.rs;
    float* row1p = S + r1 * A.rs;
    const int x0 = seg * W;
    const float* cp = copy + unit * 64;
    // The second input of column x, row1[x + d - 1], is the first input of column x - 1: lane
    // L takes it from lane L - 1 of the same block, lane 0 from lane 63 of the block below, so
    // a column costs two LDS reads instead of three.
    if (d <= 0) {
      const int xb = x0 + 64 + lane;              // block 1
      const int x1 = xb + d;                      // >= x0 since -d + 1 <= 64
      float* a0 = row0p + xb + (xb >> 5);
      float* w1 = row1p + xb + (xb >> 5);
      const float* a1 = row1p + x1 + (x1 >> 5);
      const int x = x0 + lane;                    // block 0
      const int y1 = x + d, y2 = x + d - 1;
      const int m1 = y1 & mask;
      // walking down, the first input of the next block is read one block ahead (it lies below
      // everything this walk has written); lane 63 of block 0's is inside the segment
      float nxt;
      if constexpr (NBLK >= 2) nxt = a1[66 * (NBLK - 2)];
      else nxt = row1p[m1 + (m1 >> 5)];
#pragma unroll
      for (int top = NBLK - 1; top >= 1; top -= 4) {
        float va[4], vb[4];
#pragma unroll
        for (int u2 = 0; u2 < 4; ++u2) {
          const int k = top - u2;
          if (k >= 1) {
            const int off = 66 * (k - 1);
            const float cur = nxt;
            nxt = (k >= 2) ? a1[off - 66] : row1p[m1 + (m1 >> 5)];
            const float v0 = a0[off];
            va[u2] = v0 + cur;
            vb[u2] = v0 + lanes_shift_up(cur, lane63(nxt));
          }
        }
#pragma unroll
        for (int u2 = 0; u2 < 4; ++u2) {
          const int k = top - u2;
          if (k >= 1) {
            const int off = 66 * (k - 1);
            a0[off] = va[u2];
            w1[off] = vb[u2];
          }
        }
      }
      // block 0: nxt holds row1 at y1; inputs below x0 come from the copy (lane 0's always)
      const float v0 = row0p[x + (x >> 5)];
      const float t2 = lanes_shift_up(nxt, 0.f);
      const float v1 = (y1 >= x0) ? nxt : cp[(y1 - x0 + 64) & 63];
      const float v2 = (y2 >= x0) ? t2 : cp[(y2 - x0 + 64) & 63];
      row0p[x + (x >> 5)] = v0 + v1;
      row1p[x + (x >> 5)] = v0 + v2;
    } else {
      const int xb = x0 + lane;                   // block 0
      const int x1 = xb + d;
      float* a0 = row0p + xb + (xb >> 5);
      float* w1 = row1p + xb + (xb >> 5);
      const float* a1 = row1p + x1 + (x1 >> 5);
      // lane 0 of block 0 takes row1 at x0 + d - 1, inside the segment since 1 <= d <= 64
      const int xs = x0 + d - 1;
      float below63 = uniform_float(row1p[xs + (xs >> 5)]);
#pragma unroll
      for (int bot = 0; bot <= NBLK - 2; bot += 4) {
        float va[4], vb[4];
#pragma unroll
        for (int u2 = 0; u2 < 4; ++u2) {
          const int k = bot + u2;
          if (k <= NBLK - 2) {
            const int off = 66 * k;
            const float cur = a1[off];
            const float v0 = a0[off];
            va[u2] = v0 + cur;
            vb[u2] = v0 + lanes_shift_up(cur, below63);
            below63 = lane63(cur);
          }
        }
#pragma unroll
        for (int u2 = 0; u2 < 4; ++u2) {
          const int k = bot + u2;
          if (k <= NBLK - 2) {
            const int off = 66 * k;
            a0[off] = va[u2];
            w1[off] = vb[u2];
          }
        }
      }
      // top block: reads above the segment come from the copy
      const int x = x0 + W - 64 + lane;
      const int y1 = x + d, y2 = x + d - 1;
      const int m1 = y1 & mask;
      const float v0 = row0p[x + (x >> 5)];
      const float t1 = row1p[m1 + (m1 >> 5)];
      const float t2 = lanes_shift_up(t1, below63);
      const int top_end = x0 + W;
      const float v1 = (y1 < top_end) ? t1 : cp[(y1 - top_end) & 63];
      const float v2 = (y2 < top_end) ? t2 : cp[(y2 - top_end) & 63];
      row0p[x + (x >> 5)] = v0 + v1;
      row1p[x + (x >> 5)] = v0 + v2;
    }
  }
}

// Two levels (l, l + 1) of the first pass in one LDS round trip (radix 4), for rows stored
// with their window rotations.  A unit is four rows r0 = base + ib, r1 = r0 + 2^l,
// r2 = r0 + 2^(l+1), r3 = r2 + 2^l (base a multiple of 2^(l+2), ib < 2^l).  With the shifts
// d01, d23 of level l and e of level l + 1 (each relative to the frames the rows are held in),
//   A0 = r0[x] + r1[x + d01]          A1 = r0[x] + r1[x + d01 - 1]
//   A2(y) = r2[y] + r3[y + d23]       A3(y) = r2[y] + r3[y + d23 - 1]
//   B0 = A0 + A2(x + e)   B2 = A0 + A2(x + e - 1)   B1 = A1 + A3(x + e - 1)   B3 = A1 + A3(x + e - 2)
// which are the additions of the two levels done one after the other.  A lane holds column
// x = 61 k - 3 + lane of block k and reads r0[x], r1[x + d01], r2[x + e], r3[x + e + d23]; every
// "- 1" operand is the lane below's value, moved by a DPP lane shift.  B3 reaches three lanes
// down (A3(x + e - 2) holds r3 at x + e + d23 - 3), so lanes 0..2 only feed their neighbours
// and each block writes 61 columns.  Per column of a unit that is four reads and four writes
// for two levels, against eight of each for two streaming levels.  All reads of the stage
// finish (barrier) before any write, so the shifts may have any sign.
// The last stage of the pass (stage4_store) stores its outputs to HBM directly: tile row rho's
// column x goes to column (x + sig0 + v brev(rho, F)) mod N of output row brev(rho, F) 2^k_lo + v.
constexpr int kStageMaxBlocks = 9;    // blocks of 61 columns per wave and stage
constexpr int kStageInnerLast = 7;    // last block index j that stage4_inner_ok covers

// Blocks j = 1 .. 7 of a wave never wrap around the row: with 17 blocks (N = 1024) over two
// waves per unit they cover columns 61 (first + 2 j) - 3 .. + 60, i.e. 119 .. 975, and every
// read column c + D (D = 0, d01, e, e + d23) stays in 0 .. 1023 when -119 <= D <= 48.
__device__ __forceinline__ bool stage4_inner_ok(int nb, int step, int d01, int e, int d23) {
  const int lo = min(min(0, d01), min(e, e + d23));
  const int hi = max(max(0, d01), max(e, e + d23));
  return nb == 17 && step == 2 && lo >= -119 && hi <= 48;
}

__device__ __forceinline__ int wrap_half(int d, int N) {
  d &= N - 1;
  return d > (N >> 1) ? d - N : d;
}

__device__ __forceinline__ float lanes_shift_up_any(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}

// The stage gives every wave one unit and the blocks first, first + step, ... of it (so the
// waves must outnumber the units), at most kStageMaxBlocks of them.
__host__ __device__ inline bool stage4_fits(const PassArgs& A, int threads) {
  const int N = 1 << A.log2n;
  const int waves = threads >> 6, units = (1 << A.log2r) >> 2;
  if (waves < units) return false;
  const int nb = (N + 60) / 61, step = waves / units;
  return (nb + step - 1) / step <= kStageMaxBlocks;
}

// Whether a first pass of order K runs the levels after level 0 (done in the filter when a row
// has at most 32 chunks) as radix-4 stages, the last of which stores the tile; otherwise every
// level streams and the tile is written out from LDS.  The host picks the kernel by it.
__host__ __device__ inline bool first_pass_stages(const PassArgs& A, int threads, int K) {
  const int l = (K > 0 && A.log2c <= 5) ? 1 : 0;
  return A.levels - l >= 2 && stage4_fits(A, threads);
}

// IN_SKEW: the stage reads skewed rows (from the filter or a streaming level); later stages
// read the unskewed rows an earlier stage wrote.  The stage writes its rows unskewed, at their
// frame positions (the last stage of a pass is stage4_store).
template <bool ROT, bool IN_SKEW, bool INNER_OK = true>
__device__ __forceinline__ void stage4(const PassArgs& A, float* S, int l, int row0) {
  const int N = 1 << A.log2n, mask = N - 1;
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int log2u = A.log2r - 2;                 // units: R / 4
  const int nb = (N + 60) / 61;
  const int step = (blockDim.x >> 6) >> log2u;
  const int first = wave >> log2u;
  // the unit's rows, shifts and (for the final stage) output rotations, all wave-uniform
  const int u = wave & ((1 << log2u) - 1);
  const int pp = u >> l, ib = u & ((1 << l) - 1);
  const int base = pp << (l + 2);
  const int r0 = base + ib;
  int s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  if constexpr (ROT) {
    s0 = window_start_of(row0 + base, A.log2n, A.windowed);
    s1 = window_start_of(row0 + base + (1 << l), A.log2n, A.windowed);
    s2 = window_start_of(row0 + base + (2 << l), A.log2n, A.windowed);
    s3 = window_start_of(row0 + base + (3 << l), A.log2n, A.windowed);
  }
  const int J = brev_bits(ib, l), J2 = brev_bits(ib, l + 1);
  const int d01 = wrap_half(s0 - s1, N) - J;
  const int d23 = wrap_half(s2 - s3, N) - J;
  const int e = wrap_half(s0 - s2, N) - J2;
  const int rs = A.rs;
  float* p0 = S + r0 * rs;
  float* p1 = p0 + (rs << l);
  float* p2 = p0 + (rs << (l + 1));
  float* p3 = p2 + (rs << l);
  // blocks past the wave's last repeat it: the same values are computed and stored twice
  float o0[kStageMaxBlocks], o1[kStageMaxBlocks], o2[kStageMaxBlocks], o3[kStageMaxBlocks];
  // with 17 blocks over two waves per unit (N = 1024), blocks j = 1 .. 7 of a wave lie at
  // columns 119 .. 975 and none of their reads wraps: they skip the cyclic masks
  const bool inner_ok = INNER_OK && stage4_inner_ok(nb, step, d01, e, d23);
  auto reads = [&](auto inner_tag) {
    constexpr bool INNER = decltype(inner_tag)::value;
#pragma unroll
    for (int j = 0; j < kStageMaxBlocks; ++j) {
      const bool inner = INNER && j >= 1 && j <= kStageInnerLast;
      const int blk = inner ? first + j * step : min(first + j * step, nb - 1);
      const int c = blk * 61 - 3 + lane;
      const int x0 = inner ? c : c & mask, x1 = inner ? c + d01 : (c + d01) & mask;
      const int x2 = inner ? c + e : (c + e) & mask;
      const int x3 = inner ? c + e + d23 : (c + e + d23) & mask;
      const float a = p0[IN_SKEW ? x0 + (x0 >> 5) : x0];
      const float b = p1[IN_SKEW ? x1 + (x1 >> 5) : x1];
      const float f = p2[IN_SKEW ? x2 + (x2 >> 5) : x2];
      const float g = p3[IN_SKEW ? x3 + (x3 >> 5) : x3];
      const float A0 = a + b;
      const float A1 = a + lanes_shift_up_any(b);
      const float A2e = f + g;
      const float A3e = f + lanes_shift_up_any(g);
      const float t = lanes_shift_up_any(A3e);
      o0[j] = A0 + A2e;
      o2[j] = A0 + lanes_shift_up_any(A2e);
      o1[j] = A1 + t;
      o3[j] = A1 + lanes_shift_up_any(t);
    }
  };
  if constexpr (INNER_OK) {
    if (inner_ok) reads(std::true_type{});
    else reads(std::false_type{});
  } else {
    reads(std::false_type{});
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kStageMaxBlocks; ++j) {
    const int blk = min(first + j * step, nb - 1);
    const int c = blk * 61 - 3 + lane;
    if (lane >= 3 && c < N) {
      p0[c] = o0[j];
      p1[c] = o1[j];
      p2[c] = o2[j];
      p3[c] = o3[j];
    }
  }
  __syncthreads();
}

// A block of stage4_store past the wave's last, and lanes that only feed their neighbours'
// shifts, store to this byte offset, beyond any slice: the hardware drops out-of-range buffer
// stores, so the stores need no branch.
constexpr int kDropOffset = 0x40000000;

// The last stage of the first pass: as stage4, but each block's outputs go straight to HBM
// (row brev(rho) 2^k_lo + v of the class, rotated by sig0 + v brev(rho)), one 4-byte store per
// lane and row, as soon as they are computed.  Nothing is written back to LDS, so the stage
// needs no barrier between its reads and its stores (the caller's end-of-tile barrier guards
// the reuse of LDS), and there is no separate write-out.
template <bool ROT, bool IN_SKEW, bool INNER_OK = true>
__device__ __forceinline__ void stage4_store(const PassArgs& A, const float* S, int l, int row0,
                                             int sig0, int v, float* dst, int k_lo) {
  const int N = 1 << A.log2n, mask = N - 1;
  const int F = A.levels;
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int log2u = A.log2r - 2;
  const int nb = (N + 60) / 61;
  const int step = (blockDim.x >> 6) >> log2u;
  const int first = wave >> log2u;
  const int u = wave & ((1 << log2u) - 1);
  const int pp = u >> l, ib = u & ((1 << l) - 1);
  const int base = pp << (l + 2);
  const int r0 = base + ib;
  int s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  if constexpr (ROT) {
    s0 = window_start_of(row0 + base, A.log2n, A.windowed);
    s1 = window_start_of(row0 + base + (1 << l), A.log2n, A.windowed);
    s2 = window_start_of(row0 + base + (2 << l), A.log2n, A.windowed);
    s3 = window_start_of(row0 + base + (3 << l), A.log2n, A.windowed);
  }
  const int J = brev_bits(ib, l), J2 = brev_bits(ib, l + 1);
  const int d01 = wrap_half(s0 - s1, N) - J;
  const int d23 = wrap_half(s2 - s3, N) - J;
  const int e = wrap_half(s0 - s2, N) - J2;
  const int rs = A.rs;
  const float* p0 = S + r0 * rs;
  const float* p1 = p0 + (rs << l);
  const float* p2 = p0 + (rs << (l + 1));
  const float* p3 = p2 + (rs << l);
  const int i0 = brev_bits(r0, F), i1 = brev_bits(r0 + (1 << l), F);
  const int i2 = brev_bits(r0 + (2 << l), F), i3 = brev_bits(r0 + (3 << l), F);
  // stores through a buffer resource over the slice: the output row is a scalar byte offset,
  // the cyclic column a 32-bit vector offset (two vector instructions per store)
  const __amdgpu_buffer_rsrc_t out = __builtin_amdgcn_make_buffer_rsrc(
      (void*)dst, (short)0, (N * N) * 4, kBufferDword3);
  const int so0 = (((i0 << k_lo) + v) * N) * 4, so1 = (((i1 << k_lo) + v) * N) * 4;
  const int so2 = (((i2 << k_lo) + v) * N) * 4, so3 = (((i3 << k_lo) + v) * N) * 4;
  const int m4 = N * 4 - 1;
  const int y0 = (sig0 + v * i0) * 4, y1 = (sig0 + v * i1) * 4;
  const int y2 = (sig0 + v * i2) * 4, y3 = (sig0 + v * i3) * 4;
  const int nbw = (nb - first + step - 1) / step;   // this wave's blocks
  // as in stage4, blocks j = 1 .. 7 never wrap when there are 17 blocks over two waves; on
  // unskewed rows they then read through one base per row with immediate offsets
  const bool inner_ok = INNER_OK && !IN_SKEW && stage4_inner_ok(nb, step, d01, e, d23);
  const int cb = first * 61 - 3 + lane;             // column of block j = 0
  const float* q0 = p0 + cb;
  const float* q1 = p1 + (cb + d01);
  const float* q2 = p2 + (cb + e);
  const float* q3 = p3 + (cb + e + d23);
  auto blocks = [&](auto inner_tag) {
    constexpr bool INNER = decltype(inner_tag)::value;
  // every wave issues all kStageMaxBlocks blocks' stores (kTileStores per lane): blocks past
  // the wave's last, lanes 0..2 (they only feed their neighbours' shifts) and columns past N
  // store to kDropOffset
#pragma unroll
  for (int j = 0; j < kStageMaxBlocks; ++j) {
    {
      const bool inner = INNER && j >= 1 && j <= kStageInnerLast;
      const int blk = first + j * step;
      const int c = blk * 61 - 3 + lane;
      float a, b, f, g;
      if (inner) {
        a = q0[122 * j];
        b = q1[122 * j];
        f = q2[122 * j];
        g = q3[122 * j];
      } else {
        const int x0 = c & mask, x1 = (c + d01) & mask, x2 = (c + e) & mask;
        const int x3 = (c + e + d23) & mask;
        a = p0[IN_SKEW ? x0 + (x0 >> 5) : x0];
        b = p1[IN_SKEW ? x1 + (x1 >> 5) : x1];
        f = p2[IN_SKEW ? x2 + (x2 >> 5) : x2];
        g = p3[IN_SKEW ? x3 + (x3 >> 5) : x3];
      }
      const float A0 = a + b;
      const float A1 = a + lanes_shift_up_any(b);
      const float A2e = f + g;
      const float A3e = f + lanes_shift_up_any(g);
      const float t = lanes_shift_up_any(A3e);
      const float B0 = A0 + A2e;
      const float B2 = A0 + lanes_shift_up_any(A2e);
      const float B1 = A1 + t;
      const float B3 = A1 + lanes_shift_up_any(t);
      const bool keep = j < nbw && lane >= 3 && c < N;
      const int c4 = c * 4;
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(B0), out,
                                            keep ? (c4 + y0) & m4 : kDropOffset, so0, 0);
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(B1), out,
                                            keep ? (c4 + y1) & m4 : kDropOffset, so1, 0);
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(B2), out,
                                            keep ? (c4 + y2) & m4 : kDropOffset, so2, 0);
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(B3), out,
                                            keep ? (c4 + y3) & m4 : kDropOffset, so3, 0);
    }
  }
  };
  if constexpr (INNER_OK && !IN_SKEW) {
    if (inner_ok) blocks(std::true_type{});
    else blocks(std::false_type{});
  } else {
    blocks(std::false_type{});
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

template <int L, int K, bool STREAM, bool REM = false>
__device__ void process_class(const PassArgs& A, float* S, int b, int q, int row0) {
  load_tile<L>(A, S, b, q, row0);
  __syncthreads();
  if constexpr (K > 0) filter_tile<L, K, REM>(A, S, q, row0);
  run_levels<L, STREAM>(A, S);
}

// Passes that keep the four classes apart: the first and middle passes of the back projection,
// every pass of the forward transform, and the filter alone (OUT_SAME).
template <int L, int K, bool STREAM, bool REM = false>
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
  process_class<L, K, STREAM, REM>(A, S, b, q, row0);

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
template <int L, int K, bool STREAM, bool REM = false>
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
  process_class<L, K, STREAM, REM>(A, S, b, qa, row0);
#pragma unroll
  for (int k = 0; k < L; ++k) {
    const int e = tid + k * T;
    const int i = vpair ? (e >> A.log2n) : (e & (R - 1));
    const int c = vpair ? (e & mask) : (e >> A.log2r);
    keep[k] = S[lds_at(brev_bits(i, F), c, A.rs, A.log2l)];
  }
  __syncthreads();
  process_class<L, K, STREAM, REM>(A, S, b, qa + 1, row0);
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

// Four consecutive columns x .. x + 3 (x a multiple of 4) of a skewed LDS row held with a
// rotation o (column c at position (c - o) mod N), for a wave-uniform o.  The positions fall into
// at most two 4-aligned groups, each inside one 32-column skew step and away from the wrap, so a
// group is one address plus immediate offsets; which words go to which group depends only on
// o mod 4, a wave-uniform branch.
__device__ __forceinline__ void store4_rotated(float* row, int x, int o, int mask, float4 v) {
  const int m = (-o) & 3;
  const int g0 = (x - o - m) & mask, g1 = (g0 + 4) & mask;
  float* a = row + g0 + (g0 >> 5);
  float* b = row + g1 + (g1 >> 5);
  switch (m) {
    case 0: a[0] = v.x; a[1] = v.y; a[2] = v.z; a[3] = v.w; break;
    case 1: a[1] = v.x; a[2] = v.y; a[3] = v.z; b[0] = v.w; break;
    case 2: a[2] = v.x; a[3] = v.y; b[0] = v.z; b[1] = v.w; break;
    default: a[3] = v.x; b[0] = v.y; b[1] = v.z; b[2] = v.w; break;
  }
}

__device__ __forceinline__ float4 load4_rotated(const float* row, int x, int o, int mask) {
  const int m = (-o) & 3;
  const int g0 = (x - o - m) & mask, g1 = (g0 + 4) & mask;
  const float* a = row + g0 + (g0 >> 5);
  const float* b = row + g1 + (g1 >> 5);
  switch (m) {
    case 0: return make_float4(a[0], a[1], a[2], a[3]);
    case 1: return make_float4(a[1], a[2], a[3], b[0]);
    case 2: return make_float4(a[2], a[3], b[0], b[1]);
    default: return make_float4(a[3], b[0], b[1], b[2]);
  }
}

// ---- persistent first pass: filter + top levels, the next tile's rows prefetched ------------
// Each block loops over tiles (b, q, v) with a stride of the grid.  Per tile: the rows are
// deposited in LDS rotated by their window starts; the filter runs (level 0 in registers at its
// end) while the first half of the next tile's loads goes out a load every 8 recursion steps;
// the second half goes out before the levels; levels 1 .. F - 1 run as radix-4 stages (an odd
// one streams first), the last of which stores the tile to HBM itself.  The loads of the next
// tile are in flight through all of it.
// STAGES: the levels run as radix-4 stages (first_pass_stages).  The two level forms are
// separate kernels: with both in one, the compiler's waits at the top of the tile loop also
// count the previous tile's stores (see prefetch_landed).
template <int L, int K, int NBLK, bool WIDE = false, bool REM = false, bool STAGES = true>
__global__ void __launch_bounds__(1024) fht_first_kernel(PassArgs A) {
  extern __shared__ float S[];
  const int T = blockDim.x, tid = threadIdx.x;
  const int N = 1 << A.log2n, mask = N - 1;
  const int F = A.levels;
  const int tiles = N >> A.log2r;            // tiles per class (first pass: j = 0, tile = v)
  const int k_lo = A.k_hi - F;
  constexpr int NV = (L / 4 > 0) ? L / 4 : 1;   // float4 per thread per tile
  float4 pre[NV];
  int tl = blockIdx.x;
  if (tl >= A.total_tiles) return;
  // Tile loads go through a buffer resource: the tile base and the per-load step stay in scalar
  // registers and every load shares one vector offset, so the prefetch holds only its data.
  // The next tile's loads go out in two halves, one before this tile's filter and one before
  // its levels, so that HBM stays busy through the filter, the levels and the write-out
  // (this tile's stores drain meanwhile) instead of idling after one burst.
  auto issue = [&](int t2, int half) {
    const int bq = t2 / tiles, v = t2 - bq * tiles;
    const float* base = A.in + ((size_t)bq * N + (v << F)) * N;
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (N << F) * 4, kBufferDword3);
    constexpr int H2 = (NV + 1) / 2;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      if ((k < H2) == (half == 0)) {
        const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(rsrc, tid * 16, k * T * 16, 0);
        pre[k] = make_float4(__uint_as_float(w.x), __uint_as_float(w.y), __uint_as_float(w.z),
                             __uint_as_float(w.w));
      }
    }
  };
  // one load of the first half (k < (NV + 1) / 2)
  auto issue_one = [&](int t2, int k) {
    const int bq = t2 / tiles, v = t2 - bq * tiles;
    const float* base = A.in + ((size_t)bq * N + (v << F)) * N;
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (N << F) * 4, kBufferDword3);
    constexpr int H2 = (NV + 1) / 2;
#pragma unroll
    for (int kk = 0; kk < H2; ++kk) {
      if (kk == k) {
        const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(rsrc, tid * 16, kk * T * 16, 0);
        pre[kk] = make_float4(__uint_as_float(w.x), __uint_as_float(w.y), __uint_as_float(w.z),
                              __uint_as_float(w.w));
      }
    }
  };
  // The prefetched rows are marked as landed (an empty asm that redefines them) before a tile's
  // stores are issued: the compiler waits for their loads there, where only loads were issued
  // after them, and at the next deposit (or where it reuses their registers) finds nothing to
  // wait for.  Left to itself it would wait there with a count that, across the loop, cannot
  // tell the loads from the stores issued after them, and so hold the next tile until this
  // tile's stores had drained.
  auto prefetch_landed = [&]() {
#pragma unroll
    for (int k = 0; k < NV; ++k)
      asm volatile("" : "+v"(pre[k].x), "+v"(pre[k].y), "+v"(pre[k].z), "+v"(pre[k].w));
  };
  issue(tl, 0);
  issue(tl, 1);
  prefetch_landed();
  for (; tl < A.total_tiles; tl += gridDim.x) {
    // the thread index is passed through an empty asm once per tile, so per-thread addresses
    // are recomputed each iteration instead of being held in registers across the whole loop
    int ltid = tid;
    asm volatile("" : "+v"(ltid));
    const int bq = tl / tiles, v = tl - bq * tiles;
    const int q = bq & 3;
    const int row0 = v << F;
    // the row factors go out first (scalar loads): their latency hides behind the deposit
    float ct = 0.f;
    if constexpr (K > 0) {
      // a wave holds 64 / C consecutive rows (at most 8 here): read their factors with scalar
      // loads and let each lane pick its row's
      const int wave = __builtin_amdgcn_readfirstlane(ltid >> 6);
      // all eight factors in one go (the table has spare floats past row N - 1), no waits in
      // between; lanes pick their row's (C = 128: a wave holds half of row wave / 2)
      cfloat* sc = as_constant(A.scale + row0 + ((wave << 6) >> A.log2c));
      // (rows of 32 chunks interleave by 16 lanes: see filter_tile_aligned)
      const int lr = A.log2c == 5 ? (ltid >> 4) & 1 : (ltid & 63) >> A.log2c;
      float f8[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) f8[k] = sc[k];
#pragma unroll
      for (int k = 0; k < 8; ++k) ct = (lr == k) ? f8[k] : ct;
    }
    // N >= 256 here (at least four 64-column blocks per unit), so the 256 consecutive values
    // of a wave's float4 lie in one row: the row and its window start are wave-uniform
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int e4 = (ltid + k * T) << 2;
      const int r = __builtin_amdgcn_readfirstlane(e4 >> A.log2n);
      // with the filter, row r is stored window-aligned: shift s at column s - sigma
      const int sg = K > 0 ? window_start_of(row0 + r, A.log2n, A.windowed) : 0;
      store4_rotated(S + r * A.rs, e4, sg, mask, pre[k]);
    }
    __syncthreads();
    const bool more = tl + (int)gridDim.x < A.total_tiles;
    bool level0 = false;
    // the scan's exchange area (rows of more than 64 chunks) after the tile and the streaming
    // copies
    float* xs = S + (pass_lds_bytes(A) >> 2);
    // the next tile's loads (the last tile of a block reloads itself instead of branching)
    const int tn = more ? tl + (int)gridDim.x : tl;
    if constexpr (K > 0) {
      // the first half one every 8 recursion steps
      level0 = filter_tile_aligned<K, WIDE, REM>(A, S, xs, q, row0, ct, [&](int s) {
        if ((s & 7) == 0) issue_one(tn, s >> 3);
      });
    } else {
      issue(tn, 0);
    }
    issue(tn, 1);
    const int sig0 = (K > 0) ? window_start_of(row0, A.log2n, A.windowed) : 0;
    // levels: an odd one streams, the rest go two at a time and the last pair stores the tile;
    // without radix-4 stages every level streams and the tile is written out from LDS
    float* dst = A.out + (size_t)bq * N * N;
    // the unmasked interior blocks add code: orders up to 4 have the registers for it (order
    // 8 would spill)
    constexpr bool kInner = K <= 4;
    float* copy = S + (1 << A.log2r) * A.rs;
    int l = level0 ? 1 : 0;
    if constexpr (STAGES) {
      if ((F - l) & 1) {
        level_stream_rot<NBLK, (K > 0)>(A, S, copy, l, row0);
        __syncthreads();
        ++l;
      }
      bool first_stage = true;
      for (; l + 2 < F; l += 2, first_stage = false) {
        if (first_stage) stage4<(K > 0), true, kInner>(A, S, l, row0);
        else stage4<(K > 0), false, kInner>(A, S, l, row0);
      }
      prefetch_landed();   // the next tile's rows, before this tile's stores
      if (first_stage)
        stage4_store<(K > 0), true, kInner>(A, S, l, row0, sig0, v, dst, k_lo);
      else
        stage4_store<(K > 0), false, kInner>(A, S, l, row0, sig0, v, dst, k_lo);
    } else {
      for (; l < F; ++l) {
        level_stream_rot<NBLK, (K > 0)>(A, S, copy, l, row0);
        __syncthreads();
      }
      // as in the deposit, a wave's 256 values lie in one row: row, output row and rotation
      // are wave-uniform, only the column is per lane
      prefetch_landed();   // the next tile's rows, before this tile's stores
      int stid = tid;
      asm volatile("" : "+v"(stid));
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        const int e4 = (stid + k * T) << 2;
        const int rho = __builtin_amdgcn_readfirstlane(e4 >> A.log2n);
        const int x = e4 & mask;
        const int i = brev_bits(rho, F);
        const int orow = (i << k_lo) + v;
        const int o = (sig0 + v * i) & mask;
        const float4 w = load4_rotated(S + rho * A.rs, x, o, mask);
        *reinterpret_cast<float4*>(dst + orow * N + x) = w;
      }
    }
    __syncthreads();
  }
}

// ---- column-tiled passes (no filter) ---------------------------------------------------------
// With lazy shifts, an output column of a pass depends only on the 2^F - 1 columns below it, so a
// tile can be a column block of W = 2^log2w columns plus a halo of `halo` columns below it, with
// no wrap-around inside the tile.  NCLS = 2 (a last back-projection pass of other than 5
// levels; one of 5 levels runs over square image tiles, further below): the block holds the
// matching column blocks of a class pair and sums them into the image.  NCLS = 1 (middle pass):
// one class, rows written with their pending rotation.
__device__ __forceinline__ int cat(int r, int c, int rs) { return r * rs + c + (c >> 5); }

// Load a tile of 2^log2r rows by halo + 2^log2w columns from each of NCLS classes into skewed
// LDS rows (class c at rows c R .. c R + R - 1).  Class c's tile starts at source column
// col[c] - halo (cyclically: only the halo can wrap, since col[c] + W <= N).  Both parts have
// power-of-two shapes; each class is read through its own buffer resource, so a load needs
// one 32-bit offset, and all of a thread's loads of a batch are in flight before it stores.
// A float4 at a column that is a multiple of 4 never straddles a skew step, so its four LDS
// words sit at one address plus 0..3.  The tile is stored after level 0 (below).  B: float4
// columns per class and thread whose loads are in flight together.
template <int NCLS, int B = 2>
__device__ void cols_load_tile(const PassArgs& A, float* S, int rs, const float* const* cls,
                               const int* col, int row0) {
  const int N = 1 << A.log2n, mask = N - 1;
  const int R = 1 << A.log2r;
  const int H = A.halo;
  const int T = blockDim.x, tid = threadIdx.x;
  const int lw = A.log2w - 2;                    // log2 of float4 per main row
  const int lh = 29 - __clz(H);                  // log2(H / 4)
  __amdgpu_buffer_rsrc_t rsrc[NCLS];
#pragma unroll
  for (int c = 0; c < NCLS; ++c)
    rsrc[c] = __builtin_amdgcn_make_buffer_rsrc((void*)cls[c], (short)0, N * N * 4, kBufferDword3);
  // Level 0 of the transposed transform is done here, on the loaded values: it pairs tile rows
  // 2m and 2m + 1 (relative shift 0), lower[x] = r0[x] + r1[x] and upper[x] = r0[x] +
  // r1[x - 1], so each thread loads the same float4 column of both rows.  r1[x - 1] at the
  // first column of a float4 is the previous float4's last value, held by the previous lane
  // (the previous float4 of the row) except at the start of a wave's run, where it is read
  // from memory; tile column 0 has no column below and stays as loaded (it only feeds
  // outputs below the halo), as in the LDS levels.
  auto butterfly = [&](int c, int m, int lc, const u32x4& a, const u32x4& b, float prev) {
    const float a0 = __uint_as_float(a.x), a1 = __uint_as_float(a.y);
    const float a2 = __uint_as_float(a.z), a3 = __uint_as_float(a.w);
    const float b0 = __uint_as_float(b.x), b1 = __uint_as_float(b.y);
    const float b2 = __uint_as_float(b.z), b3 = __uint_as_float(b.w);
    float* lo = S + (c * R + 2 * m) * rs + lc + (lc >> 5);
    float* up = lo + rs;
    lo[0] = a0 + b0;
    lo[1] = a1 + b1;
    lo[2] = a2 + b2;
    lo[3] = a3 + b3;
    up[0] = lc == 0 ? b0 : a0 + prev;
    up[1] = a1 + b0;
    up[2] = a2 + b1;
    up[3] = a3 + b2;
    if (lc == 0) lo[0] = a0;
  };
  const int lane = tid & 63;
  // main part: columns H .. H + W - 1 of the tile
  const int per = (R >> 1) << lw;                 // float4 columns of the row pairs
  for (int base = tid; base < per; base += B * T) {
    u32x4 va[NCLS][B], vb[NCLS][B];
    float pv[NCLS][B];
#pragma unroll
    for (int c = 0; c < NCLS; ++c)
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int e = base + k * T;
        if (e < per) {
          const int m = e >> lw, j = e & ((1 << lw) - 1);
          const int o0 = ((row0 + 2 * m) * N + col[c] + 4 * j) * 4;
          va[c][k] = __builtin_amdgcn_raw_buffer_load_b128(rsrc[c], o0, 0, 0);
          vb[c][k] = __builtin_amdgcn_raw_buffer_load_b128(rsrc[c], o0 + N * 4, 0, 0);
          // the value below the float4 in row 2m + 1, from memory where no lane holds it
          pv[c][k] = 0.f;
          if ((j & 63) == 0 || lane == 0)
            pv[c][k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
                rsrc[c], ((row0 + 2 * m + 1) * N + ((col[c] + 4 * j - 1) & mask)) * 4, 0, 0));
        }
      }
#pragma unroll
    for (int c = 0; c < NCLS; ++c)
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int e = base + k * T;
        // every lane takes part in the shuffle (the float4 of the previous lane)
        const float w = __shfl_up(__uint_as_float(vb[c][k].w), 1);
        if (e < per) {
          const int j = e & ((1 << lw) - 1);
          const float prev = ((j & 63) == 0 || lane == 0) ? pv[c][k] : w;
          butterfly(c, e >> lw, H + 4 * j, va[c][k], vb[c][k], prev);
        }
      }
  }
  // halo: columns 0 .. H - 1 of the tile, source columns col[c] - H .. col[c] - 1 cyclically
  const int perh = (R >> 1) << lh;
  for (int e0 = tid - lane; e0 < perh; e0 += T) {   // whole waves, for the shuffle
    const int e = e0 + lane;
    const int m = e >> lh, j = e & ((1 << lh) - 1);
    u32x4 va[NCLS], vb[NCLS];
    float pv[NCLS];
#pragma unroll
    for (int c = 0; c < NCLS; ++c) {
      va[c] = u32x4{0, 0, 0, 0};
      vb[c] = u32x4{0, 0, 0, 0};
      pv[c] = 0.f;
      if (e < perh) {
        const int o0 = ((row0 + 2 * m) * N + ((col[c] - H + 4 * j) & mask)) * 4;
        va[c] = __builtin_amdgcn_raw_buffer_load_b128(rsrc[c], o0, 0, 0);
        vb[c] = __builtin_amdgcn_raw_buffer_load_b128(rsrc[c], o0 + N * 4, 0, 0);
        if (j != 0 && lane == 0)
          pv[c] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
              rsrc[c], ((row0 + 2 * m + 1) * N + ((col[c] - H + 4 * j - 1) & mask)) * 4, 0, 0));
      }
    }
#pragma unroll
    for (int c = 0; c < NCLS; ++c) {
      const float w = __shfl_up(__uint_as_float(vb[c].w), 1);
      if (e < perh) butterfly(c, m, 4 * j, va[c], vb[c], lane == 0 ? pv[c] : w);
    }
  }
}

// One level on all units (class, row pair) of the block; walks each unit's columns from the
// top in batches of four 64-column blocks (reads before writes).  Columns below J + 1 are left
// as they are (they only feed outputs below the halo).
__device__ void cols_level(float* S, int rs, int log2r, int ncls, int wt, int l) {
  const int lane = threadIdx.x & 63, wave = wave_id(), waves = blockDim.x >> 6;
  const int pairs = 1 << (log2r - 1);
  const int units = ncls * pairs;
  const int R = 1 << log2r;
  const int nblk = (wt + 63) >> 6;
  const int pad = (nblk << 6) - wt;       // block bb covers columns bb * 64 - pad + lane
  for (int unit = wave; unit < units; unit += waves) {
    const int cls = unit / pairs, pair = unit - cls * pairs;
    const int ib = pair & ((1 << l) - 1), pp = pair >> l;
    const int r0 = (pp << (l + 1)) | ib, r1 = r0 | (1 << l);
    const int J = brev_bits(ib, l);
    float* base = S + cls * R * rs;
    for (int top = nblk - 1; top >= 0; top -= 4) {
      float va[4], vb[4];
#pragma unroll
      for (int u2 = 0; u2 < 4; ++u2) {
        const int c = (top - u2) * 64 + lane - pad;
        va[u2] = 0.f;
        vb[u2] = 0.f;
        if (top - u2 >= 0 && c >= J + 1 && c < wt) {
          const float v0 = base[cat(r0, c, rs)];
          va[u2] = v0 + base[cat(r1, c - J, rs)];
          vb[u2] = v0 + base[cat(r1, c - J - 1, rs)];
        }
      }
#pragma unroll
      for (int u2 = 0; u2 < 4; ++u2) {
        const int c = (top - u2) * 64 + lane - pad;
        if (top - u2 >= 0 && c >= J + 1 && c < wt) {
          base[cat(r0, c, rs)] = va[u2];
          base[cat(r1, c, rs)] = vb[u2];
        }
      }
    }
  }
}

// Column-tile level with a compile-time block count (immediate LDS offsets, as above).  Block
// bb >= 1 covers columns 64 bb - pad + lane, all of them >= J + 1; block 0 is masked.
template <int NBLK>
__device__ void cols_level_fast(float* S, int rs, int log2r, int ncls, int pad, int l) {
  const int lane = threadIdx.x & 63, wave = wave_id(), waves = blockDim.x >> 6;
  const int pairs = 1 << (log2r - 1);
  const int units = ncls * pairs;
  const int R = 1 << log2r;
  for (int unit = wave; unit < units; unit += waves) {
    const int cls = unit / pairs, pair = unit - cls * pairs;
    const int ib = pair & ((1 << l) - 1), pp = pair >> l;
    const int r0 = (pp << (l + 1)) | ib, r1 = r0 | (1 << l);
    const int J = brev_bits(ib, l);
    float* base = S + cls * R * rs;
    const int cb1 = 64 - pad + lane;
    const int c1 = cb1 - J, c2 = cb1 - J - 1;
    float* a0 = base + r0 * rs + cb1 + (cb1 >> 5);
    float* w1 = base + r1 * rs + cb1 + (cb1 >> 5);
    const float* a1 = base + r1 * rs + c1 + (c1 >> 5);
    const float* a2 = base + r1 * rs + c2 + (c2 >> 5);
#pragma unroll
    for (int top = NBLK - 1; top >= 1; top -= 4) {
      float va[4], vb[4];
#pragma unroll
      for (int u2 = 0; u2 < 4; ++u2) {
        const int k = top - u2;
        if (k >= 1) {
          const int off = 66 * (k - 1);
          const float v0 = a0[off];
          va[u2] = v0 + a1[off];
          vb[u2] = v0 + a2[off];
        }
      }
#pragma unroll
      for (int u2 = 0; u2 < 4; ++u2) {
        const int k = top - u2;
        if (k >= 1) {
          const int off = 66 * (k - 1);
          a0[off] = va[u2];
          w1[off] = vb[u2];
        }
      }
    }
    const int c = lane - pad;
    if (c >= J + 1) {
      const float v0 = base[cat(r0, c, rs)];
      const float v1 = base[cat(r1, c - J, rs)];
      const float v2 = base[cat(r1, c - J - 1, rs)];
      base[cat(r0, c, rs)] = v0 + v1;
      base[cat(r1, c, rs)] = v0 + v2;
    }
  }
}

// Two levels (l, l + 1) of a column tile in one LDS round trip: the radix-4 form of the first
// pass (see stage4) with the lazy shifts of a tile that carries no rotations (d01 = d23 = -J,
// e = -J2, J = brev(ib, l), J2 = brev(ib, l + 1)).  Reads below column 0 are clamped: those
// columns, like the ones the streaming form leaves untouched, only feed columns under the halo.
// Tiles of NB blocks of 61 columns (W + halo <= 61 NB), UPW units (four rows of one class) per
// wave.
template <int UPW, int NB>
__device__ __forceinline__ void cols_stage4(float* S, int rs, int log2r, int l, int wt) {
  const int lane = threadIdx.x & 63, wave = wave_id(), waves = blockDim.x >> 6;
  const int R = 1 << log2r;
  const int log2upc = log2r - 2;                   // units per class: R / 4
  int rb[UPW], J[UPW], J2[UPW];
#pragma unroll
  for (int k = 0; k < UPW; ++k) {
    const int unit = wave + k * waves;
    const int cls = unit >> log2upc, u = unit & ((1 << log2upc) - 1);
    const int pp = u >> l, ib = u & ((1 << l) - 1);
    rb[k] = cls * R + (pp << (l + 2)) + ib;
    J[k] = brev_bits(ib, l);
    J2[k] = brev_bits(ib, l + 1);
  }
  float o0[UPW * NB], o1[UPW * NB], o2[UPW * NB], o3[UPW * NB];
#pragma unroll
  for (int k = 0; k < UPW; ++k) {
    const float* p0 = S + rb[k] * rs;
    const float* p1 = p0 + (rs << l);
    const float* p2 = p0 + (rs << (l + 1));
    const float* p3 = p2 + (rs << l);
#pragma unroll
    for (int blk = 0; blk < NB; ++blk) {
      const int c = min(blk * 61 - 3 + lane, wt - 1);
      const int x0 = max(c, 0), x1 = max(c - J[k], 0), x2 = max(c - J2[k], 0);
      const int x3 = max(c - J2[k] - J[k], 0);
      const float a = p0[x0 + (x0 >> 5)];
      const float b = p1[x1 + (x1 >> 5)];
      const float f = p2[x2 + (x2 >> 5)];
      const float g = p3[x3 + (x3 >> 5)];
      const float A0 = a + b;
      const float A1 = a + lanes_shift_up_any(b);
      const float A2e = f + g;
      const float A3e = f + lanes_shift_up_any(g);
      const float t = lanes_shift_up_any(A3e);
      const int j = k * NB + blk;
      o0[j] = A0 + A2e;
      o2[j] = A0 + lanes_shift_up_any(A2e);
      o1[j] = A1 + t;
      o3[j] = A1 + lanes_shift_up_any(t);
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < UPW; ++k) {
    float* q = S + rb[k] * rs;
#pragma unroll
    for (int blk = 0; blk < NB; ++blk) {
      const int c = blk * 61 - 3 + lane;
      if (lane >= 3 && c < wt) {
        const int j = k * NB + blk;
        const int sk = c + (c >> 5);
        q[sk] = o0[j];
        q[(rs << l) + sk] = o1[j];
        q[(rs << (l + 1)) + sk] = o2[j];
        q[(rs << (l + 1)) + (rs << l) + sk] = o3[j];
      }
    }
  }
  __syncthreads();
}

// Levels 1 .. F - 1 of a column tile (level 0 was done by the loader): radix-4 stages when the
// tile has 5 blocks of 61 columns and one or two units per wave, else streaming levels; with an
// odd count the first level streams.
__device__ __forceinline__ void cols_levels(float* S, int rs, int log2r, int ncls, int wt, int F) {
  const int waves = blockDim.x >> 6;
  const int units = (ncls << log2r) >> 2;
  const int pad = 64 * ((wt + 63) >> 6) - wt;
  const bool r4 = F >= 3 && (wt + 60) / 61 == 5 && (units == waves || units == 2 * waves);
  int l = 1;
  for (; l < F && (!r4 || ((F - l) & 1)); ++l) {
    if (((wt + 63) >> 6) == 5) cols_level_fast<5>(S, rs, log2r, ncls, pad, l);
    else cols_level(S, rs, log2r, ncls, wt, l);
    __syncthreads();
  }
  for (; l < F; l += 2) {
    if (units == waves) cols_stage4<1, 5>(S, rs, log2r, l, wt);
    else cols_stage4<2, 5>(S, rs, log2r, l, wt);
  }
}

template <int NCLS>
__global__ void __launch_bounds__(512) fht_cols_kernel(PassArgs A) {
  extern __shared__ float S[];
  const int T = blockDim.x, tid = threadIdx.x;
  const int N = 1 << A.log2n, mask = N - 1;
  const int R = 1 << A.log2r;
  const int F = A.levels;
  const int W = 1 << A.log2w, H = A.halo, wt = W + H;
  const int rs = (wt + (wt >> 5) + 1) | 1;
  const int cblocks = N >> A.log2w;
  const int cb = blockIdx.x % cblocks;
  const int cx = cb << A.log2w;                 // first output column of the tile
  if constexpr (NCLS == 2) {
    const int strips = N >> A.log2r;
    const int rest = blockIdx.x / cblocks;
    const int j = rest % strips, b = rest / strips;
    const int qa = (A.out_mode == OUT_IMG_V) ? 0 : 2;
    const int row0 = j * R;
    const float* c0 = A.in + ((size_t)b * 4 + qa) * N * N;
    const float* c1 = c0 + (size_t)N * N;
    float* img = A.out + (size_t)b * N * N;
    const bool hpass = A.out_mode == OUT_IMG_H;
    const bool vec = R >= 4;                      // float4 image access along i (H) or u (V)
    const int n4 = (R * W) >> 2;
    {
      const float* cl[2] = {c0, c1};
      const int cc[2] = {cx, N - cx - W};
      cols_load_tile<2>(A, S, rs, cl, cc, row0);
    }
    // the H pass adds into image values that do not depend on the levels: load them now
    constexpr int kOld = 8;
    float4 old[kOld];
    if (hpass && vec) {
#pragma unroll
      for (int k = 0; k < kOld; ++k) {
        const int e4 = tid + k * T;
        if (e4 < n4) {
          const int i4 = (e4 & ((R >> 2) - 1)) << 2, u = e4 >> (A.log2r - 2);
          old[k] = *reinterpret_cast<const float4*>(img + (size_t)(cx + u) * N + row0 + i4);
        }
      }
    }
    __syncthreads();
    cols_levels(S, rs, A.log2r, 2, wt, F);
    const float* s0 = S;
    const float* s1 = S + R * rs;
    if (vec && !hpass) {
      // image[j R + i][cx + u] = c0[i][cx + u] + c1[i][N - 1 - cx - u], four u per thread
      for (int e4 = tid; e4 < n4; e4 += T) {
        const int i = e4 >> (A.log2w - 2), u = (e4 & ((W >> 2) - 1)) << 2;
        const int rho = brev_bits(i, F);
        // H, W and u are multiples of 4, so each class's four columns are one aligned group
        // inside a skew step: one address, immediate offsets (class 1 read backwards)
        const float* p0 = s0 + cat(rho, H + u, rs);
        const float* p1 = s1 + cat(rho, H + W - 4 - u, rs);
        float4 w;
        w.x = p0[0] + p1[3];
        w.y = p0[1] + p1[2];
        w.z = p0[2] + p1[1];
        w.w = p0[3] + p1[0];
        *reinterpret_cast<float4*>(img + (size_t)(row0 + i) * N + cx + u) = w;
      }
    } else if (vec) {
      // image[cx + u][j R + i] += c2[i][cx + u] + c3[i][N - 1 - cx - u], four i per thread
      auto add4 = [&](int e4, float4 o) {
        const int i = (e4 & ((R >> 2) - 1)) << 2, u = e4 >> (A.log2r - 2);
        // i is a multiple of 4 and F >= 2: rows i + 1, i + 2, i + 3 sit 2^(F-1), 2^(F-2) and
        // 3 2^(F-2) rows after row brev(i) in bit-reversed order
        const int d1 = rs << (F - 1), d2 = rs << (F - 2);
        const float* p0 = s0 + cat(brev_bits(i, F), H + u, rs);
        const float* p1 = s1 + cat(brev_bits(i, F), H + W - 1 - u, rs);
        float4 w;
        w.x = o.x + p0[0] + p1[0];
        w.y = o.y + p0[d1] + p1[d1];
        w.z = o.z + p0[d2] + p1[d2];
        w.w = o.w + p0[d1 + d2] + p1[d1 + d2];
        *reinterpret_cast<float4*>(img + (size_t)(cx + u) * N + row0 + i) = w;
      };
#pragma unroll
      for (int k = 0; k < kOld; ++k) {
        const int e4 = tid + k * T;
        if (e4 < n4) add4(e4, old[k]);
      }
      for (int e4 = tid + kOld * T; e4 < n4; e4 += T) {
        const int i = (e4 & ((R >> 2) - 1)) << 2, u = e4 >> (A.log2r - 2);
        add4(e4, *reinterpret_cast<const float4*>(img + (size_t)(cx + u) * N + row0 + i));
      }
    } else if (A.out_mode == OUT_IMG_V) {
      // image[j R + i][cx + u] = c0[i][cx + u] + c1[i][N - 1 - cx - u]
      for (int e = tid; e < R * W; e += T) {
        const int i = e >> A.log2w, u = e & (W - 1);
        const int rho = brev_bits(i, F);
        img[(size_t)(row0 + i) * N + cx + u] = s0[cat(rho, H + u, rs)] + s1[cat(rho, H + W - 1 - u, rs)];
      }
    } else {
      // image[cx + u][j R + i] += c2[i][cx + u] + c3[i][N - 1 - cx - u]
      for (int e = tid; e < R * W; e += T) {
        const int i = e & (R - 1), u = e >> A.log2r;
        const int rho = brev_bits(i, F);
        float* p = img + (size_t)(cx + u) * N + row0 + i;
        *p = *p + s0[cat(rho, H + u, rs)] + s1[cat(rho, H + W - 1 - u, rs)];
      }
    }
  } else {
    const int tiles = N >> A.log2r;
    const int rest = blockIdx.x / cblocks;
    const int tile = rest % tiles, bq = rest / tiles;
    const int vbits = A.k_hi - F;
    const int j = tile >> vbits, v = tile & ((1 << vbits) - 1);
    const int row0 = (j << A.k_hi) + (v << F);
    const int k_lo = A.k_hi - F;
    const float* cls = A.in + (size_t)bq * N * N;
    {
      const float* cl[1] = {cls};
      const int cc[1] = {cx};
      cols_load_tile<1>(A, S, rs, cl, cc, row0);
    }
    __syncthreads();
    cols_levels(S, rs, A.log2r, 1, wt, F);
    float* dst = A.out + (size_t)bq * N * N;
    // a wave writes 64 consecutive columns of one row (W >= 64): row, output row and rotation
    // are wave-uniform
    const int lane = tid & 63;
    for (int e0 = wave_id() << 6; e0 < R * W; e0 += T) {
      const int rho = e0 >> A.log2w, u = (e0 & (W - 1)) + lane;
      const int i = brev_bits(rho, F);
      const int orow = (((j << F) + i) << k_lo) + v;
      const int o = (v * i) & mask;
      dst[orow * N + ((cx + u + o) & mask)] = S[cat(rho, H + u, rs)];
    }
  }
}

// ---- last pass over square image tiles -------------------------------------------------------
// All four classes of the last back-projection pass (5 levels to go) in one block, which owns a
// 128 x 128 image tile: rows y0 .. y0 + 127, columns x0 .. x0 + 127 (eq 20-22).  Classes 0 and 1
// reach it through the 4 strips of rows y0 .. y0 + 127, column block x0:
//     image[y][x] = c0[y][x] + c1[y][N-1-x];
// classes 2 and 3 through the 4 strips of rows x0 .. x0 + 127, column block y0, transposed:
//     image[y][x] += c2[x][y] + c3[x][N-1-y].
// Each strip is a column tile of 32 rows by 128 + 32 columns (the halo below), run through
// level 0 in registers and levels 1 .. 4 in LDS, and added into accumulators held in registers;
// the additions are those of the split V and H kernels in the same order, so the results are
// bit-identical to them.  The image is written once and never read: 16 N^2 bytes in (plus the
// halo) and 4 N^2 out, against 28 N^2 (plus the halo) for the two launches.
//
// LDS layout: unskewed rows of kTileRs floats after a margin of kTileMargin floats (class c,
// row i at kTileMargin + (32 c + i) kTileRs).  Columns 0 .. 159 hold the tile; the radix-4
// stages compute 3 blocks of 61 columns (-3 .. 182) with no clamping: reads below column 0 land
// in the margin or in the padding of the row before, reads above 159 in the row's own padding,
// and those values only feed columns outside 32 .. 159, which nothing reads.  The padding also
// keeps every row 16-byte aligned (float4 deposits).
constexpr int kTileRs = 188;       // >= 186: written columns -3 .. 182 never reach another row's 0 .. 182
constexpr int kTileMargin = 64;    // >= 37: the lowest read is column -3 - J - J2 of row 0
constexpr int kTileLdsFloats = kTileMargin + 64 * kTileRs;

// Two levels (l, l + 1) of a tile in the layout above: the radix-4 form of the column passes
// (d01 = d23 = -J, e = -J2), two units (four rows of one class) per wave, 3 blocks of 61
// columns.  Every address is one per-unit base plus an immediate offset.  All reads end at a
// barrier before any write.
__device__ __forceinline__ void tile_stage4(float* S, int l) {
  constexpr int UPW = 2, NB = 3, rs = kTileRs;
  const int lane = threadIdx.x & 63, wave = wave_id(), waves = blockDim.x >> 6;
  float* q[UPW];
  int J[UPW], J2[UPW];
#pragma unroll
  for (int k = 0; k < UPW; ++k) {
    const int unit = wave + k * waves;
    const int cls = unit >> 3, u = unit & 7;         // 8 units of four rows per class
    const int pp = u >> l, ib = u & ((1 << l) - 1);
    const int rb = cls * 32 + (pp << (l + 2)) + ib;
    J[k] = brev_bits(ib, l);
    J2[k] = brev_bits(ib, l + 1);
    q[k] = S + rb * rs + lane - 3;
  }
  float o0[UPW * NB], o1[UPW * NB], o2[UPW * NB], o3[UPW * NB];
#pragma unroll
  for (int k = 0; k < UPW; ++k) {
    const float* p0 = q[k];
    const float* p1 = p0 + (rs << l) - J[k];
    const float* p2 = p0 + (rs << (l + 1)) - J2[k];
    const float* p3 = p2 + (rs << l) - J[k];
#pragma unroll
    for (int blk = 0; blk < NB; ++blk) {
      const float a = p0[61 * blk];
      const float b = p1[61 * blk];
      const float f = p2[61 * blk];
      const float g = p3[61 * blk];
      const float A0 = a + b;
      const float A1 = a + lanes_shift_up_any(b);
      const float A2e = f + g;
      const float A3e = f + lanes_shift_up_any(g);
      const float t = lanes_shift_up_any(A3e);
      const int j = k * NB + blk;
      o0[j] = A0 + A2e;
      o2[j] = A0 + lanes_shift_up_any(A2e);
      o1[j] = A1 + t;
      o3[j] = A1 + lanes_shift_up_any(t);
    }
  }
  __syncthreads();
  auto put = [&](int k, int blk) {
    float* p = q[k];
    const int j = k * NB + blk;
    p[61 * blk] = o0[j];
    p[(rs << l) + 61 * blk] = o1[j];
    p[(rs << (l + 1)) + 61 * blk] = o2[j];
    p[(rs << (l + 1)) + (rs << l) + 61 * blk] = o3[j];
  };
  // blocks above the first: lanes 0 .. 2 repeat the previous block's top columns without their
  // shifted inputs and are left out (no two lanes write one word, in whatever order the
  // compiler groups the stores); the first block's lanes 0 .. 2 write into the padding
  if (lane >= 3) {
#pragma unroll
    for (int k = 0; k < UPW; ++k)
#pragma unroll
      for (int blk = 1; blk < NB; ++blk) put(k, blk);
  }
#pragma unroll
  for (int k = 0; k < UPW; ++k) put(k, 0);
  __syncthreads();
}

// One strip in registers between its loads and its LDS deposit, so that the next strip's loads
// are in flight while the current one runs its levels.  Thread t takes row pair m = t >> 5: the
// float4 at tile column 32 + 4 j (j = t & 31) of both rows, and the halo column j of both rows,
// for each class of the pair.
struct StripRegs {
  u32x4 a[2], b[2];   // main float4 of rows 2m, 2m + 1
  float pv[2];        // row 2m + 1 one column below the float4 (j = 0 only)
  float ha[2], hb[2]; // halo column j of rows 2m, 2m + 1
};

__device__ __forceinline__ void strip_issue(StripRegs& P, const float* c0, size_t nn, int col0,
                                            int row0, int log2n) {
  const int N = 1 << log2n, mask = N - 1;
  const int tid = threadIdx.x, m = tid >> 5, j = tid & 31;
#pragma unroll
  for (int cl = 0; cl < 2; ++cl) {
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(c0 + cl * nn), (short)0, N * N * 4, kBufferDword3);
    const int col = cl == 0 ? col0 : N - col0 - 128;
    const int rowb = (row0 + 2 * m) * N;
    const int o0 = (rowb + col + 4 * j) * 4;
    P.a[cl] = __builtin_amdgcn_raw_buffer_load_b128(rsrc, o0, 0, 0);
    P.b[cl] = __builtin_amdgcn_raw_buffer_load_b128(rsrc, o0 + N * 4, 0, 0);
    P.pv[cl] = 0.f;
    if (j == 0)
      P.pv[cl] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
          rsrc, (rowb + N + ((col - 1) & mask)) * 4, 0, 0));
    const int oh = (rowb + ((col - 32 + j) & mask)) * 4;
    P.ha[cl] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rsrc, oh, 0, 0));
    P.hb[cl] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rsrc, oh + N * 4, 0, 0));
  }
}

// Level 0 on a strip's registers (lower = r0[x] + r1[x], upper = r0[x] + r1[x - 1]; tile column
// 0 stays as loaded, as in the column loader) and the deposit into the tile layout.
__device__ __forceinline__ void strip_deposit(const StripRegs& P, float* S) {
  const int tid = threadIdx.x, m = tid >> 5, j = tid & 31;
#pragma unroll
  for (int cl = 0; cl < 2; ++cl) {
    const float a0 = __uint_as_float(P.a[cl].x), a1 = __uint_as_float(P.a[cl].y);
    const float a2 = __uint_as_float(P.a[cl].z), a3 = __uint_as_float(P.a[cl].w);
    const float b0 = __uint_as_float(P.b[cl].x), b1 = __uint_as_float(P.b[cl].y);
    const float b2 = __uint_as_float(P.b[cl].z), b3 = __uint_as_float(P.b[cl].w);
    const float w = __shfl_up(b3, 1);                 // the previous float4 of row 2m + 1
    const float prev = j == 0 ? P.pv[cl] : w;
    float* lo = S + kTileMargin + (cl * 32 + 2 * m) * kTileRs;
    float* up = lo + kTileRs;
    float4* lo4 = reinterpret_cast<float4*>(__builtin_assume_aligned(lo + 32 + 4 * j, 16));
    float4* up4 = reinterpret_cast<float4*>(__builtin_assume_aligned(up + 32 + 4 * j, 16));
    *lo4 = make_float4(a0 + b0, a1 + b1, a2 + b2, a3 + b3);
    *up4 = make_float4(a0 + prev, a1 + b0, a2 + b1, a3 + b2);
    const float hbm = __shfl_up(P.hb[cl], 1);
    lo[j] = j == 0 ? P.ha[cl] : P.ha[cl] + P.hb[cl];
    up[j] = j == 0 ? P.hb[cl] : P.ha[cl] + hbm;
  }
}

// Thread t owns rows (t >> 5) + 16 m (m < 8) and columns (t & 31) + 32 k (k < 4) of the tile.
// At most 128 VGPRs, so that two blocks (16 waves) share a compute unit.
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
fht_image_tile_kernel(PassArgs A) {
  extern __shared__ float S[];
  constexpr int F = 5, R = 32, TT = 128, W = 128, H = 32, NS = TT / R, rs = kTileRs;
  const int tid = threadIdx.x;
  const int N = 1 << A.log2n;
  const int tpr = N / TT;                            // tiles per image row
  const int per_slice = tpr * tpr;
  // consecutive tiles of a row go to one XCD (blocks are dealt to the 8 XCDs in turn), so the
  // halo columns that neighbouring tiles share are read through that XCD's L2
  int id = blockIdx.x;
  if ((gridDim.x & 7) == 0) id = (id & 7) * (gridDim.x >> 3) + (id >> 3);
  const int b = id / per_slice, rest = id - b * per_slice;
  const int ty = rest / tpr, tx = rest - ty * tpr;
  const int y0 = ty * TT, x0 = tx * TT;
  const size_t nn = (size_t)N * N;
  const float* lino = A.in + (size_t)b * 4 * nn;
  const int c = tid & 31, r = tid >> 5;
  float acc[8][4];
#pragma unroll
  for (int m = 0; m < 8; ++m)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[m][k] = 0.f;
  float* T0 = S + kTileMargin;
  const float* s0 = T0;
  const float* s1 = T0 + R * rs;
  StripRegs P;
  strip_issue(P, lino, nn, x0, y0, A.log2n);
  for (int ph = 0; ph < 2 * NS; ++ph) {
    const bool hpart = ph >= NS;
    const int s = hpart ? ph - NS : ph;
    strip_deposit(P, S);
    __syncthreads();
    if (ph + 1 < 2 * NS) {
      // the next strip's loads go out now and land during this strip's levels
      const int pn = ph + 1;
      const bool hn = pn >= NS;
      const int sn = hn ? pn - NS : pn;
      strip_issue(P, lino + (hn ? 2 : 0) * nn, nn, hn ? y0 : x0, (hn ? x0 : y0) + sn * R, A.log2n);
    }
    // levels 1 .. 4 as two radix-4 stages
    tile_stage4(T0, 1);
    tile_stage4(T0, 3);
    if (!hpart) {
      // tile rows 32 s .. 32 s + 31: this thread's rows r and r + 16 of the strip, columns
      // x = c + 32 k: class 0 at H + x, class 1 at H + W - 1 - x
#pragma unroll
      for (int s2 = 0; s2 < NS; ++s2) {
        if (s2 != s) continue;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int rho = brev_bits(r + 16 * h, F);
          const float* p0 = s0 + rho * rs + H + c;
          const float* p1 = s1 + rho * rs + (H + W - 1) - c;
#pragma unroll
          for (int k = 0; k < 4; ++k) acc[2 * s2 + h][k] += p0[32 * k] + p1[-32 * k];
        }
      }
    } else {
      // tile columns 32 s .. 32 s + 31 are strip rows: this thread's column c (strip row c),
      // its rows u = r + 16 m: class 2 at column H + u, class 3 at H + W - 1 - u
      const int rho = brev_bits(c, F);
      const float* p0 = s0 + rho * rs + H + r;
      const float* p1 = s1 + rho * rs + (H + W - 1) - r;
#pragma unroll
      for (int s2 = 0; s2 < NS; ++s2) {
        if (s2 != s) continue;
#pragma unroll
        for (int m = 0; m < 8; ++m) acc[m][s2] = acc[m][s2] + p0[16 * m] + p1[-16 * m];
      }
    }
    __syncthreads();
  }
  float* img = A.out + (size_t)b * nn + (size_t)y0 * N + x0;
#pragma unroll
  for (int m = 0; m < 8; ++m)
#pragma unroll
    for (int k = 0; k < 4; ++k) img[(size_t)(r + 16 * m) * N + c + 32 * k] = acc[m][k];
}

// ---- last pass of 7 levels over square image tiles ----------------------------------------------
// The same image tile as above (128 x 128, all four classes, the image written once), for a last
// pass of 7 levels: each class reaches the tile through one strip of 128 rows (the tile's rows
// for classes 0 and 1, its columns for classes 2 and 3) by 128 + 128 columns (the halo below).
// A strip fills the LDS, so the block runs the classes one after the other: level 0 in
// registers at the deposit, levels 1 .. 6 as three radix-4 stages, then the strip is added
// into accumulators held in registers (class 0, + class 1, then + class 2, + class 3: the
// additions, and their order, of the other last-pass kernels, so results are bit-identical).
// The next strip's loads are in flight while the current one runs its levels.
//
// LDS layout: one class, rows of kT7Rs floats after a margin of kT7Margin floats (row i at
// kT7Margin + i kT7Rs).  Columns 0 .. 255 hold the strip; the stages compute 5 blocks of 61
// columns (-3 .. 301) with no clamping: reads below column 0 land in the margin or the row
// before's padding, writes of columns -3 .. -1 in the row before's padding, columns above 255
// are garbage, and none of these feed columns 128 .. 255, the only ones read out (an output
// column depends only on the 127 columns below it).
constexpr int kT7Rows = 128, kT7Cols = 256;
constexpr int kT7Rs = 308;       // > 304 + 3: rows written over -3 .. 304 never overlap
constexpr int kT7Margin = 128;   // >= 100: the lowest read is column -3 - 31 - 63 of row 0
constexpr int kT7LdsFloats = kT7Margin + kT7Rows * kT7Rs;
static_assert(kT7LdsFloats * 4 <= kLdsBudget, "a 128-row strip fits the LDS");
static_assert((kT7Rs % 4) == 0 && (kT7Margin % 4) == 0, "16-byte aligned rows");

// Levels (l, l + 1) of a 128-row strip (l = 1, 3, 5): 32 units of four rows, two per wave (16
// waves), 5 blocks of 61 columns each; the radix-4 form of tile_stage4.  A unit's rows belong to
// no other unit of the stage, so a wave reads all blocks of one unit, writes them, then takes
// its next unit, with no barrier in between.  (Reads at negative columns reach into the row
// before, which another wave may be rewriting; they only feed columns below 128 - 127 + ...,
// i.e. columns that no output reads, as everything below column 0 does.)
__device__ __forceinline__ void tile7_stage4(float* S, int l) {
  constexpr int UPW = 2, NB = 5, rs = kT7Rs;
  const int lane = threadIdx.x & 63, wave = wave_id(), waves = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < UPW; ++k) {
    const int u = wave + k * waves;                  // 32 units of four rows
    const int pp = u >> l, ib = u & ((1 << l) - 1);
    const int rb = (pp << (l + 2)) + ib;
    const int J = brev_bits(ib, l);
    const int J2 = brev_bits(ib, l + 1);
    float* p0 = S + rb * rs + lane - 3;
    const float* p1 = p0 + (rs << l) - J;
    const float* p2 = p0 + (rs << (l + 1)) - J2;
    const float* p3 = p2 + (rs << l) - J;
    float o0[NB], o1[NB], o2[NB], o3[NB];
#pragma unroll
    for (int blk = 0; blk < NB; ++blk) {
      const float a = p0[61 * blk];
      const float b = p1[61 * blk];
      const float f = p2[61 * blk];
      const float g = p3[61 * blk];
      const float A0 = a + b;
      const float A1 = a + lanes_shift_up_any(b);
      const float A2e = f + g;
      const float A3e = f + lanes_shift_up_any(g);
      const float t = lanes_shift_up_any(A3e);
      o0[blk] = A0 + A2e;
      o2[blk] = A0 + lanes_shift_up_any(A2e);
      o1[blk] = A1 + t;
      o3[blk] = A1 + lanes_shift_up_any(t);
    }
    // every read of the unit is done (its values are in registers) before its first write
    asm volatile("" ::: "memory");
    auto put = [&](int blk) {
      p0[61 * blk] = o0[blk];
      p0[(rs << l) + 61 * blk] = o1[blk];
      p0[(rs << (l + 1)) + 61 * blk] = o2[blk];
      p0[(rs << (l + 1)) + (rs << l) + 61 * blk] = o3[blk];
    };
    // as in tile_stage4: lanes 0 .. 2 of the blocks above the first are left out (they repeat
    // the previous block's top columns without their shifted inputs)
    if (lane >= 3) {
#pragma unroll
      for (int blk = 1; blk < NB; ++blk) put(blk);
    }
    put(0);
  }
  __syncthreads();
}

// One 128-row strip in registers: thread t takes row pair m = t >> 4 and the float4 columns
// 4 (j + 16 i), j = t & 15, i < 4, of both rows (256 columns from `col` - 128, cyclically).
struct Strip7Regs {
  u32x4 a[4], b[4];
};

__device__ __forceinline__ void strip7_issue(Strip7Regs& P, const float* cls, int col, int row0,
                                             int log2n) {
  const int N = 1 << log2n, mask = N - 1;
  const int tid = threadIdx.x, m = tid >> 4, j = tid & 15;
  const __amdgpu_buffer_rsrc_t rsrc =
      __builtin_amdgcn_make_buffer_rsrc((void*)cls, (short)0, N * N * 4, kBufferDword3);
  const int rowb = (row0 + 2 * m) * N;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int o = (rowb + ((col - 128 + 4 * (j + 16 * i)) & mask)) * 4;
    P.a[i] = __builtin_amdgcn_raw_buffer_load_b128(rsrc, o, 0, 0);
    P.b[i] = __builtin_amdgcn_raw_buffer_load_b128(rsrc, o + N * 4, 0, 0);
  }
}

// Level 0 on the strip's registers (lower = r0[x] + r1[x], upper = r0[x] + r1[x - 1]) and the
// deposit.  r1[x - 1] at the first column of a float4 is the last value of the float4 before
// (the lane below, or lane 15 of the previous i); strip column 0 has none and is not needed.
__device__ __forceinline__ void strip7_deposit(const Strip7Regs& P, float* S) {
  const int tid = threadIdx.x, m = tid >> 4, j = tid & 15;
  float* lo = S + kT7Margin + (2 * m) * kT7Rs;
  float* up = lo + kT7Rs;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float a0 = __uint_as_float(P.a[i].x), a1 = __uint_as_float(P.a[i].y);
    const float a2 = __uint_as_float(P.a[i].z), a3 = __uint_as_float(P.a[i].w);
    const float b0 = __uint_as_float(P.b[i].x), b1 = __uint_as_float(P.b[i].y);
    const float b2 = __uint_as_float(P.b[i].z), b3 = __uint_as_float(P.b[i].w);
    const float below = __shfl_up(b3, 1, 16);                       // float4 j - 1, same i
    const float wrap = i > 0 ? __shfl(__uint_as_float(P.b[i - 1].w), 15, 16) : 0.f;
    const float prev = j == 0 ? wrap : below;
    const int x = 4 * (j + 16 * i);
    float4* lo4 = reinterpret_cast<float4*>(__builtin_assume_aligned(lo + x, 16));
    float4* up4 = reinterpret_cast<float4*>(__builtin_assume_aligned(up + x, 16));
    *lo4 = make_float4(a0 + b0, a1 + b1, a2 + b2, a3 + b3);
    *up4 = make_float4(a0 + prev, a1 + b0, a2 + b1, a3 + b2);
  }
}

// Thread t owns rows (t >> 5) + 32 m and columns (t & 31) + 32 k (m, k < 4) of the tile.
__global__ void __launch_bounds__(1024) fht_image_tile7_kernel(PassArgs A) {
  extern __shared__ float S[];
  constexpr int F = 7, TT = 128, W = 128, H = 128, rs = kT7Rs;
  const int tid = threadIdx.x;
  const int N = 1 << A.log2n;
  const int tpr = N / TT;
  const int per_slice = tpr * tpr;
  // consecutive tiles of a row go to one XCD, whose L2 then serves the halo columns they share
  int id = blockIdx.x;
  if ((gridDim.x & 7) == 0) id = (id & 7) * (gridDim.x >> 3) + (id >> 3);
  const int b = id / per_slice, rest = id - b * per_slice;
  const int ty = rest / tpr, tx = rest - ty * tpr;
  const int y0 = ty * TT, x0 = tx * TT;
  const size_t nn = (size_t)N * N;
  const float* lino = A.in + (size_t)b * 4 * nn;
  const int c = tid & 31, r = tid >> 5;
  float acc[4][4];
  const float* T0 = S + kT7Margin;
  // class q's strip: rows (q < 2 ? y0 : x0) .. + 127, column block at (q even ? x0 or y0 : the
  // mirrored block)
  auto issue = [&](Strip7Regs& P, int q) {
    const int blk = q < 2 ? x0 : y0;
    const int col = (q & 1) ? N - blk - W : blk;
    strip7_issue(P, lino + q * nn, col, q < 2 ? y0 : x0, A.log2n);
  };
  Strip7Regs P;
  issue(P, 0);
  for (int q = 0; q < 4; ++q) {
    strip7_deposit(P, S);
    __syncthreads();
    if (q + 1 < 4) issue(P, q + 1);
    tile7_stage4(S + kT7Margin, 1);
    tile7_stage4(S + kT7Margin, 3);
    tile7_stage4(S + kT7Margin, 5);
    if (q < 2) {
      // image row i = r + 32 m is strip row brev(i); column x = c + 32 k is strip column
      // H + x (class 0) or H + W - 1 - x (class 1)
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const float* row = T0 + brev_bits(r + 32 * m, F) * rs;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if (q == 0) acc[m][k] = row[H + c + 32 * k];
          else acc[m][k] = acc[m][k] + row[H + W - 1 - c - 32 * k];
        }
      }
    } else {
      // image column x = c + 32 k is strip row brev(x); row y = r + 32 m is strip column H + y
      // (class 2) or H + W - 1 - y (class 3)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float* row = T0 + brev_bits(c + 32 * k, F) * rs;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          if (q == 2) acc[m][k] = acc[m][k] + row[H + r + 32 * m];
          else acc[m][k] = acc[m][k] + row[H + W - 1 - r - 32 * m];
        }
      }
    }
    __syncthreads();
  }
  float* img = A.out + (size_t)b * nn + (size_t)y0 * N + x0;
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int k = 0; k < 4; ++k) img[(size_t)(r + 32 * m) * N + c + 32 * k] = acc[m][k];
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

template <int L, int K, bool STREAM, bool REM>
hipError_t launch_lksd(const PassArgs& a, int batch, hipStream_t stream) {
  const int N = 1 << a.log2n;
  const int R = 1 << a.log2r;
  const int threads = R << a.log2c;
  const size_t lds = pass_lds_bytes(a);
  const int tiles = N >> a.log2r;
  if (a.out_mode == OUT_IMG_V || a.out_mode == OUT_IMG_H) {
    if constexpr (L <= 32 || K == 0)
      return launch_kernel(fht_combine_kernel<L, K, STREAM, REM>, a, batch * tiles, threads,
                           lds, stream);
    else
      return hipErrorInvalidValue;   // the filter runs in a combining pass only when N <= 128
  }
  return launch_kernel(fht_rows_kernel<L, K, STREAM, REM>, a, batch * 4 * tiles, threads, lds,
                       stream);
}

// The remainder term of the first-difference numerator exists for orders >= 2 only.
template <int L, int K, bool STREAM>
hipError_t launch_lks(const PassArgs& a, int batch, hipStream_t stream) {
  if constexpr (K >= 2) {
    if (a.rem) return launch_lksd<L, K, STREAM, true>(a, batch, stream);
  }
  return launch_lksd<L, K, STREAM, false>(a, batch, stream);
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

// The first-pass kernel of order K, with the numerator's remainder term when the plan's
// coefficients have one (orders >= 2, unbalanced numerators).
template <int L, int K, int NBLK, bool WIDE, bool STAGES>
hipError_t launch_first_ks(const PassArgs& a, int grid, int threads, size_t lds,
                           hipStream_t stream) {
  if constexpr (K >= 2) {
    if (a.rem)
      return launch_kernel(fht_first_kernel<L, K, NBLK, WIDE, true, STAGES>, a, grid, threads,
                           lds, stream);
  }
  return launch_kernel(fht_first_kernel<L, K, NBLK, WIDE, false, STAGES>, a, grid, threads, lds,
                       stream);
}
template <int L, int K, int NBLK, bool WIDE>
hipError_t launch_first_k(const PassArgs& a, int grid, int threads, size_t lds,
                          hipStream_t stream) {
  if (first_pass_stages(a, threads, K))
    return launch_first_ks<L, K, NBLK, WIDE, true>(a, grid, threads, lds, stream);
  return launch_first_ks<L, K, NBLK, WIDE, false>(a, grid, threads, lds, stream);
}

template <int L, int NBLK>
hipError_t launch_first_ln(const PassArgs& a, int grid, hipStream_t stream) {
  const int threads = (1 << a.log2r) << a.log2c;
  const size_t lds = pass_lds_bytes(a) + first_xchg_floats(a) * sizeof(float);
  if (a.log2c > 6) {
    // rows of 128 chunks (N = 4096) over two waves: 16 blocks per unit, orders up to 4
    if constexpr (NBLK == 16) {
      switch (a.order) {
        case 0: return launch_first_k<L, 0, 16, true>(a, grid, threads, lds, stream);
        case 1: return launch_first_k<L, 1, 16, true>(a, grid, threads, lds, stream);
        case 2: return launch_first_k<L, 2, 16, true>(a, grid, threads, lds, stream);
        case 3: return launch_first_k<L, 3, 16, true>(a, grid, threads, lds, stream);
        case 4: return launch_first_k<L, 4, 16, true>(a, grid, threads, lds, stream);
        default: break;
      }
    }
    return hipErrorInvalidValue;
  }
  switch (a.order) {
    case 0: return launch_first_k<L, 0, NBLK, false>(a, grid, threads, lds, stream);
    case 1: return launch_first_k<L, 1, NBLK, false>(a, grid, threads, lds, stream);
    case 2: return launch_first_k<L, 2, NBLK, false>(a, grid, threads, lds, stream);
    case 3: return launch_first_k<L, 3, NBLK, false>(a, grid, threads, lds, stream);
    case 4: return launch_first_k<L, 4, NBLK, false>(a, grid, threads, lds, stream);
    case 8: return launch_first_k<L, 8, NBLK, false>(a, grid, threads, lds, stream);
    default: return hipErrorInvalidValue;
  }
}

// 64-column blocks per streaming unit of a pass: W / 64 with W = N / max(1, waves / pairs).
inline int stream_blocks(const PassArgs& a) {
  const int threads = (1 << a.log2r) << a.log2c;
  const int waves = threads >> 6, pairs = 1 << (a.log2r - 1);
  const int segs = waves > pairs ? waves / pairs : 1;
  return ((1 << a.log2n) / segs) >> 6;
}

template <int L>
hipError_t launch_first_l(const PassArgs& a, int grid, hipStream_t stream) {
  switch (stream_blocks(a)) {
    case 4: return launch_first_ln<L, 4>(a, grid, stream);
    case 8: return launch_first_ln<L, 8>(a, grid, stream);
    case 16: return launch_first_ln<L, 16>(a, grid, stream);
    default: return hipErrorInvalidValue;
  }
}

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
