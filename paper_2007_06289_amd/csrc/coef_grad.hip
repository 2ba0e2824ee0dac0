// Gradient of a loss with respect to the coefficients of the recursive ramp pair (Sec. 3,
// eq 9-13), for learning them.  For one row in window order, with g = c_t dL/d(out):
//   causal part   A y+ = B x      ->  lam = A^-T g  (anticausal recursion of g, feed-forward 1)
//   anticausal    y- mirrored     ->  mu  = causal recursion of g
//   dL/db_k =  sum_i lam(i) x(i-k) + sum_i mu(i) x(i+k)
//   dL/da_k = -sum_i lam(i) y+(i-k) - sum_i mu(i) y-(i+k)     (k = 1..K)
// (A, B the lower-triangular Toeplitz matrices of 1 + sum a_k z^-k and sum b_k z^-k.)  All four
// recursions run in the chunked form of the filter: each chunk from zero state, a scan of the
// end states through Phi^(L 2^j) over the row's lanes, then the response to the entering state.
// Each block writes its per-coefficient sums to `partial`; a second kernel adds the blocks of
// each coefficient group in a fixed order (deterministic).
#include "fhtfbp_internal.h"

namespace fhtfbp {
namespace {

__device__ __forceinline__ int skew(int s, int log2l) { return s + (s >> log2l); }

// Exact recursion over one chunk.  DIR = +1 causal (positions base..base+L-1), -1 anticausal.
// `in(p)` gives the input at window position p (zero outside the window).  NB feed-forward
// taps.  y[i] is the output at position base + i; ent[k] the output at the k-th position before
// the chunk in the direction of the recursion (base - 1 - k, or base + L + k).
template <int L, int K, int NB, int DIR, typename In>
__device__ void chunk_rec(In in, const float* bk, const float* ak, const float* phi, int c, int C,
                          int levels, int base, float (&y)[L], float (&ent)[K]) {
  float st[K];
#pragma unroll
  for (int k = 0; k < K; ++k) st[k] = 0.f;
#pragma unroll
  for (int s = 0; s < L; ++s) {
    const int i = (DIR > 0) ? s : L - 1 - s;
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < NB; ++k) acc = fmaf(bk[k], in(base + i - DIR * k), acc);
#pragma unroll
    for (int k = 0; k < K; ++k) acc = fmaf(-ak[k], st[k], acc);
    y[i] = acc;
#pragma unroll
    for (int k = K - 1; k > 0; --k) st[k] = st[k - 1];
    st[0] = acc;
  }
  float tv[K];
#pragma unroll
  for (int k = 0; k < K; ++k) tv[k] = st[k];
  for (int j = 0; (1 << j) < C && j < levels; ++j) {   // the plan's scan depth
    const int d = 1 << j;
    float u[K];
#pragma unroll
    for (int k = 0; k < K; ++k) u[k] = (DIR > 0) ? __shfl_up(tv[k], d, C) : __shfl_down(tv[k], d, C);
    const bool take = (DIR > 0) ? (c >= d) : (c + d < C);
    if (take) {
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
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float v = (C > 1) ? ((DIR > 0) ? __shfl_up(tv[k], 1, C) : __shfl_down(tv[k], 1, C)) : 0.f;
    ent[k] = ((DIR > 0) ? (c == 0) : (c == C - 1)) ? 0.f : v;
    st[k] = ent[k];
  }
#pragma unroll
  for (int s = 0; s < L; ++s) {
    const int i = (DIR > 0) ? s : L - 1 - s;
    float z = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) z = fmaf(-ak[k], st[k], z);
    y[i] += z;
#pragma unroll
    for (int k = K - 1; k > 0; --k) st[k] = st[k - 1];
    st[0] = z;
  }
}

// Block: R rows (one class, consecutive slope indices) of one slice; threads (row, chunk).
template <int L, int K>
__global__ void __launch_bounds__(512) coef_grad_kernel(PassArgs A, const float* __restrict__ gin,
                                                        double* __restrict__ partial) {
  extern __shared__ float S[];
  const int N = 1 << A.log2n, mask = N - 1;
  const int R = 1 << A.log2r, C = 1 << A.log2c;
  const int tiles = N >> A.log2r;
  const int tile = blockIdx.x % tiles, bq = blockIdx.x / tiles;
  const int q = bq & 3;
  const int row0 = tile * R;
  float* X = S;
  float* Gs = S + R * A.rs;
  // load x and g rows (natural shift order, skewed): four consecutive samples per load (one
  // chunk, so four consecutive skewed slots), and each thread issues the loads of 4 rounds
  // before their stores, so that their memory latencies overlap
  const float* xs = A.in + ((size_t)bq * N + row0) * N;
  const float* gs = gin + ((size_t)bq * N + row0) * N;
  if (((reinterpret_cast<uintptr_t>(xs) | reinterpret_cast<uintptr_t>(gs)) & 15) == 0) {
    constexpr int U = 4;
    const int total4 = (R * N) >> 2;
    for (int e0 = threadIdx.x; e0 < total4; e0 += U * blockDim.x) {
      float4 xv[U], gv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * blockDim.x;
        if (e < total4) {
          xv[u] = reinterpret_cast<const float4*>(xs)[e];
          gv[u] = reinterpret_cast<const float4*>(gs)[e];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * blockDim.x;
        if (e < total4) {
          const int r = (4 * e) >> A.log2n, s = (4 * e) & mask;
          float* xd = X + r * A.rs + skew(s, A.log2l);
          float* gd = Gs + r * A.rs + skew(s, A.log2l);
          xd[0] = xv[u].x, xd[1] = xv[u].y, xd[2] = xv[u].z, xd[3] = xv[u].w;
          gd[0] = gv[u].x, gd[1] = gv[u].y, gd[2] = gv[u].z, gd[3] = gv[u].w;
        }
      }
    }
  } else {
    for (int e = threadIdx.x; e < R * N; e += blockDim.x) {
      const int r = e >> A.log2n, s = e & mask;
      X[r * A.rs + skew(s, A.log2l)] = xs[e];
      Gs[r * A.rs + skew(s, A.log2l)] = gs[e];
    }
  }
  __syncthreads();
  const int r = threadIdx.x >> A.log2c, c = threadIdx.x & (C - 1);
  const int t = row0 + r;
  const int g = ((q * N + t) * A.groups) / (4 * N);
  const float* cf = A.coef + (size_t)g * A.coef_stride;
  float bk[K], ak[K], one[1] = {1.f};
#pragma unroll
  for (int k = 0; k < K; ++k) {
    bk[k] = cf[k];
    ak[k] = cf[K + k];
  }
  const float* phi = cf + 2 * K;
  const int sig = A.sigma[t];
  const float ct = A.scale[t];
  const int base = c * L;
  const float* xr = X + r * A.rs;
  const float* gr = Gs + r * A.rs;
  auto xin = [&](int p) -> float {
    const int s = (sig + ((p < 0 || p >= N) ? 0 : p)) & mask;
    const float v = xr[skew(s, A.log2l)];
    return (p >= 0 && p < N) ? v : 0.f;
  };
  auto gin_ = [&](int p) -> float {
    const int s = (sig + ((p < 0 || p >= N) ? 0 : p)) & mask;
    const float v = gr[skew(s, A.log2l)];
    return (p >= 0 && p < N) ? ct * v : 0.f;
  };
  // this lane's input samples (positions base - K .. base + L + K - 1) and output gradient
  // samples (base .. base + L - 1), read from LDS once; every later use has a fixed offset
  float xv[L + 2 * K], gv[L];
#pragma unroll
  for (int j = 0; j < L + 2 * K; ++j) xv[j] = xin(base - K + j);
#pragma unroll
  for (int j = 0; j < L; ++j) gv[j] = gin_(base + j);
  auto xreg = [&](int p) -> float { return xv[p - base + K]; };
  auto greg = [&](int p) -> float { return gv[p - base]; };
  float db[K], da[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    db[k] = 0.f;
    da[k] = 0.f;
  }
  {
    float yp[L], ep[K], lam[L], el[K];
    chunk_rec<L, K, K, +1>(xreg, bk, ak, phi, c, C, A.scan_levels, base, yp, ep);
    chunk_rec<L, K, 1, -1>(greg, one, ak, phi, c, C, A.scan_levels, base, lam, el);
#pragma unroll
    for (int i = 0; i < L; ++i) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        db[k] = fmaf(lam[i], xv[i - k + K], db[k]);
        // a[k] is the coefficient of the output delayed by k + 1
        const int d = k + 1;
        const float yv = (i - d >= 0) ? yp[(i - d) >= 0 ? i - d : 0] : ep[(d - i - 1) >= 0 ? d - i - 1 : 0];
        da[k] = fmaf(-lam[i], yv, da[k]);
      }
    }
  }
  {
    float ym[L], em[K], mu[L], eu[K];
    chunk_rec<L, K, K, -1>(xreg, bk, ak, phi, c, C, A.scan_levels, base, ym, em);
    chunk_rec<L, K, 1, +1>(greg, one, ak, phi, c, C, A.scan_levels, base, mu, eu);
#pragma unroll
    for (int i = 0; i < L; ++i) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        db[k] = fmaf(mu[i], xv[i + k + K], db[k]);
        const int d = k + 1;
        const float yv = (i + d < L) ? ym[(i + d) < L ? i + d : 0] : em[(i + d - L) < K ? i + d - L : 0];
        da[k] = fmaf(-mu[i], yv, da[k]);
      }
    }
  }
  // block sums: lanes of a row, then rows (one row per C lanes), in double
  __syncthreads();
  double* red = reinterpret_cast<double*>(S);   // [R][2K] (the tile is no longer needed)
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double vb = db[k], va = da[k];
    for (int d = C >> 1; d > 0; d >>= 1) {
      vb += __shfl_down(vb, d, C);
      va += __shfl_down(va, d, C);
    }
    if (c == 0) {
      red[r * 2 * K + k] = vb;
      red[r * 2 * K + K + k] = va;
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * K) {
    double s = 0.0;
    for (int rr = 0; rr < R; ++rr) s += red[rr * 2 * K + threadIdx.x];
    partial[(size_t)blockIdx.x * 2 * K + threadIdx.x] = s;
  }
}

// out[g][0][k] (b) and out[g][1][k] (a), k < K0: the sum over the blocks of group g of
// partial[block][j] (j = k for b, K + k for a), in a fixed order.  Taps K0..K-1 of a padded
// kernel order are not reported.
__global__ void __launch_bounds__(256) coef_grad_reduce(const double* __restrict__ partial,
                                                        double* __restrict__ out, int blocks,
                                                        int tiles, int log2r, int n, int groups,
                                                        int K2, int K0) {
  __shared__ double sh[256];
  const int g = blockIdx.x / K2, j = blockIdx.x % K2;
  const int K = K2 / 2, which = j / K, k = j % K;
  if (k >= K0) return;
  double s = 0.0;
  for (int blk = threadIdx.x; blk < blocks; blk += blockDim.x) {
    const int tile = blk % tiles, q = (blk / tiles) & 3;
    const int t = tile << log2r;
    if (((q * n + t) * groups) / (4 * n) == g) s += partial[(size_t)blk * K2 + j];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(size_t)g * 2 * K0 + which * K0 + k] = sh[0];
}

template <int L, int K>
hipError_t launch_cg(const PassArgs& a, const float* g, double* partial, double* out, int batch,
                     int K0, hipStream_t stream) {
  const int N = 1 << a.log2n;
  const int R = 1 << a.log2r;
  const int tiles = N >> a.log2r;
  const int blocks = batch * 4 * tiles;
  const size_t lds = (size_t)2 * R * a.rs * sizeof(float);
  hipError_t e = hipFuncSetAttribute((const void*)coef_grad_kernel<L, K>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((coef_grad_kernel<L, K>), dim3(blocks), dim3(R << a.log2c), lds, stream, a,
                     g, partial);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(coef_grad_reduce, dim3(a.groups * 2 * K), dim3(256), 0, stream, partial, out,
                     blocks, tiles, a.log2r, N, a.groups, 2 * K, K0);
  return hipGetLastError();
}

template <int L>
hipError_t launch_cg_l(const PassArgs& a, const float* g, double* partial, double* out, int batch,
                       int K0, hipStream_t stream) {
  switch (a.order) {
    case 1: return launch_cg<L, 1>(a, g, partial, out, batch, K0, stream);
    case 2: return launch_cg<L, 2>(a, g, partial, out, batch, K0, stream);
    case 3: return launch_cg<L, 3>(a, g, partial, out, batch, K0, stream);
    case 4: return launch_cg<L, 4>(a, g, partial, out, batch, K0, stream);
    case 8: return launch_cg<L, 8>(a, g, partial, out, batch, K0, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_coef_grad(const PassArgs& a, const float* g, double* partial, double* out,
                            int batch, int K0, hipStream_t stream) {
  switch (a.log2l) {
    case 2: return launch_cg_l<4>(a, g, partial, out, batch, K0, stream);
    case 3: return launch_cg_l<8>(a, g, partial, out, batch, K0, stream);
    case 4: return launch_cg_l<16>(a, g, partial, out, batch, K0, stream);
    case 5: return launch_cg_l<32>(a, g, partial, out, batch, K0, stream);
    default: return hipErrorInvalidValue;   // N = 4096 (64-sample chunks) not supported here
  }
}

}  // namespace fhtfbp
