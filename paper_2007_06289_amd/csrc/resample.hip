// Scanner input: a parallel-beam sinogram resampled onto the four linogram line classes
// (Sec. 4.2, eq 14).  Each linogram line is looked up by its normal angle in [0, pi) and its
// signed distance from the image centre, linearly in both (bilinear), zero off the detector;
// the cell's two folds (shift s and s - N) are summed.  The geometry of a row (class q, slope
// index t) is one angle and a detector position affine in s, tabulated on the host in double.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fhtfbp_internal.h"

namespace fhtfbp {
namespace {

// Linear interpolation of one sinogram row at fractional detector position u, zero outside
// [0, D - 1] (each neighbour is read only if it is on the detector).
__device__ __forceinline__ float lerp_row(const float* __restrict__ row, float u, int D) {
  const float fl = floorf(u);
  const float f = u - fl;
  const int j = (int)fl;
  const float v0 = (j >= 0 && j < D) ? row[j] : 0.f;
  const float v1 = (j + 1 >= 0 && j + 1 < D) ? row[j + 1] : 0.f;
  return fmaf(f, v1 - v0, v0);
}

// One block per (slice, class, slope row); each thread writes four consecutive shifts.
__global__ void __launch_bounds__(256) resample_kernel(const float* __restrict__ sino,
                                                       float* __restrict__ lino,
                                                       const ResampleRow* __restrict__ tab,
                                                       int N, int P, int D) {
  const int row = blockIdx.x % (4 * N);
  const int b = blockIdx.x / (4 * N);
  const ResampleRow g = tab[row];
  const float* s0 = sino + ((size_t)b * P + g.a0) * D;
  const float* s1 = sino + ((size_t)b * P + g.a1) * D;
  float* out = lino + ((size_t)b * 4 * N + row) * N;
  for (int s4 = threadIdx.x * 4; s4 < N; s4 += blockDim.x * 4) {
    float v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      float acc = 0.f;
#pragma unroll
      for (int fold = 0; fold < 2; ++fold) {
        const float u = fmaf(g.du, (float)(s4 + e), fold ? g.u1 : g.u0);
        const float u1 = g.wrap ? (float)(D - 1) - u : u;   // angle pi = angle 0, mirrored
        acc += (1.f - g.wa) * lerp_row(s0, u, D) + g.wa * lerp_row(s1, u1, D);
      }
      v[e] = acc;
    }
    *reinterpret_cast<float4*>(out + s4) = make_float4(v[0], v[1], v[2], v[3]);
  }
}

}  // namespace

hipError_t launch_resample(const float* sino, float* lino, const ResampleRow* tab, int batch,
                           int N, int P, int D, hipStream_t stream) {
  const int threads = std::min(256, std::max(64, N / 4));
  hipLaunchKernelGGL(resample_kernel, dim3(batch * 4 * N), dim3(threads), 0, stream, sino, lino,
                     tab, N, P, D);
  return hipGetLastError();
}

}  // namespace fhtfbp
