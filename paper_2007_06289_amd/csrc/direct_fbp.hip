// Direct FBP on a uniform parallel-beam sinogram (Sec. 2: eq 3-5 with the band-limited ramp of
// eq 7 applied as the full-length FIR of eq 8).  This is the Theta(N^3) reconstruction the
// method is measured against; it is tuned (LDS-staged rows and detector windows, several
// pixels per thread) but otherwise the textbook algorithm.
#include "fhtfbp_internal.h"

namespace fhtfbp {
namespace {

constexpr float kPi = 3.14159265358979323846f;

// One block per sinogram row: out[i] = w * (x[i]/4 - sum_{odd m} x[i - m] / (m pi)^2), every
// odd m with 0 <= i - m < n_det (the row is zero outside the detector).
__global__ void __launch_bounds__(256) direct_filter_kernel(const float* __restrict__ sino,
                                                            float* __restrict__ work,
                                                            int n_det, float weight) {
  extern __shared__ float sh[];
  float* x = sh;                 // [n_det]
  float* hodd = sh + n_det;      // hodd[k] = -1 / ((2k+1) pi)^2, k < n_det
  const size_t row = blockIdx.x;
  const float* src = sino + row * n_det;
  for (int i = threadIdx.x; i < n_det; i += blockDim.x) {
    x[i] = src[i];
    const float m = (float)(2 * i + 1) * kPi;
    hodd[i] = -1.0f / (m * m);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n_det; i += blockDim.x) {
    float acc = 0.25f * x[i];
    // left taps i - m >= 0 and right taps i + m < n_det, m = 2k + 1
    for (int k = 0; 2 * k + 1 <= i; ++k) acc = fmaf(hodd[k], x[i - 2 * k - 1], acc);
    for (int k = 0; i + 2 * k + 1 < n_det; ++k) acc = fmaf(hodd[k], x[i + 2 * k + 1], acc);
    work[row * n_det + i] = weight * acc;
  }
}

// Back projection: a block owns a 32 x 32 pixel tile (256 threads x 4 pixels, one column and
// four rows each).  Angles are taken in chunks of kA: for each angle the detector samples the
// tile can touch (a window of kW samples starting at ws) are staged in LDS with zeros outside
// the detector, then every pixel interpolates linearly between its two neighbours.
constexpr int kTile = 32;
constexpr int kA = 32;
constexpr int kW = 64;

__global__ void __launch_bounds__(256) direct_backproject_kernel(const float* __restrict__ work,
                                                                 float* __restrict__ img, int n,
                                                                 int n_angles, int n_det) {
  __shared__ float win[kA][kW + 1];
  __shared__ float cs[kA], sn[kA];
  __shared__ int ws[kA];
  const int tiles_x = n / kTile;
  const int tiles_per_slice = tiles_x * tiles_x;
  const int b = blockIdx.x / tiles_per_slice;
  const int tile = blockIdx.x % tiles_per_slice;
  const int x0 = (tile % tiles_x) * kTile, y0 = (tile / tiles_x) * kTile;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 columns x 8 row groups
  const float half = 0.5f * n;
  const float X = x0 + tx + 0.5f - half;
  float Y[4];
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int p = 0; p < 4; ++p) Y[p] = y0 + ty + 8 * p + 0.5f - half;
  const float off = 0.5f * n_det - 0.5f;
  // tile centre and its half diagonal, for the window start
  const float cx = x0 + 0.5f * kTile - half, cy = y0 + 0.5f * kTile - half;
  const float* wb = work + (size_t)b * n_angles * n_det;
  for (int a0 = 0; a0 < n_angles; a0 += kA) {
    __syncthreads();
    if (threadIdx.x < kA) {
      const int a = a0 + threadIdx.x;
      float s = 0.f, c = 1.f;
      if (a < n_angles) sincospif((float)a / (float)n_angles, &s, &c);
      cs[threadIdx.x] = c;
      sn[threadIdx.x] = s;
      const float rc = cx * c + cy * s + off;
      ws[threadIdx.x] = (int)floorf(rc) - kW / 2;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kA * kW; e += blockDim.x) {
      const int ai = e / kW, k = e % kW;
      const int a = a0 + ai;
      const int d = ws[ai] + k;
      win[ai][k] = (a < n_angles && d >= 0 && d < n_det) ? wb[(size_t)a * n_det + d] : 0.f;
    }
    __syncthreads();
    const int na = min(kA, n_angles - a0);
    for (int ai = 0; ai < na; ++ai) {
      const float c = cs[ai], s = sn[ai];
      const float base = X * c + off - (float)ws[ai];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const float pos = fmaf(Y[p], s, base);
        const float fl = floorf(pos);
        const int i0 = (int)fl;
        const float fr = pos - fl;
        const float v0 = win[ai][i0], v1 = win[ai][i0 + 1];
        acc[p] += fmaf(fr, v1 - v0, v0);
      }
    }
  }
  float* dst = img + (size_t)b * n * n;
#pragma unroll
  for (int p = 0; p < 4; ++p) dst[(size_t)(y0 + ty + 8 * p) * n + x0 + tx] = acc[p];
}

}  // namespace

hipError_t launch_direct_filter(const float* sino, float* work, int rows, int n_det,
                                float weight, hipStream_t stream) {
  const size_t lds = (size_t)2 * n_det * sizeof(float);
  hipError_t e = hipFuncSetAttribute((const void*)direct_filter_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(direct_filter_kernel, dim3(rows), dim3(256), lds, stream, sino, work, n_det,
                     weight);
  return hipGetLastError();
}

hipError_t launch_direct_backproject(const float* work, float* img, int batch, int n,
                                     int n_angles, int n_det, hipStream_t stream) {
  const int tiles = (n / kTile) * (n / kTile);
  hipLaunchKernelGGL(direct_backproject_kernel, dim3(batch * tiles), dim3(256), 0, stream, work,
                     img, n, n_angles, n_det);
  return hipGetLastError();
}

}  // namespace fhtfbp
