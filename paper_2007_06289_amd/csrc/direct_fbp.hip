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
// Optional per-row tables (rows repeat every `period` rows): start[r] rotates the row (the row is
// read from sample start[r] on, cyclically), wrow[r] replaces the uniform weight.
__global__ void __launch_bounds__(256) direct_filter_kernel(const float* __restrict__ sino,
                                                            float* __restrict__ work,
                                                            int n_det, float weight,
                                                            const int* __restrict__ start,
                                                            const float* __restrict__ wrow,
                                                            int period) {
  extern __shared__ float sh[];
  float* x = sh;                 // [n_det]
  float* hodd = sh + n_det;      // hodd[k] = -1 / ((2k+1) pi)^2, k < n_det
  const size_t row = blockIdx.x;
  const float* src = sino + row * n_det;
  const int pr = (int)(row % (size_t)period);
  const int st = start ? start[pr] : 0;
  if (wrow) weight = wrow[pr];
  for (int i = threadIdx.x; i < n_det; i += blockDim.x) {
    int j = i + st;
    if (j >= n_det) j -= n_det;
    x[i] = src[j];
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
// four rows each).  Row a of a slice maps the pixel centre (X, Y), measured from the image
// centre, to the detector position pos = X aff[a].x + Y aff[a].y + aff[a].z (|x| + |y| <= 2).
// Rows are taken in chunks of kA: for each row the detector samples the tile can touch (a
// window of kW samples starting at ws) are staged in LDS with zeros outside the detector, then
// every pixel interpolates linearly between its two neighbours.
constexpr int kTile = 32;
constexpr int kA = 32;
constexpr int kW = 80;

__global__ void __launch_bounds__(256) direct_backproject_kernel(const float* __restrict__ work,
                                                                 float* __restrict__ img, int n,
                                                                 int n_rows, int n_det,
                                                                 const float4* __restrict__ aff) {
  __shared__ float win[kA][kW + 1];
  __shared__ float ca[kA], cb[kA], cc[kA];
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
  const float cx = x0 + 0.5f * kTile - half, cy = y0 + 0.5f * kTile - half;
  const float* wb = work + (size_t)b * n_rows * n_det;
  for (int a0 = 0; a0 < n_rows; a0 += kA) {
    __syncthreads();
    if (threadIdx.x < kA) {
      const int a = a0 + threadIdx.x;
      const float4 f = (a < n_rows) ? aff[a] : make_float4(0.f, 0.f, 0.f, 0.f);
      ca[threadIdx.x] = f.x;
      cb[threadIdx.x] = f.y;
      cc[threadIdx.x] = f.z;
      const float rc = cx * f.x + cy * f.y + f.z;
      ws[threadIdx.x] = (int)floorf(rc) - kW / 2;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kA * kW; e += blockDim.x) {
      const int ai = e / kW, k = e % kW;
      const int a = a0 + ai;
      const int d = ws[ai] + k;
      win[ai][k] = (a < n_rows && d >= 0 && d < n_det) ? wb[(size_t)a * n_det + d] : 0.f;
    }
    __syncthreads();
    const int na = min(kA, n_rows - a0);
    for (int ai = 0; ai < na; ++ai) {
      const float base = X * ca[ai] + cc[ai] - (float)ws[ai];
      const float s = cb[ai];
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
                                float weight, const int* start, const float* wrow, int period,
                                hipStream_t stream) {
  const size_t lds = (size_t)2 * n_det * sizeof(float);
  hipError_t e = hipFuncSetAttribute((const void*)direct_filter_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(direct_filter_kernel, dim3(rows), dim3(256), lds, stream, sino, work, n_det,
                     weight, start, wrow, period > 0 ? period : 1);
  return hipGetLastError();
}

hipError_t launch_direct_backproject(const float* work, float* img, int batch, int n,
                                     int n_rows, int n_det, const float* aff4,
                                     hipStream_t stream) {
  const int tiles = (n / kTile) * (n / kTile);
  hipLaunchKernelGGL(direct_backproject_kernel, dim3(batch * tiles), dim3(256), 0, stream, work,
                     img, n, n_rows, n_det, reinterpret_cast<const float4*>(aff4));
  return hipGetLastError();
}

}  // namespace fhtfbp
