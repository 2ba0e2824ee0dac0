// Internal declarations shared by the HIP sources of libfhtfbp (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fhtfbp {

constexpr int kMaxOrder = 8;       // largest recursive-filter order supported
constexpr int kScalePad = 8;       // the row-factor table has 8 spare floats (whole-block scalar loads)
constexpr int kScanLevels = 7;     // chunk transition matrices Phi^(L 2^j), j < 7 (C <= 128)
constexpr int kMaxPasses = 12;
constexpr int kLdsBudget = 160 * 1024;

// Where a pass reads its tile rows from.
enum InMode : int {
  IN_ROWS = 0,    // rows of a [batch][4][N][N] buffer (linogram or inter-pass scratch)
  IN_IMAGE = 1,   // forward transform: the class frame of an image, columns mirrored
};

// Where a pass writes its tile rows to.
enum OutMode : int {
  OUT_ROWS = 0,         // next pass's rows of a [batch][4][N][N] buffer, offsets applied
  OUT_SAME = 1,         // back to the rows it read (filter alone)
  OUT_IMG_V = 2,        // last back-projection pass, classes 0 and 1 summed into image rows
  OUT_IMG_H = 3,        // last back-projection pass, classes 2 and 3 transposed, added in
  OUT_LINO_MIRROR = 4,  // last forward pass: rows with mirrored columns into the linogram
};

struct PassArgs {
  const float* in;
  float* out;
  int log2n;        // N = 2^log2n
  int levels;       // butterfly levels done in this pass (0: filter alone)
  int log2r;        // rows per tile = 2^log2r
  int k_hi;         // strip height at the start of the pass is 2^k_hi
  int log2c;        // chunks per row = 2^log2c (filter work items per row)
  int in_mode;
  int out_mode;
  int order;        // recursive filter order K, 0 = no filtering in this pass
  int groups;       // coefficient groups
  int coef_stride;  // floats per group in `coef`
  const float* coef;   // per group: b[K], a[K], Phi_j[K][K] for j < kScanLevels, h_k[L] for k < K,
                       // c[K] (c_k = -(b_{k+1} + .. + b_{K-1}) for k < K - 1, c[K - 1] = sum(b)
                       // or exactly 0 for a balanced numerator)
  const float* scale;  // [N] row factor c_t
  const int* sigma;    // [N] window start of row t
  int rs;              // LDS row stride in floats
  int log2l;           // chunk length L = 2^log2l (also the skew period of the LDS rows)
  int log2w;           // column-tiled passes: output columns per tile = 2^log2w
  int halo;            // column-tiled passes: extra columns loaded below the tile (>= 2^F - 1)
  int total_tiles;     // persistent passes: tiles over the whole batch
  int windowed;        // 1: rows start at the window start below, 0: at shift 0
  int rem;             // 1: the first-difference numerator has a remainder s x[i] (sum(b) != 0)
  int scan_levels;     // levels of the chunk-state scan the filter runs (<= kScanLevels): the
                       // contributions of chunks 2^scan_levels or more back, which the scan
                       // leaves out, are below 2^-30 of the chunk states in every group
};

// Fourth word of a raw buffer resource on gfx9-family devices (32-bit data, no swizzle).
constexpr int kBufferDword3 = 0x00020000;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Tables that stay constant for a whole launch (coefficients, row factors), read through the
// constant address space so that wave-uniform reads become scalar loads.
typedef const __attribute__((address_space(4))) float cfloat;
__device__ inline cfloat* as_constant(const float* p) { return (cfloat*)(uintptr_t)p; }

// Window start of row t (the same values as the `sigma` table): the window is centred on
// floor((N-1-t)/2), the intercept of the row's central line, and begins N/2 shifts below it.
__host__ __device__ inline int window_start_of(int t, int log2n, int windowed) {
  const int N = 1 << log2n;
  return windowed ? ((((N - 1 - t) >> 1) - (N >> 1)) & (N - 1)) : 0;
}

// Launch one pass over `batch` slices on `stream`.  Returns hipSuccess or the launch error.
// `a.order` is the kernel order: 0 (no filter), 1..4 or 8 (orders 5..7 zero-padded to 8).
hipError_t launch_pass(const PassArgs& a, int batch, hipStream_t stream);
template <int L>
hipError_t launch_pass_l(const PassArgs& a, int batch, hipStream_t stream);

// Kernel order used for a filter of order K.
inline int kernel_order(int K) { return K <= 4 ? K : kMaxOrder; }

// Whether a pass runs its levels in the streaming form (rows of >= 64 columns, whole waves).
__host__ __device__ inline bool pass_streams(const PassArgs& a) {
  const int threads = (1 << a.log2r) << a.log2c;
  return a.levels > 0 && a.log2n >= 6 && (threads & 63) == 0;
}

// LDS bytes of a pass: the tile of 2^log2r skewed rows, plus 64 floats per streaming unit.
__host__ __device__ inline size_t pass_lds_bytes(const PassArgs& a) {
  const size_t tile = (size_t)(1 << a.log2r) * a.rs * sizeof(float);
  if (!pass_streams(a)) return tile;
  const int threads = (1 << a.log2r) << a.log2c;
  const int waves = threads >> 6, pairs = 1 << (a.log2r - 1);
  return tile + (size_t)(waves > pairs ? waves : pairs) * 64 * sizeof(float);
}

// The persistent first pass with more than 64 chunks per row (a row over two waves) exchanges
// the chunk scan's end states between the row's waves through LDS: per row, 2 x 64 lanes x K
// floats after the pass's other LDS.
__host__ __device__ inline size_t first_xchg_floats(const PassArgs& a) {
  return a.log2c > 6 ? (size_t)(1 << a.log2r) * 128 * a.order : 0;
}

// Kernel families a pass can run on.
enum PassKind : int {
  PASS_ROWS = 0,        // full-row tiles, one per block (any mode)
  PASS_FIRST = 1,       // full-row tiles, persistent blocks with the next tile prefetched
  PASS_COLS = 2,        // column tiles with a halo (no filter): OUT_ROWS, OUT_IMG_V, OUT_IMG_H
  PASS_IMAGE = 3,       // last pass of 5 levels over square image tiles, all four classes
};
hipError_t launch_pass_kind(const PassArgs& a, int batch, int kind, int grid, hipStream_t stream);
template <int L>
hipError_t launch_first_l(const PassArgs& a, int grid, hipStream_t stream);
hipError_t launch_cols(const PassArgs& a, int batch, hipStream_t stream);
hipError_t launch_image_tiles(const PassArgs& a, int batch, hipStream_t stream);
bool first_pass_supported(const PassArgs& a);

// LDS bytes and threads of a column-tiled pass.
inline int cols_rs(const PassArgs& a) {
  const int wt = (1 << a.log2w) + a.halo;
  return (wt + (wt >> 5) + 1) | 1;
}
inline int cols_classes(const PassArgs& a) {
  return (a.out_mode == OUT_IMG_V || a.out_mode == OUT_IMG_H) ? 2 : 1;
}
inline size_t cols_lds_bytes(const PassArgs& a) {
  return (size_t)cols_classes(a) * (1 << a.log2r) * cols_rs(a) * sizeof(float);
}
inline int cols_threads(const PassArgs& a) { return cols_classes(a) == 2 ? 512 : 256; }

// Sinogram-to-linogram resampling: per linogram row (class q, slope t), the two sinogram
// angles it lies between (a1 = a0 + 1, or 0 when a0 + 1 = P with the detector mirrored: wrap),
// the weight of a1, and the detector position u = u0 + du * s of the line at shift s, and
// u = u1 + du * s of its fold at s - N (both bases computed in double).
struct ResampleRow {
  int a0, a1, wrap;
  float wa, u0, u1, du, pad;
};
hipError_t launch_resample(const float* sino, float* lino, const ResampleRow* tab, int batch,
                           int N, int P, int D, hipStream_t stream);

// Coefficient gradient of the recursive pair (writes out[groups][2][K0]).
hipError_t launch_coef_grad(const PassArgs& a, const float* g, double* partial, double* out,
                            int batch, int K0, hipStream_t stream);

// Learned residual correction (3x3 convolutions, BF16 matrix cores).
hipError_t launch_cnn_pack(const float* w, uint16_t* packed, int cin, int cout, int transpose_flip,
                           hipStream_t stream);
hipError_t launch_cnn_conv(int cin, int cout, const float* in32, const uint16_t* in16,
                           const uint16_t* wop, const float* bias, const uint16_t* mask,
                           const float* resid, uint16_t* out16, float* out32, int relu, int batch,
                           int H, int W, hipStream_t stream);
hipError_t launch_cnn_wgrad(int cin, int cout, const float* dz32, const uint16_t* dz16,
                            const float* in32, const uint16_t* in16, float* partial, float* out,
                            int batch, int H, int W, hipStream_t stream);
int cnn_wgrad_rows();
// floats of the weight gradient's partial buffer (block sums, then FP64 chunk sums)
int64_t cnn_wgrad_partial_floats(int cin, int cout, int batch, int H, int W);
hipError_t launch_cnn_fused(const float* in, const uint16_t* w1, const float* b1,
                            const uint16_t* w2, const float* b2, const uint16_t* w3,
                            const float* b3, float* out, int batch, int H, int W,
                            hipStream_t stream);

// Direct FBP comparator kernels.
hipError_t launch_direct_filter(const float* sino, float* work, int rows, int n_det,
                                float weight, const int* start, const float* wrow, int period,
                                hipStream_t stream);
hipError_t launch_direct_backproject(const float* work, float* img, int batch, int n,
                                     int n_rows, int n_det, const float* aff4,
                                     hipStream_t stream);

}  // namespace fhtfbp
