// Host side of libfhtfbp: plans, argument checks, pass scheduling and the C ABI entry points.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/fhtfbp.h"
#include "fhtfbp_internal.h"

using namespace fhtfbp;

struct fbp_plan_s {
  int n = 0, log2n = 0, max_batch = 0, order = 0, groups = 1;
  uint32_t flags = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  int cus = 0;                // compute units of the device
  int log2l = 0, log2c = 0;   // chunk length and chunks per row of the filter
  int rs = 0;                 // LDS row stride
  std::vector<int> levels;    // levels per back-projection pass, first pass first
  std::vector<int> fwd_levels;   // levels per forward-transform pass (full-row tiles)
  int log2w = 8;              // column-tiled passes: output columns per tile = 2^log2w
  int fmax = 0;               // most levels a first pass (full rows in LDS) can fuse
  unsigned generation = 0;    // bumped when the schedule or the numerator form changes
                              // (captured graphs go stale)
  std::vector<double> b, a;   // host copies [groups][order]
  // the filters take the numerator in first-difference form (orders >= 2), which keeps a zero
  // response at zero frequency exact in float32; `rem`: some group's sum(b) is not zero, so
  // the kernels add the remainder term
  bool rem = false;
  // levels of the filter's chunk-state scan for the plan's chunks and for 32-sample chunks
  // (scan_depth); a change makes captured graphs stale
  int scan_levels = kScanLevels, scan_levels32 = kScanLevels;
  int coef_stride = 0;
  float* d_coef = nullptr;
  // N = 4096: the filter's own chunks are 64 samples (C = 64), while the persistent first pass
  // runs 32-sample chunks over two waves per row (C = 128), with a table of its own
  float* d_coef32 = nullptr;
  int coef_stride32 = 0;
  float* d_scale = nullptr;
  int* d_sigma = nullptr;
  float* d_scratch[2] = {nullptr, nullptr};
  size_t scratch_floats = 0;
  double* d_partial = nullptr;   // per-block sums of the coefficient gradient
  size_t partial_doubles = 0;
  // kernel timing: event pairs recorded around launches while profiling is on
  bool profiling = false;
  struct Rec {
    hipEvent_t start, stop;
    int kind;
  };
  std::vector<Rec> recs;
};

// A captured reconstruction of one or more sub-batches (see fbp_graph_create).
struct fbp_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<std::pair<fbp_plan_s*, unsigned>> plans;   // distinct plans, schedule generation
};

// ---- fixed scratch of fbp_reconstruct_noalloc ----------------------------------------------
// The inter-pass intermediate of the no-allocation entry point lives in this array, one copy
// per device, held from the code object's load until the process ends.  Host code never uses
// the array's name as an address: fbp_plan resolves each device's copy once, with that device
// current, and the entry point passes that address to the kernels.
constexpr size_t kNoAllocScratchFloats = FBP_NOALLOC_SCRATCH_BYTES / sizeof(float);
static __device__ __align__(256) float scratch[kNoAllocScratchFloats];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
float* g_noalloc_ptr[kMaxDevices] = {};

void resolve_noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (g_noalloc_ptr[device]) return;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess && ptr)
    g_noalloc_ptr[device] = static_cast<float*>(ptr);
}

float* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  return g_noalloc_ptr[device];
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}
bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Schur-Cohn step-down test: every root of 1 + a_1 z^-1 + ... + a_K z^-K inside |z| < 1.
bool stable(const double* a, int K) {
  std::vector<double> c(K + 1);
  c[0] = 1.0;
  for (int k = 0; k < K; ++k) {
    if (!isfinite(a[k])) return false;
    c[k + 1] = a[k];
  }
  for (int m = K; m >= 1; --m) {
    const double km = c[m];
    if (!(fabs(km) < 1.0)) return false;
    std::vector<double> d(m);
    const double den = 1.0 - km * km;
    for (int i = 0; i < m; ++i) d[i] = (c[i] - km * c[m - i]) / den;
    for (int i = 0; i < m; ++i) c[i] = d[i];
  }
  return true;
}

// Phi_j = C^(L 2^j) for the companion matrix C of the recursion (state (y[i-1], ..., y[i-K])).
void transition_powers(const double* a, int K, int L, double* out /* [kScanLevels][K][K] */) {
  std::vector<double> C(K * K, 0.0), P(K * K, 0.0), tmp(K * K);
  for (int m = 0; m < K; ++m) C[m] = -a[m];
  for (int i = 1; i < K; ++i) C[i * K + i - 1] = 1.0;
  auto mul = [&](const std::vector<double>& X, const std::vector<double>& Y,
                 std::vector<double>& Z) {
    for (int i = 0; i < K; ++i)
      for (int j = 0; j < K; ++j) {
        double s = 0;
        for (int m = 0; m < K; ++m) s += X[i * K + m] * Y[m * K + j];
        Z[i * K + j] = s;
      }
  };
  for (int i = 0; i < K; ++i) P[i * K + i] = 1.0;   // P = C^L
  for (int s = 0; s < L; ++s) {
    mul(P, C, tmp);
    P.swap(tmp);
  }
  for (int j = 0; j < kScanLevels; ++j) {
    for (int i = 0; i < K * K; ++i) out[j * K * K + i] = P[i];
    mul(P, P, tmp);
    P.swap(tmp);
  }
}

// Homogeneous response of the recursion over one chunk of L samples: h_k[s] is the output at
// step s of y[s] = -sum_m a_m y[s-1-m] started from y[-1-k] = 1 (the other initial values 0).
// A chunk's carry correction is then sum_k h_k[s] y_in[-1-k], K multiply-adds per sample.
void homogeneous_table(const double* a, int K, int L, double* out /* [K][L] */) {
  for (int k = 0; k < K; ++k) {
    std::vector<double> z(L + K, 0.0);   // z[K + s] = y[s], z[K - 1 - m] = y[-1-m]
    z[K - 1 - k] = 1.0;
    for (int s = 0; s < L; ++s) {
      double acc = 0.0;
      for (int m = 0; m < K; ++m) acc -= a[m] * z[K + s - 1 - m];
      z[K + s] = acc;
    }
    for (int s = 0; s < L; ++s) out[k * L + s] = z[K + s];
  }
}

// Levels per pass: as few passes as LDS allows, balanced, extra levels to the later passes.
std::vector<int> split_levels(int n, int fmax) {
  const int P = (n + fmax - 1) / fmax;
  std::vector<int> v(P, n / P);
  for (int i = 0; i < n % P; ++i) v[P - 1 - i] += 1;
  return v;
}

// Default back-projection schedule.  Below 256 every pass holds full rows (split_levels).  From
// 256 on the passes after the first are column-tiled, which lets them fuse kColsLevels levels
// whatever the row length (two radix-4 stages after the loader's level 0), so: as few passes as
// possible, kColsLevels levels in every column-tiled pass and the rest in the first; if that
// leaves the first pass fewer than two levels, the middle passes give theirs up first.
// Measured fastest on MI355X among all groupings (N = 256 .. 4096).
constexpr int kColsLevels = 5;
std::vector<int> backprojection_levels(int n, int fmax) {
  if (n < 8 || n <= fmax) return split_levels(n, fmax);
  int P = 2;
  while (fmax + kColsLevels * (P - 1) < n) ++P;
  std::vector<int> v(P, kColsLevels);
  v[0] = n - kColsLevels * (P - 1);
  for (int i = 1; v[0] < 2 && i < P; ++i) {   // first pass: at least two levels
    while (v[0] < 2 && v[i] > 2) {
      v[i] -= 1;
      v[0] += 1;
    }
  }
  return v;
}

// A numerator whose taps sum to zero within their rounding in double: its remainder s is
// taken as exactly zero.
bool balanced_numerator(double sum, double mag) { return fabs(sum) <= 1e-12 * mag; }

// Whether some group's numerator has a remainder (orders >= 2).
bool numerator_remainder(const fbp_plan_s* p) {
  if (p->order < 2) return false;
  for (int g = 0; g < p->groups; ++g) {
    double sum = 0.0, mag = 0.0;
    for (int k = 0; k < p->order; ++k) {
      sum += p->b[(size_t)g * p->order + k];
      mag += fabs(p->b[(size_t)g * p->order + k]);
    }
    if (!balanced_numerator(sum, mag)) return true;
  }
  return false;
}

// Levels of the chunk-state scan one group needs.  After j levels a chunk's end state holds
// the local end states of the 2^j chunks up to it, each carried through Phi^(L m); the chunks
// 2^j and more back are left out.  With n_j = ||Phi^(L 2^j)|| (infinity norm) and n_0 < 1,
// what is left out is at most n_j / (1 - n_0) times the largest local end state
// (||Phi^(L (2^j + i))|| <= n_j n_0^i): the depth is the first j where that is below 2^-30,
// far under the float32 rounding of the states.  Without n_0 < 1, every level.
int scan_depth(const double* phi /* [kScanLevels][K][K] */, int K) {
  double n[kScanLevels];
  for (int j = 0; j < kScanLevels; ++j) {
    double m = 0.0;
    for (int r = 0; r < K; ++r) {
      double row = 0.0;
      for (int c = 0; c < K; ++c) row += fabs(phi[(j * K + r) * K + c]);
      m = row > m ? row : m;
    }
    n[j] = m;
  }
  if (!(n[0] < 1.0)) return kScanLevels;
  for (int j = 0; j < kScanLevels; ++j)
    if (n[j] / (1.0 - n[0]) <= 0x1p-30) return j;
  return kScanLevels;
}

// One coefficient table for chunks of L samples: per group b[K], a[K], Phi^(L 2^j) for
// j < kScanLevels, the homogeneous responses h_k[0 .. L-1], and the first-difference
// numerator's taps c[0 .. K-2] and remainder s.  *depth: the scan levels the groups need.
int fill_coefficients(const fbp_plan_s* p, int L, int stride, std::vector<float>& host,
                      int* depth) {
  const int K0 = p->order, G = p->groups;
  const int K = kernel_order(K0);   // taps K0..K-1 are zero
  host.assign((size_t)G * stride, 0.f);
  std::vector<double> phi(kScanLevels * K * K), hom((size_t)K * L);
  *depth = K > 0 ? 0 : kScanLevels;
  for (int g = 0; g < G; ++g) {
    std::vector<double> bg(K, 0.0), ag(K, 0.0);
    for (int k = 0; k < K0; ++k) {
      bg[k] = p->b[(size_t)g * K0 + k];
      ag[k] = p->a[(size_t)g * K0 + k];
    }
    if (!stable(ag.data(), K0)) return FBP_EUNSTABLE;
    for (int k = 0; k < K; ++k) {
      if (!isfinite(bg[k])) return FBP_EUNSTABLE;
      host[(size_t)g * stride + k] = (float)bg[k];
      host[(size_t)g * stride + K + k] = (float)ag[k];
    }
    transition_powers(ag.data(), K, L, phi.data());
    for (int i = 0; i < kScanLevels * K * K; ++i)
      host[(size_t)g * stride + 2 * K + i] = (float)phi[i];
    if (K > 0) {
      const int d = scan_depth(phi.data(), K);
      *depth = d > *depth ? d : *depth;
    }
    homogeneous_table(ag.data(), K, L, hom.data());
    for (int i = 0; i < K * L; ++i)
      host[(size_t)g * stride + 2 * K + kScanLevels * K * K + i] = (float)hom[i];
    // first-difference form B(z) = (1 - z^-1) C(z) + s: c_k = -(b_{k+1} + .. + b_{K-1}) for
    // k < K - 1, s = sum(b) in the last slot, exactly zero for a balanced numerator (|sum(b)|
    // within rounding of its taps in double); each summed in double and rounded once
    double sum = 0.0, mag = 0.0;
    for (int k = 0; k < K; ++k) {
      sum += bg[k];
      mag += fabs(bg[k]);
    }
    const bool balanced = balanced_numerator(sum, mag);
    double tail = 0.0;
    for (int k = K - 2; k >= 0; --k) {
      tail += bg[k + 1];
      host[(size_t)g * stride + stride - K + k] = (float)(-tail);
    }
    host[(size_t)g * stride + stride - 1] = balanced ? 0.f : (float)sum;
  }
  return FBP_OK;
}

int upload_coefficients(fbp_plan_s* p) {
  std::vector<float> host, host32;
  // the remainder term is compiled into the kernels a graph captured: a change makes such
  // graphs stale, as a schedule change does
  const bool rem = numerator_remainder(p);
  int depth = kScanLevels, depth32 = kScanLevels;
  int rc = fill_coefficients(p, 1 << p->log2l, p->coef_stride, host, &depth);
  if (rc == FBP_OK && p->d_coef32)
    rc = fill_coefficients(p, 32, p->coef_stride32, host32, &depth32);
  if (rc != FBP_OK) return rc;
  // so is the scan depth (a kernel argument)
  if (rem != p->rem || depth != p->scan_levels || depth32 != p->scan_levels32)
    p->generation += 1;
  p->rem = rem;
  p->scan_levels = depth;
  p->scan_levels32 = depth32;
  if (hipStreamSynchronize(p->stream) != hipSuccess) return FBP_EDEVICE;
  if (hipMemcpy(p->d_coef, host.data(), host.size() * sizeof(float), hipMemcpyHostToDevice) !=
      hipSuccess)
    return FBP_EDEVICE;
  if (p->d_coef32 && hipMemcpy(p->d_coef32, host32.data(), host32.size() * sizeof(float),
                               hipMemcpyHostToDevice) != hipSuccess)
    return FBP_EDEVICE;
  return FBP_OK;
}

void clear_recs(fbp_plan_s* p) {
  for (auto& r : p->recs) {
    hipEventDestroy(r.start);
    hipEventDestroy(r.stop);
  }
  p->recs.clear();
}

// Where and how a call's kernels are issued: the stream, and whether the plan's profiling
// events may be recorded (never inside a graph capture).
struct Issue {
  hipStream_t stream;
  bool timing;
};
Issue plan_issue(const fbp_plan_s* p) { return Issue{p->stream, p->profiling}; }

hipError_t dispatch(fbp_plan_s* p, const PassArgs& A, int batch, int family, hipStream_t s) {
  if (family == PASS_COLS) return launch_cols(A, batch, s);
  if (family == PASS_IMAGE) return launch_image_tiles(A, batch, s);
  if (family == PASS_FIRST) return launch_pass_kind(A, batch, PASS_FIRST, p->cus, s);
  return launch_pass(A, batch, s);
}

// Launch one pass, bracketed by timing events when the plan is profiling.
hipError_t timed_pass(fbp_plan_s* p, const PassArgs& A, int batch, int kind, const Issue& is,
                      int family = PASS_ROWS) {
  if (!is.timing) return dispatch(p, A, batch, family, is.stream);
  fbp_plan_s::Rec r;
  r.kind = kind;
  if (hipEventCreate(&r.start) != hipSuccess) return hipErrorOutOfMemory;
  if (hipEventCreate(&r.stop) != hipSuccess) {
    hipEventDestroy(r.start);
    return hipErrorOutOfMemory;
  }
  hipEventRecord(r.start, is.stream);
  hipError_t e = dispatch(p, A, batch, family, is.stream);
  hipEventRecord(r.stop, is.stream);
  p->recs.push_back(r);
  return e;
}

void free_plan(fbp_plan_s* p) {
  if (!p) return;
  clear_recs(p);
  hipFree(p->d_partial);
  hipFree(p->d_coef);
  hipFree(p->d_coef32);
  hipFree(p->d_scale);
  hipFree(p->d_sigma);
  hipFree(p->d_scratch[0]);
  hipFree(p->d_scratch[1]);
  delete p;
}

int check_batch(const fbp_plan_s* p, int32_t batch) {
  if (!p) return FBP_EINVAL;
  if (batch < 0) return FBP_EINVAL;
  if (batch > p->max_batch) return FBP_ERANGE;
  return FBP_OK;
}

// Scratch buffers a schedule of P passes ping-pongs through.
int scratch_needed(size_t passes) { return passes >= 3 ? 2 : (passes == 2 ? 1 : 0); }

// Can the kernels run this back-projection schedule?  Pass 0 holds 2^F full rows (and runs the
// filter); for N >= 256 the later passes are column-tiled (2^F rows of 2^log2w + halo columns,
// two classes for the last pass), below that they hold full rows too.
int check_schedule(const fbp_plan_s* p, const std::vector<int>& lv, int log2w) {
  if (lv.empty() || lv.size() > 16) return FBP_EINVAL;
  int sum = 0;
  for (int F : lv) {
    if (F < 1) return FBP_EINVAL;
    sum += F;
  }
  if (sum != p->log2n) return FBP_EINVAL;
  if (lv[0] > p->fmax) return FBP_ERANGE;
  const bool cols = p->log2n >= 8;
  if (cols && (log2w < 6 || log2w > std::min(10, p->log2n))) return FBP_ERANGE;
  for (size_t i = 1; i < lv.size(); ++i) {
    const int F = lv[i];
    if (!cols) {
      if (F > p->fmax) return FBP_ERANGE;
      continue;
    }
    PassArgs t;
    memset(&t, 0, sizeof(t));
    t.log2n = p->log2n;
    t.log2r = F;
    t.log2w = log2w;
    t.halo = std::max(4, 1 << F);
    t.out_mode = (i + 1 == lv.size()) ? OUT_IMG_V : OUT_ROWS;
    // a last pass of 5 or 7 levels runs over square image tiles, whatever the width
    if (i + 1 == lv.size() && (F == 5 || F == 7)) continue;
    if (cols_lds_bytes(t) > (size_t)kLdsBudget) return FBP_ERANGE;
  }
  return FBP_OK;
}

// Arguments of a many-plan call, checked before anything is launched.
int check_many(const fbp_plan_t* plans, const float* const* lino, float* const* img,
               const int32_t* batch, int32_t count) {
  if (count < 0) return FBP_EINVAL;
  if (count == 0) return FBP_OK;
  if (!plans || !lino || !img || !batch) return FBP_EINVAL;
  for (int i = 0; i < count; ++i) {
    const fbp_plan_s* p = plans[i];
    if (!p || batch[i] < 0) return FBP_EINVAL;
    if (batch[i] > p->max_batch) return FBP_ERANGE;
    if (batch[i] > 0 && (!lino[i] || !img[i] || !aligned16(lino[i]) || !aligned16(img[i])))
      return FBP_EINVAL;
    if (p->device != plans[0]->device) return FBP_EINVAL;
  }
  return FBP_OK;
}

PassArgs base_args(const fbp_plan_s* p) {
  PassArgs A;
  memset(&A, 0, sizeof(A));
  A.log2n = p->log2n;
  A.log2c = p->log2c;
  A.log2l = p->log2l;
  A.rs = p->rs;
  A.groups = p->groups;
  A.coef_stride = p->coef_stride;
  A.coef = p->d_coef;
  A.scale = p->d_scale;
  A.sigma = p->d_sigma;
  A.windowed = (p->flags & FBP_ZERO_WINDOW) ? 0 : 1;
  A.rem = p->rem ? 1 : 0;
  A.scan_levels = p->scan_levels;
  return A;
}

// Whether pass 0 of a back projection can run on the persistent first-pass kernel, which needs
// 32-sample chunks.  At N = 4096 the plan's filter chunks are 64 samples; pass 0 then switches
// to 32-sample chunks over two waves per row (its own coefficient table and LDS row stride).
// A keeps the plan's values when the answer is no.
bool first_pass_args(const fbp_plan_s* p, PassArgs& A) {
  PassArgs F = A;
  if (p->log2l != 5) {
    if (!p->d_coef32) return false;
    F.log2l = 5;
    F.log2c = p->log2n - 5;
    F.rs = p->n + (p->n >> 5);
    F.coef = p->d_coef32;
    F.coef_stride = p->coef_stride32;
    F.scan_levels = p->scan_levels32;
  }
  const size_t lds = pass_lds_bytes(F) + first_xchg_floats(F) * sizeof(float);
  if (!pass_streams(F) || !first_pass_supported(F) || lds > (size_t)kLdsBudget) return false;
  A = F;
  return true;
}

// Run the transposed FHT passes.  forward: image -> linogram through the mirrored transform;
// otherwise linogram -> image (with the filter fused into the first pass when `filter`).
// The intermediate of `batch` slices ping-pongs through scratch[0] and scratch[1] (NULL for
// the plan's own buffers); a buffer the schedule needs and does not have gives FBP_EINVAL
// before anything is launched.
int run_passes(fbp_plan_s* p, const float* in, float* out, int batch, bool forward,
               bool filter, const Issue& is, float* const* scratch = nullptr) {
  if (batch == 0) return FBP_OK;
  const std::vector<int>& levels = forward ? p->fwd_levels : p->levels;
  const int P = (int)levels.size();
  float* const* bufs = scratch ? scratch : p->d_scratch;
  for (int i = 0; i < scratch_needed(levels.size()); ++i)
    if (!bufs[i]) return FBP_EINVAL;
  int k = p->log2n;
  const float* src = in;
  for (int pi = 0; pi < P; ++pi) {
    const int F = levels[pi];
    const bool first = pi == 0, last = pi == P - 1;
    PassArgs A = base_args(p);
    A.levels = F;
    A.log2r = F;
    A.k_hi = k;
    A.in = src;
    A.in_mode = (first && forward) ? IN_IMAGE : IN_ROWS;
    A.order = (first && filter) ? kernel_order(p->order) : 0;
    hipError_t e;
    const int kind = forward ? FBP_KERNEL_FORWARD : (first ? FBP_KERNEL_FIRST : FBP_KERNEL_MIDDLE);
    // column tiles for the middle and last back-projection passes (they carry no filter)
    const bool cols = !forward && !first && p->log2n >= 8;
    if (cols) {
      A.log2w = std::min(p->log2w, p->log2n);
      A.halo = std::max(4, 1 << F);
    }
    if (!last) {
      float* dst = bufs[pi & 1];
      A.out = dst;
      A.out_mode = OUT_ROWS;
      if (cols) {
        e = timed_pass(p, A, batch, kind, is, PASS_COLS);
      } else if (first && !forward && first_pass_args(p, A)) {
        A.total_tiles = batch * 4 * (p->n >> F);
        e = timed_pass(p, A, batch, kind, is, PASS_FIRST);
      } else {
        e = timed_pass(p, A, batch, kind, is, PASS_ROWS);
      }
      src = dst;
    } else if (forward) {
      A.out = out;
      A.out_mode = OUT_LINO_MIRROR;
      e = timed_pass(p, A, batch, kind, is, PASS_ROWS);
    } else {
      A.out = out;
      A.out_mode = OUT_IMG_V;
      if (cols && (F == 5 || F == 7)) {
        // all four classes over square image tiles: the image is written once
        e = timed_pass(p, A, batch, FBP_KERNEL_LAST, is, PASS_IMAGE);
      } else {
        e = timed_pass(p, A, batch, FBP_KERNEL_LAST_V, is, cols ? PASS_COLS : PASS_ROWS);
        if (e == hipSuccess) {
          A.out_mode = OUT_IMG_H;
          e = timed_pass(p, A, batch, FBP_KERNEL_LAST_H, is, cols ? PASS_COLS : PASS_ROWS);
        }
      }
    }
    if (e != hipSuccess) return FBP_EDEVICE;
    k -= F;
  }
  return FBP_OK;
}

}  // namespace

namespace fhtfbp {
// The persistent first pass is instantiated for 4, 8 or 16 column blocks per streaming unit.
bool first_pass_supported(const PassArgs& a) {
  const int threads = (1 << a.log2r) << a.log2c;
  const int waves = threads >> 6, pairs = 1 << (a.log2r - 1);
  const int segs = waves > pairs ? waves / pairs : 1;
  const int nblk = ((1 << a.log2n) / segs) >> 6;
  // the filter reads a wave's coefficients once for all its rows: the rows of a wave
  // (64 / C of them) must lie in one angle group (4N / groups consecutive rows)
  const int rows_per_wave = std::max(1, 64 >> a.log2c);   // C = 128: half a row per wave
  const int rows_per_group = (4 << a.log2n) / std::max(1, a.groups);
  if (a.order > 0 && (rows_per_group < 1 || rows_per_group % rows_per_wave != 0)) return false;
  // rows over two waves: orders up to 4 (the exchange area, 128 K floats per row, must fit)
  if (a.log2c > 6 && (a.log2c > 7 || a.order > 4 || threads > 1024 || nblk != 16)) return false;
  return nblk == 4 || nblk == 8 || nblk == 16;
}

// Persistent passes: one block per compute unit times the blocks a unit holds at once.
hipError_t launch_pass_kind(const PassArgs& a, int batch, int kind, int cus, hipStream_t stream) {
  (void)batch;
  (void)kind;
  if (a.log2l != 5) return hipErrorInvalidValue;
  const int threads = (1 << a.log2r) << a.log2c;
  const size_t lds = pass_lds_bytes(a) + first_xchg_floats(a) * sizeof(float);
  int per_cu = (int)(kLdsBudget / std::max<size_t>(lds, 1));
  per_cu = std::max(1, std::min(per_cu, 2048 / threads));
  const int grid = std::min(a.total_tiles, cus * per_cu);
  return launch_first_l<32>(a, grid, stream);
}

hipError_t launch_pass(const PassArgs& a, int batch, hipStream_t stream) {
  switch (a.log2l) {
    case 2: return launch_pass_l<4>(a, batch, stream);
    case 3: return launch_pass_l<8>(a, batch, stream);
    case 4: return launch_pass_l<16>(a, batch, stream);
    case 5: return launch_pass_l<32>(a, batch, stream);
    case 6: return launch_pass_l<64>(a, batch, stream);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace fhtfbp

namespace {

// Per-row tables of the direct FBPs, built once per (geometry, sizes, device) and kept in device
// memory for the life of the process.
struct DirectTables {
  int kind, n, rows, ndet, device;
  float* aff = nullptr;   // [rows] float4: pos = X x + Y y + z
  int* start = nullptr;   // [rows] window start (linogram only)
  float* w = nullptr;     // [rows] row weight (linogram only)
};
std::mutex g_tables_mu;
std::deque<DirectTables> g_tables;   // a deque keeps earlier entries in place as it grows

const DirectTables* direct_tables(int kind, int n, int rows, int ndet) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lock(g_tables_mu);
  for (auto& t : g_tables)
    if (t.kind == kind && t.n == n && t.rows == rows && t.ndet == ndet && t.device == dev)
      return &t;
  DirectTables t{kind, n, rows, ndet, dev};
  std::vector<float> aff((size_t)rows * 4, 0.f), w(rows, 0.f);
  std::vector<int> start(rows, 0);
  const double pi = 3.14159265358979323846;
  if (kind == 0) {   // uniform parallel beam: rows are angles i pi / rows
    for (int a = 0; a < rows; ++a) {
      aff[4 * a + 0] = (float)cos(pi * a / rows);
      aff[4 * a + 1] = (float)sin(pi * a / rows);
      aff[4 * a + 2] = (float)(0.5 * ndet - 0.5);
    }
  } else {           // linogram: row (q, t) over its window, pixel -> window position
    const int N = n;
    std::vector<double> th(N);
    for (int tt = 0; tt < N; ++tt) th[tt] = atan((double)tt / (N - 1));
    for (int q = 0; q < 4; ++q)
      for (int tt = 0; tt < N; ++tt) {
        const int r = q * N + tt;
        const double m = (double)tt / (N - 1);
        const int su = (N - 1 - tt) / 2 - N / 2;               // unwrapped window start
        const double g = (0.5 * N - 0.5) * (1.0 - m) - su;
        double al, be;
        if (q == 0) { al = 1; be = -m; }
        else if (q == 1) { al = -1; be = -m; }
        else if (q == 2) { al = -m; be = 1; }
        else { al = -m; be = -1; }
        aff[4 * r + 0] = (float)al;
        aff[4 * r + 1] = (float)be;
        aff[4 * r + 2] = (float)g;
        start[r] = ((su % N) + N) % N;
        double wt;
        if (tt == 0) wt = 0.5 * (th[1] - th[0]);
        else if (tt == N - 1) wt = 0.5 * (th[N - 1] - th[N - 2]);
        else wt = 0.5 * (th[tt + 1] - th[tt - 1]);
        w[r] = (float)(sqrt(1.0 + m * m) * wt);
      }
  }
  if (hipMalloc(&t.aff, aff.size() * sizeof(float)) != hipSuccess ||
      hipMalloc(&t.start, rows * sizeof(int)) != hipSuccess ||
      hipMalloc(&t.w, rows * sizeof(float)) != hipSuccess ||
      hipMemcpy(t.aff, aff.data(), aff.size() * sizeof(float), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(t.start, start.data(), rows * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t.w, w.data(), rows * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
    hipFree(t.aff);
    hipFree(t.start);
    hipFree(t.w);
    return nullptr;
  }
  g_tables.push_back(t);
  return &g_tables.back();
}

// Per-row geometry of the sinogram resampling (Sec. 4.2, eq 14), one table per (N, P, D,
// device), kept for the life of the process.
struct ResampleTables {
  int n, angles, ndet, device;
  ResampleRow* rows = nullptr;
};
std::deque<ResampleTables> g_resample;

const ResampleTables* resample_tables(int n, int P, int D) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lock(g_tables_mu);
  for (auto& t : g_resample)
    if (t.n == n && t.angles == P && t.ndet == D && t.device == dev) return &t;
  const int N = n;
  const double pi = 3.14159265358979323846;
  const double c = 0.5 * (N - 1);
  std::vector<ResampleRow> rows(4 * N);
  for (int q = 0; q < 4; ++q)
    for (int tt = 0; tt < N; ++tt) {
      const double m = N > 1 ? (double)tt / (N - 1) : 0.0;
      const double k = sqrt(1.0 + m * m);
      // class lines in pixel-centre coordinates: x = s + m y (q = 0), x = N-1-s - m y (q = 1),
      // x and y swapped for q = 2, 3; normal (nx, ny), signed distance alpha + beta s from the
      // image centre
      double nx, ny, alpha, beta;
      if (q == 0 || q == 2) {
        alpha = -c * (1.0 - m) / k;
        beta = 1.0 / k;
      } else {
        alpha = (N - 1 - c * (1.0 + m)) / k;
        beta = -1.0 / k;
      }
      if (q == 0) { nx = 1.0 / k; ny = -m / k; }
      else if (q == 1) { nx = 1.0 / k; ny = m / k; }
      else if (q == 2) { nx = -m / k; ny = 1.0 / k; }
      else { nx = m / k; ny = 1.0 / k; }
      double phi = atan2(ny, nx);
      if (phi < 0) {   // normal angle into [0, pi): flip the normal and the distance
        phi += pi;
        alpha = -alpha;
        beta = -beta;
      }
      const double a = phi * P / pi;
      int a0 = (int)floor(a);
      double wa = a - a0;
      if (a0 >= P) {
        a0 = P - 1;
        wa = 1.0;
      }
      ResampleRow r;
      r.a0 = a0;
      r.a1 = a0 + 1 < P ? a0 + 1 : 0;
      r.wrap = a0 + 1 < P ? 0 : 1;
      r.wa = (float)wa;
      r.u0 = (float)(alpha + 0.5 * D - 0.5);
      r.u1 = (float)(alpha - beta * N + 0.5 * D - 0.5);
      r.du = (float)beta;
      r.pad = 0.f;
      rows[q * N + tt] = r;
    }
  ResampleTables t{n, P, D, dev};
  if (hipMalloc(&t.rows, rows.size() * sizeof(ResampleRow)) != hipSuccess) return nullptr;
  if (hipMemcpy(t.rows, rows.data(), rows.size() * sizeof(ResampleRow),
                hipMemcpyHostToDevice) != hipSuccess) {
    hipFree(t.rows);
    return nullptr;
  }
  g_resample.push_back(t);
  return &g_resample.back();
}

}  // namespace

extern "C" {

const char* fbp_strerror(int code) {
  switch (code) {
    case FBP_OK: return "ok";
    case FBP_EINVAL: return "invalid argument";
    case FBP_EUNSTABLE: return "recursive filter is unstable or has non-finite coefficients";
    case FBP_ENOMEM: return "device allocation failed";
    case FBP_EDEVICE: return "HIP runtime or kernel launch failure";
    case FBP_ERANGE: return "size out of range (batch above max_batch, or a schedule or shape the kernels cannot run)";
    default: return "unknown error";
  }
}

int fbp_plan(const fbp_plan_desc* d, fbp_plan_t* out) {
  if (!out) return FBP_EINVAL;
  *out = nullptr;
  if (!d) return FBP_EINVAL;
  if (!is_pow2(d->n) || d->n < 4 || d->n > 4096) return FBP_EINVAL;
  if (d->max_batch < 1) return FBP_EINVAL;
  if (d->order < 1 || d->order > kMaxOrder) return FBP_EINVAL;
  if (d->groups < 1 || d->groups > 64 || (4 * d->n) % d->groups != 0) return FBP_EINVAL;
  if (!d->a || !d->b) return FBP_EINVAL;
  if (d->flags & ~(FBP_NO_ROW_SCALE | FBP_INPUT_IS_FHT | FBP_ZERO_WINDOW | FBP_NO_SCRATCH))
    return FBP_EINVAL;
  const int K = d->order, G = d->groups;
  for (int i = 0; i < G * K; ++i)
    if (!isfinite(d->a[i]) || !isfinite(d->b[i])) return FBP_EUNSTABLE;
  for (int g = 0; g < G; ++g)
    if (!stable(d->a + (size_t)g * K, K)) return FBP_EUNSTABLE;

  fbp_plan_s* p = new (std::nothrow) fbp_plan_s();
  if (!p) return FBP_ENOMEM;
  p->n = d->n;
  p->log2n = ilog2(d->n);
  p->max_batch = d->max_batch;
  p->order = K;
  p->groups = G;
  p->flags = d->flags;
  p->stream = (hipStream_t)d->stream;
  p->b.assign(d->b, d->b + (size_t)G * K);
  p->a.assign(d->a, d->a + (size_t)G * K);
  if (hipGetDevice(&p->device) != hipSuccess ||
      hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, p->device) !=
          hipSuccess) {
    delete p;
    return FBP_EDEVICE;
  }
  // set-up of fbp_reconstruct_noalloc on this device (its fixed scratch array's address),
  // with the device current; a failure shows only in that call (FBP_EDEVICE)
  resolve_noalloc_scratch(p->device);
  // filter chunks: C = min(64, N / 32) chunks of L = N / C samples per row (C = 1, L = N
  // below N = 32); C never exceeds a wavefront so a row's scan stays in one wave
  const int N = p->n;
  const int C = std::max(1, std::min(64, N / 32));
  p->log2c = ilog2(C);
  p->log2l = p->log2n - p->log2c;
  // LDS row stride: N words plus one skew word per L.  It is 33 C words, = C (mod 64): with a
  // wave holding 64 / C rows of C chunks, the filter's chunk-strided accesses (bank 33 c + C r
  // mod 64) then hit 64 distinct banks
  p->rs = N + (N >> p->log2l);
  // levels per pass: the tile of 2^F full rows must fit the LDS and 2^F * C <= 1024 threads
  int lds_max = 0;
  if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device) !=
      hipSuccess) {
    delete p;
    return FBP_EDEVICE;
  }
  lds_max = std::min(lds_max, kLdsBudget);
  int fmax = 0;
  for (int F = 1; F <= p->log2n && (1 << F) * C <= 1024; ++F) {
    PassArgs t;
    memset(&t, 0, sizeof(t));
    t.log2n = p->log2n;
    t.log2r = F;
    t.log2c = p->log2c;
    t.levels = F;
    t.rs = p->rs;
    if (pass_lds_bytes(t) <= (size_t)lds_max) fmax = F;
  }
  if (fmax < 1) {
    delete p;
    return FBP_ERANGE;
  }
  p->fmax = fmax;
  p->fwd_levels = split_levels(p->log2n, fmax);
  p->levels = backprojection_levels(p->log2n, fmax);
  {
    const int KK = kernel_order(K);
    p->coef_stride = 3 * KK + kScanLevels * KK * KK + KK * (1 << p->log2l);
    // rows of more than 64 chunks of 32 (N = 4096): a second table for the first pass
    if (p->log2n > 11) p->coef_stride32 = 3 * KK + kScanLevels * KK * KK + KK * 32;
  }

  // per-row tables: c_t = k_t w_t (times k_t again for FHT-normalised input), window starts
  std::vector<float> scale(N);
  std::vector<int> sigma(N);
  std::vector<double> th(N);
  for (int t = 0; t < N; ++t) th[t] = atan((double)t / (double)(N - 1));
  for (int t = 0; t < N; ++t) {
    double w;
    if (t == 0) w = 0.5 * (th[1] - th[0]);
    else if (t == N - 1) w = 0.5 * (th[N - 1] - th[N - 2]);
    else w = 0.5 * (th[t + 1] - th[t - 1]);
    const double m = (double)t / (double)(N - 1);
    const double k = sqrt(1.0 + m * m);
    double c = k * w;
    if (p->flags & FBP_INPUT_IS_FHT) c *= k;
    if (p->flags & FBP_NO_ROW_SCALE) c = 1.0;
    scale[t] = (float)c;
    sigma[t] = window_start_of(t, p->log2n, (p->flags & FBP_ZERO_WINDOW) ? 0 : 1);
  }
  const size_t per_class = (size_t)N * N;
  p->scratch_floats = (size_t)p->max_batch * 4 * per_class;
  const int nscratch = (p->flags & FBP_NO_SCRATCH)
                           ? 0
                           : scratch_needed(std::max(p->levels.size(), p->fwd_levels.size()));
  bool ok = hipMalloc(&p->d_coef, (size_t)G * p->coef_stride * sizeof(float)) == hipSuccess &&
            (p->coef_stride32 == 0 ||
             hipMalloc(&p->d_coef32, (size_t)G * p->coef_stride32 * sizeof(float)) ==
                 hipSuccess) &&
            hipMalloc(&p->d_scale, (N + kScalePad) * sizeof(float)) == hipSuccess &&
            hipMalloc(&p->d_sigma, N * sizeof(int)) == hipSuccess;
  for (int i = 0; ok && i < nscratch; ++i)
    ok = hipMalloc(&p->d_scratch[i], p->scratch_floats * sizeof(float)) == hipSuccess;
  if (!ok) {
    free_plan(p);
    return FBP_ENOMEM;
  }
  if (hipMemcpy(p->d_scale, scale.data(), N * sizeof(float), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(p->d_sigma, sigma.data(), N * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
    free_plan(p);
    return FBP_EDEVICE;
  }
  int rc = upload_coefficients(p);
  if (rc != FBP_OK) {
    free_plan(p);
    return rc;
  }
  *out = p;
  return FBP_OK;
}

int fbp_plan_destroy(fbp_plan_t p) {
  if (!p) return FBP_OK;
  hipStreamSynchronize(p->stream);
  free_plan(p);
  return FBP_OK;
}

int fbp_plan_set_stream(fbp_plan_t p, void* stream) {
  if (!p) return FBP_EINVAL;
  p->stream = (hipStream_t)stream;
  return FBP_OK;
}

int fbp_plan_set_coefficients(fbp_plan_t p, const double* b, const double* a) {
  if (!p || !b || !a) return FBP_EINVAL;
  const size_t n = (size_t)p->groups * p->order;
  for (size_t i = 0; i < n; ++i)
    if (!isfinite(a[i]) || !isfinite(b[i])) return FBP_EUNSTABLE;
  for (int g = 0; g < p->groups; ++g)
    if (!stable(a + (size_t)g * p->order, p->order)) return FBP_EUNSTABLE;
  p->b.assign(b, b + n);
  p->a.assign(a, a + n);
  return upload_coefficients(p);
}

int fbp_plan_profile(fbp_plan_t p, int32_t enable) {
  if (!p) return FBP_EINVAL;
  if (enable) clear_recs(p);
  p->profiling = enable != 0;
  return FBP_OK;
}

int fbp_plan_profile_read(fbp_plan_t p, double* total_ms, int32_t* launches) {
  if (!p || !total_ms || !launches) return FBP_EINVAL;
  for (int k = 0; k < FBP_KERNEL_KINDS; ++k) {
    total_ms[k] = 0.0;
    launches[k] = 0;
  }
  int rc = FBP_OK;
  for (auto& r : p->recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.stop) != hipSuccess ||
        hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) {
      rc = FBP_EDEVICE;
      continue;
    }
    total_ms[r.kind] += ms;
    launches[r.kind] += 1;
  }
  clear_recs(p);
  return rc;
}

int fbp_plan_passes(fbp_plan_t p, int32_t* levels, int32_t cap) {
  if (!p || (cap > 0 && !levels)) return FBP_EINVAL;
  const int P = (int)p->levels.size();
  for (int i = 0; i < P && i < cap; ++i) levels[i] = p->levels[i];
  return P;
}

int fbp_filter(fbp_plan_t p, const float* in, float* out, int32_t batch) {
  int rc = check_batch(p, batch);
  if (rc != FBP_OK) return rc;
  if (batch == 0) return FBP_OK;
  if (!in || !out || !aligned16(in) || !aligned16(out)) return FBP_EINVAL;
  PassArgs A = base_args(p);
  // tiles of R rows with the plan's chunking: R * C = 1024 threads at most, LDS permitting
  int log2r = std::min(p->log2n, 10 - p->log2c);
  while (log2r > 0 && (size_t)(1 << log2r) * p->rs * 4 > (size_t)kLdsBudget) --log2r;
  A.levels = 0;
  A.log2r = log2r;
  A.k_hi = p->log2n;
  A.in = in;
  A.out = out;
  A.in_mode = IN_ROWS;
  A.out_mode = OUT_SAME;
  A.order = kernel_order(p->order);
  return timed_pass(p, A, batch, FBP_KERNEL_FILTER, plan_issue(p)) == hipSuccess ? FBP_OK : FBP_EDEVICE;
}

int fht_backproject(fbp_plan_t p, const float* lino, float* img, int32_t batch) {
  int rc = check_batch(p, batch);
  if (rc != FBP_OK) return rc;
  if (batch == 0) return FBP_OK;
  if (!lino || !img || !aligned16(lino) || !aligned16(img)) return FBP_EINVAL;
  return run_passes(p, lino, img, batch, false, false, plan_issue(p));
}

int fbp_reconstruct(fbp_plan_t p, const float* lino, float* img, int32_t batch) {
  int rc = check_batch(p, batch);
  if (rc != FBP_OK) return rc;
  if (batch == 0) return FBP_OK;
  if (!lino || !img || !aligned16(lino) || !aligned16(img)) return FBP_EINVAL;
  return run_passes(p, lino, img, batch, false, true, plan_issue(p));
}

int fbp_reconstruct_noalloc(fbp_plan_t p, const float* lino, float* img, int32_t batch) {
  int rc = check_batch(p, batch);
  if (rc != FBP_OK) return rc;
  if (batch == 0) return FBP_OK;
  if (!lino || !img || !aligned16(lino) || !aligned16(img)) return FBP_EINVAL;
  float* base = noalloc_scratch(p->device);
  if (!base) return FBP_EDEVICE;
  const size_t n2 = (size_t)p->n * p->n;
  const size_t per_buffer = 4 * n2;                 // floats of one slice's intermediate
  const int nbuf = scratch_needed(p->levels.size());
  const size_t chunk = nbuf ? kNoAllocScratchFloats / (nbuf * per_buffer) : (size_t)batch;
  if (chunk == 0) return FBP_ERANGE;                // one slice needs more than the array
  const Issue is{p->stream, false};                 // no timing events: they would allocate
  for (int b0 = 0; b0 < batch; b0 += (int)chunk) {
    const int nb = (int)std::min<size_t>(chunk, (size_t)(batch - b0));
    float* bufs[2] = {base, base + (size_t)nb * per_buffer};
    rc = run_passes(p, lino + (size_t)b0 * per_buffer, img + (size_t)b0 * n2, nb, false, true,
                    is, bufs);
    if (rc != FBP_OK) return rc;
  }
  return FBP_OK;
}

int fht_forward(fbp_plan_t p, const float* img, float* lino, int32_t batch) {
  int rc = check_batch(p, batch);
  if (rc != FBP_OK) return rc;
  if (batch == 0) return FBP_OK;
  if (!lino || !img || !aligned16(lino) || !aligned16(img)) return FBP_EINVAL;
  return run_passes(p, img, lino, batch, true, false, plan_issue(p));
}

int fbp_direct_filter(const float* sino, float* work, int32_t batch, int32_t n_angles,
                      int32_t n_det, void* stream) {
  if (batch < 0 || n_angles < 1 || n_det < 1 || n_det > 16384) return FBP_EINVAL;
  if (batch == 0) return FBP_OK;
  if (!sino || !work) return FBP_EINVAL;
  const float w = (float)(3.14159265358979323846 / n_angles);
  return launch_direct_filter(sino, work, batch * n_angles, n_det, w, nullptr, nullptr, 1,
                              (hipStream_t)stream) == hipSuccess
             ? FBP_OK
             : FBP_EDEVICE;
}

int fbp_direct_backproject(const float* work, float* img, int32_t batch, int32_t n,
                           int32_t n_angles, int32_t n_det, void* stream) {
  if (batch < 0 || n < 32 || n % 32 != 0 || n > 8192 || n_angles < 1 || n_det < 1)
    return FBP_EINVAL;
  if (batch == 0) return FBP_OK;
  if (!work || !img) return FBP_EINVAL;
  const DirectTables* t = direct_tables(0, n, n_angles, n_det);
  if (!t) return FBP_ENOMEM;
  return launch_direct_backproject(work, img, batch, n, n_angles, n_det, t->aff,
                                   (hipStream_t)stream) == hipSuccess
             ? FBP_OK
             : FBP_EDEVICE;
}

int fbp_direct_parallel(const float* sino, float* work, float* img, int32_t batch, int32_t n,
                        int32_t n_angles, int32_t n_det, void* stream) {
  if (batch < 0 || n < 32 || n % 32 != 0 || n > 8192 || n_angles < 1 || n_det < 1 ||
      n_det > 16384)
    return FBP_EINVAL;
  if (batch == 0) return FBP_OK;
  if (!sino || !work || !img) return FBP_EINVAL;
  int rc = fbp_direct_filter(sino, work, batch, n_angles, n_det, stream);
  if (rc != FBP_OK) return rc;
  return fbp_direct_backproject(work, img, batch, n, n_angles, n_det, stream);
}

int fbp_filter_coef_grad(fbp_plan_t p, const float* lino, const float* grad_out, double* grad,
                         int32_t batch) {
  int rc = check_batch(p, batch);
  if (rc != FBP_OK) return rc;
  if (!lino || !grad_out || !grad) return FBP_EINVAL;
  if (p->log2l > 5) return FBP_ERANGE;   // 64-sample chunks (N = 4096) are not supported here
  PassArgs A = base_args(p);
  A.in = lino;
  A.order = kernel_order(p->order);
  // rows per block: <= 512 threads, two tiles of rows in LDS, inside one coefficient group
  int log2r = std::min(p->log2n, 9 - p->log2c);
  while (log2r > 0 && (size_t)2 * (1 << log2r) * p->rs * 4 > (size_t)kLdsBudget) --log2r;
  while (log2r > 0 && ((4 * p->n / p->groups) % (1 << log2r)) != 0) --log2r;
  A.log2r = log2r;
  const int K = A.order;
  const size_t blocks = (size_t)std::max(batch, 1) * 4 * (p->n >> log2r);
  const size_t need = blocks * 2 * K;
  if (need > p->partial_doubles) {
    hipStreamSynchronize(p->stream);
    hipFree(p->d_partial);
    p->d_partial = nullptr;
    p->partial_doubles = 0;
    if (hipMalloc(&p->d_partial, need * sizeof(double)) != hipSuccess) return FBP_ENOMEM;
    p->partial_doubles = need;
  }
  if (batch == 0) {
    std::vector<double> zeros((size_t)p->groups * 2 * p->order, 0.0);
    return hipMemcpyAsync(grad, zeros.data(), zeros.size() * sizeof(double),
                          hipMemcpyHostToDevice, p->stream) == hipSuccess &&
                   hipStreamSynchronize(p->stream) == hipSuccess
               ? FBP_OK
               : FBP_EDEVICE;
  }
  return launch_coef_grad(A, grad_out, p->d_partial, grad, batch, p->order, p->stream) ==
                 hipSuccess
             ? FBP_OK
             : FBP_EDEVICE;
}

namespace {
bool cnn_shape_ok(int cin, int cout) {
  return (cin == 1 && cout == 16) || (cin == 16 && cout == 16) || (cin == 16 && cout == 1);
}
}  // namespace

int fbp_cnn_pack(const float* w, uint16_t* packed, int32_t cin, int32_t cout,
                 int32_t transpose_flip, void* stream) {
  if (!w || !packed || !(cnn_shape_ok(cin, cout) || (cin == 1 && cout == 1))) return FBP_EINVAL;
  return launch_cnn_pack(w, packed, cin, cout, transpose_flip ? 1 : 0, (hipStream_t)stream) ==
                 hipSuccess
             ? FBP_OK
             : FBP_EDEVICE;
}

int32_t fbp_cnn_packed_elems(int32_t cin) { return cin == 16 ? 5 * 64 * 8 : 64 * 8; }

int fbp_cnn_conv(int32_t cin, int32_t cout, const float* in32, const uint16_t* in16,
                 const uint16_t* wpacked, const float* bias, const uint16_t* mask,
                 const float* resid, uint16_t* out16, float* out32, int32_t relu, int32_t batch,
                 int32_t h, int32_t w, void* stream) {
  if (!cnn_shape_ok(cin, cout) || batch < 0 || h < 1 || w < 16 || (w % 16) != 0) return FBP_EINVAL;
  if (batch == 0) return FBP_OK;
  if (!wpacked || (cin == 1 && !in32) || (cin == 16 && !in16) || (cout == 16 && !out16) ||
      (cout == 1 && !out32) || (mask && cout != 16))
    return FBP_EINVAL;
  // BF16 operands and activations move 8 or 16 bytes at a time
  if (!aligned16(wpacked) || (in16 && !aligned16(in16)) || (out16 && !aligned16(out16)) ||
      (mask && !aligned16(mask)))
    return FBP_EINVAL;
  // a block reads input pixels (its halo) that other blocks write: no output over the input
  const size_t px = (size_t)batch * h * w;
  const uintptr_t in = cin == 16 ? reinterpret_cast<uintptr_t>(in16) : reinterpret_cast<uintptr_t>(in32);
  const uintptr_t out =
      cout == 16 ? reinterpret_cast<uintptr_t>(out16) : reinterpret_cast<uintptr_t>(out32);
  const size_t in_bytes = px * (cin == 16 ? 32 : 4), out_bytes = px * (cout == 16 ? 32 : 4);
  if (in < out + out_bytes && out < in + in_bytes) return FBP_EINVAL;
  return launch_cnn_conv(cin, cout, in32, in16, wpacked, bias, mask, resid, out16, out32,
                         relu ? 1 : 0, batch, h, w, (hipStream_t)stream) == hipSuccess
             ? FBP_OK
             : FBP_EDEVICE;
}

int fbp_cnn_forward(const float* img, const uint16_t* w1, const float* b1, const uint16_t* w2,
                    const float* b2, const uint16_t* w3, const float* b3, float* out,
                    int32_t batch, int32_t h, int32_t w, void* stream) {
  if (batch < 0 || h < 1 || w < 1) return FBP_EINVAL;
  if (batch == 0) return FBP_OK;
  if (!img || !w1 || !b1 || !w2 || !b2 || !w3 || !b3 || !out) return FBP_EINVAL;
  if (!aligned16(w1) || !aligned16(w2) || !aligned16(w3)) return FBP_EINVAL;
  if (img == out) return FBP_EINVAL;   // blocks read a halo that other blocks write
  return launch_cnn_fused(img, w1, b1, w2, b2, w3, b3, out, batch, h, w, (hipStream_t)stream) ==
                 hipSuccess
             ? FBP_OK
             : FBP_EDEVICE;
}

int64_t fbp_cnn_wgrad_partial_floats(int32_t cin, int32_t cout, int32_t batch, int32_t h,
                                     int32_t w) {
  if (!cnn_shape_ok(cin, cout) || batch < 1 || h < 1 || w < 64 || (w % 64) != 0) return FBP_EINVAL;
  return cnn_wgrad_partial_floats(cin, cout, batch, h, w);
}

int fbp_cnn_wgrad(int32_t cin, int32_t cout, const float* dz32, const uint16_t* dz16,
                  const float* in32, const uint16_t* in16, float* partial, float* out,
                  int32_t batch, int32_t h, int32_t w, void* stream) {
  if (!cnn_shape_ok(cin, cout) || batch < 1 || h < 1 || w < 64 || (w % 64) != 0) return FBP_EINVAL;
  if (!partial || !out || (cout == 1 && !dz32) || (cout == 16 && !dz16) || (cin == 1 && !in32) ||
      (cin == 16 && !in16))
    return FBP_EINVAL;
  // a pixel's BF16 channels are read 16 bytes at a time; the chunk sums in partial are FP64
  if ((dz16 && !aligned16(dz16)) || (in16 && !aligned16(in16)) ||
      (reinterpret_cast<uintptr_t>(partial) & 7) != 0)
    return FBP_EINVAL;
  return launch_cnn_wgrad(cin, cout, dz32, dz16, in32, in16, partial, out, batch, h, w,
                          (hipStream_t)stream) == hipSuccess
             ? FBP_OK
             : FBP_EDEVICE;
}

int fbp_resample_sinogram(const float* sino, float* lino, int32_t batch, int32_t n,
                          int32_t n_angles, int32_t n_det, void* stream) {
  if (batch < 0 || !is_pow2(n) || n < 4 || n > 4096 || n_angles < 1 || n_det < 1 ||
      n_det > (1 << 16) || (int64_t)n_angles * n_det > (1ll << 31) / 4)
    return FBP_EINVAL;
  if (batch == 0) return FBP_OK;
  if (!sino || !lino || !aligned16(lino)) return FBP_EINVAL;
  const ResampleTables* t = resample_tables(n, n_angles, n_det);
  if (!t) return FBP_ENOMEM;
  return launch_resample(sino, lino, t->rows, batch, n, n_angles, n_det, (hipStream_t)stream) ==
                 hipSuccess
             ? FBP_OK
             : FBP_EDEVICE;
}

int fbp_reconstruct_sinogram(fbp_plan_t p, const float* sino, float* work, float* img,
                             int32_t batch, int32_t n_angles, int32_t n_det) {
  int rc = check_batch(p, batch);
  if (rc != FBP_OK) return rc;
  if (batch == 0) return FBP_OK;
  if (!work || !img || !aligned16(work) || !aligned16(img)) return FBP_EINVAL;
  rc = fbp_resample_sinogram(sino, work, batch, p->n, n_angles, n_det, p->stream);
  if (rc != FBP_OK) return rc;
  return run_passes(p, work, img, batch, false, true, plan_issue(p));
}

int fbp_direct_linogram(const float* lino, float* work, float* img, int32_t batch, int32_t n,
                        void* stream) {
  if (batch < 0 || n < 32 || !is_pow2(n) || n > 4096) return FBP_EINVAL;
  if (batch == 0) return FBP_OK;
  if (!lino || !work || !img) return FBP_EINVAL;
  const DirectTables* t = direct_tables(1, n, 4 * n, n);
  if (!t) return FBP_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  if (launch_direct_filter(lino, work, batch * 4 * n, n, 1.f, t->start, t->w, 4 * n, s) !=
      hipSuccess)
    return FBP_EDEVICE;
  return launch_direct_backproject(work, img, batch, n, 4 * n, n, t->aff, s) == hipSuccess
             ? FBP_OK
             : FBP_EDEVICE;
}

int fbp_plan_set_schedule(fbp_plan_t p, const int32_t* levels, int32_t passes, int32_t log2w) {
  if (!p || !levels || passes < 1) return FBP_EINVAL;
  std::vector<int> lv(levels, levels + passes);
  const int w = log2w == 0 ? p->log2w : log2w;
  int rc = check_schedule(p, lv, w);
  if (rc != FBP_OK) return rc;
  const int have = scratch_needed(std::max(p->levels.size(), p->fwd_levels.size()));
  const int need = scratch_needed(lv.size());
  if (need > have && !(p->flags & FBP_NO_SCRATCH)) {
    if (hipStreamSynchronize(p->stream) != hipSuccess) return FBP_EDEVICE;
    for (int i = 0; i < need; ++i) {
      if (p->d_scratch[i]) continue;
      if (hipMalloc(&p->d_scratch[i], p->scratch_floats * sizeof(float)) != hipSuccess) {
        p->d_scratch[i] = nullptr;
        return FBP_ENOMEM;
      }
    }
  }
  p->levels = lv;
  p->log2w = w;
  p->generation += 1;
  return FBP_OK;
}

int fbp_plan_schedule_info(fbp_plan_t p, int32_t* log2w, int32_t* first_max) {
  if (!p) return FBP_EINVAL;
  if (log2w) *log2w = p->log2w;
  if (first_max) *first_max = p->fmax;
  return FBP_OK;
}

int fbp_plan_filter_info(fbp_plan_t p, int32_t* chunk, int32_t* scan_levels,
                         int32_t* first_levels, int32_t* remainder) {
  if (!p) return FBP_EINVAL;
  if (chunk) *chunk = 1 << p->log2l;
  if (scan_levels) *scan_levels = p->scan_levels;
  if (first_levels) *first_levels = p->d_coef32 ? p->scan_levels32 : p->scan_levels;
  if (remainder) *remainder = p->rem ? 1 : 0;
  return FBP_OK;
}

int fbp_reconstruct_many(const fbp_plan_t* plans, const float* const* lino, float* const* img,
                         const int32_t* batch, int32_t count, void* stream) {
  int rc = check_many(plans, lino, img, batch, count);
  if (rc != FBP_OK) return rc;
  for (int i = 0; i < count; ++i) {
    fbp_plan_s* p = plans[i];
    rc = run_passes(p, lino[i], img[i], batch[i], false, true,
                    Issue{(hipStream_t)stream, p->profiling});
    if (rc != FBP_OK) return rc;
  }
  return FBP_OK;
}

int fbp_graph_create(const fbp_plan_t* plans, const float* const* lino, float* const* img,
                     const int32_t* batch, int32_t count, fbp_graph_t* out) {
  if (!out) return FBP_EINVAL;
  *out = nullptr;
  int rc = check_many(plans, lino, img, batch, count);
  if (rc != FBP_OK) return rc;
  fbp_graph_s* g = new (std::nothrow) fbp_graph_s();
  if (!g) return FBP_ENOMEM;
  // distinct plans, in order of first appearance: branch j of the graph runs plan j's work
  std::vector<int> branch(count);
  for (int i = 0; i < count; ++i) {
    int j = 0;
    while (j < (int)g->plans.size() && g->plans[j].first != plans[i]) ++j;
    if (j == (int)g->plans.size()) g->plans.emplace_back(plans[i], plans[i]->generation);
    branch[i] = j;
  }
  if (count == 0) {   // an empty graph: launches do nothing
    *out = g;
    return FBP_OK;
  }
  const int D = (int)g->plans.size();
  std::vector<hipStream_t> st(D, nullptr);
  std::vector<hipEvent_t> ev(D, nullptr);   // ev[0]: fork, ev[j >= 1]: join of branch j
  bool ok = true;
  for (int j = 0; ok && j < D; ++j)
    ok = hipStreamCreateWithFlags(&st[j], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&ev[j], hipEventDisableTiming) == hipSuccess;
  if (ok) ok = hipStreamBeginCapture(st[0], hipStreamCaptureModeThreadLocal) == hipSuccess;
  const bool capturing = ok;
  if (ok && D > 1) {
    ok = hipEventRecord(ev[0], st[0]) == hipSuccess;
    for (int j = 1; ok && j < D; ++j) ok = hipStreamWaitEvent(st[j], ev[0], 0) == hipSuccess;
  }
  for (int i = 0; ok && i < count; ++i)
    ok = run_passes(plans[i], lino[i], img[i], batch[i], false, true,
                    Issue{st[branch[i]], false}) == FBP_OK;
  for (int j = 1; ok && j < D; ++j)
    ok = hipEventRecord(ev[j], st[j]) == hipSuccess &&
         hipStreamWaitEvent(st[0], ev[j], 0) == hipSuccess;
  if (capturing) {
    hipGraph_t graph = nullptr;
    const bool ended = hipStreamEndCapture(st[0], &graph) == hipSuccess;
    if (ok && ended) {
      g->graph = graph;
      ok = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) == hipSuccess;
    } else {
      ok = false;
      if (graph) hipGraphDestroy(graph);
    }
  }
  for (int j = 0; j < D; ++j) {
    if (ev[j]) hipEventDestroy(ev[j]);
    if (st[j]) hipStreamDestroy(st[j]);
  }
  if (!ok) {
    fbp_graph_destroy(g);
    return FBP_EDEVICE;
  }
  *out = g;
  return FBP_OK;
}

int fbp_graph_launch(fbp_graph_t g, void* stream) {
  if (!g) return FBP_EINVAL;
  for (auto& pg : g->plans)
    if (pg.first->generation != pg.second) return FBP_EINVAL;   // schedule changed since capture
  if (!g->exec) return FBP_OK;
  return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? FBP_OK : FBP_EDEVICE;
}

int fbp_graph_destroy(fbp_graph_t g) {
  if (!g) return FBP_OK;
  if (g->exec) hipGraphExecDestroy(g->exec);
  if (g->graph) hipGraphDestroy(g->graph);
  delete g;
  return FBP_OK;
}

}  // extern "C"
