/*
 * fhtfbp.h -- C ABI of the accelerated filtered back projection library (HIP, gfx950).
 *
 * Method: Dolmatova, Chukalina, Nikolaev, "Accelerated FBP for computed tomography image
 * reconstruction" (ICIP 2020).  A CT slice of N x N pixels (N = 2^n) is rebuilt from its
 * linogram: four N x N images of line integrals, one per line class of the (s, t)
 * parameterisation (Sec. 4.1).  Each detector row is ramp-filtered by a causal plus an
 * anticausal recursive filter (Sec. 3, eq 9-13); the filtered classes are back-projected by
 * the transposed dyadic Fast Hough Transform (Sec. 4.4-4.5, eq 19-21) and summed (eq 22).
 *
 * Data layout (all float32, row-major, caller-owned device memory):
 *   linogram  [batch][4][N][N]   index [b][q][t][s]: class q, slope index t, cyclic shift s
 *   image     [batch][N][N]      index [b][y][x]: pixel row y, column x
 * Class q: 0 = mostly vertical lines with positive shift (x = s + m_t y), 1 = mostly vertical
 * with negative shift (mirror of 0 in x), 2 = mostly horizontal with positive shift (class 0
 * of the transposed image, eq 16), 3 = mostly horizontal with negative shift.  Slope
 * m_t = t / (N - 1).  Linogram values are physical line integrals.
 *
 * Conventions: every call returns 0 or a negative FBP_E* code; argument errors are detected
 * before anything is launched; nothing throws across the ABI.  Calls enqueue work on the
 * plan's HIP stream and return without synchronising.  Pointers must be device pointers
 * (or host-visible device memory) aligned to 16 bytes.  A plan is not thread-safe: do not
 * issue calls on one plan from several host threads at once.
 */
#ifndef FHTFBP_H
#define FHTFBP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------------------------- */
#define FBP_OK          0
#define FBP_EINVAL     -1   /* bad argument: null pointer, N not a power of two, order ... */
#define FBP_EUNSTABLE  -2   /* recursive filter has a pole with |p| >= 1 (or a NaN/Inf)    */
#define FBP_ENOMEM     -3   /* device allocation failed                                    */
#define FBP_EDEVICE    -4   /* a HIP call or kernel launch failed                          */
#define FBP_ERANGE     -5   /* batch above the plan's max_batch, or a size out of range    */

/* ---- plan flags ----------------------------------------------------------------------- */
#define FBP_NO_ROW_SCALE  1u  /* skip the per-row factor c_t = k_t * w_t after the filter  */
#define FBP_INPUT_IS_FHT  2u  /* rows are sums over image rows (eq 15 normalisation): apply
                                 one more k_t, i.e. c_t = k_t^2 * w_t                      */
#define FBP_ZERO_WINDOW   4u  /* filter every row over shifts 0..N-1 instead of the window
                                 centred on the row's central intercept                   */
#define FBP_NO_SCRATCH    8u  /* allocate no inter-pass scratch: the plan then serves
                                 fbp_reconstruct_noalloc (and one-pass sizes, N <= 128);
                                 calls that need the plan's scratch give FBP_EINVAL         */

/* Size of the fixed scratch array of fbp_reconstruct_noalloc, per device. */
#define FBP_NOALLOC_SCRATCH_BYTES (256u << 20)

typedef struct fbp_plan_s* fbp_plan_t;

typedef struct {
  int32_t n;          /* N: power of two, 4 <= N <= 4096 (the dyadic FHT needs 2^k, Sec 4.4) */
  int32_t max_batch;  /* largest batch any call on this plan will pass (>= 1)                */
  int32_t order;      /* K = M = Q of eq 9 (the paper's experiments use Q = M), 1..8          */
  int32_t groups;     /* coefficient sets: the 4N rows in (q, t) order are split into
                         `groups` equal consecutive ranges (angle groups); 1 = one set; must
                         divide 4N and be <= 64                                               */
  const double* b;    /* host [groups][order]: feed-forward b_0..b_{K-1} (eq 9); the causal
                         and the anticausal pass share them (Sec. 3)                          */
  const double* a;    /* host [groups][order]: feedback a_1..a_K (eq 9).  The kernels hold a
                         as float32 (rounded to nearest on upload).  For K >= 2 they take the
                         numerator as B(z) = (1 - z^-1) C(z) + s: float32 taps
                         c_k = -(b_{k+1} + .. + b_{K-1}) (summed in double) applied to the first
                         difference of each row, plus s = sum(b) times the sample.  A group
                         whose b sums to zero (|sum b| <= 1e-12 sum |b|: the zero response at
                         zero frequency that the ramp of eq 6 has) gets s = 0 exactly, so the
                         float32 filter keeps that zero exactly                                */
  uint32_t flags;     /* FBP_* flags above                                                    */
  void* stream;       /* hipStream_t used by every call (NULL = default stream)               */
} fbp_plan_desc;

/* Create a plan for the recursive ramp pair of eq 9 (Sec. 3) and the line geometry of
 * Sec. 4.1: validates the description, checks filter stability (every root of
 * 1 + a_1 z^-1 + ... + a_K z^-K inside the unit circle), builds the per-row tables (window
 * start; row scale c_t = k_t w_t with k_t = sqrt(1 + m_t^2) of eq 15 and the angular weight
 * of the row's slope), the chunk transition matrices of the recursion, and allocates the
 * inter-pass scratch (2 x max_batch x 16 N^2 bytes at most).  Synchronous.
 * On error *out is set to NULL and nothing is allocated. */
int fbp_plan(const fbp_plan_desc* desc, fbp_plan_t* out);

/* Release the plan and its device memory (synchronises its stream first).  NULL is a no-op. */
int fbp_plan_destroy(fbp_plan_t plan);

/* Switch the stream later calls enqueue on. */
int fbp_plan_set_stream(fbp_plan_t plan, void* stream);

/* Replace the recursive-filter coefficients (host arrays shaped as in the description).
 * Synchronises the plan's stream, checks stability, uploads.  Used by the learned filter.
 * The plan also sets how many levels of the filter's chunk-state scan it runs: the first
 * depth at which the chunks left out weigh at most 2^-30 of the chunk states, from the norms
 * of the chunk transition matrices A's coefficients give (no level for fast-decaying poles,
 * every level for poles near the unit circle).
 * Graphs captured on the plan keep working unless the numerator form changes (every group's
 * new b balanced where some old one was not, or the reverse: the kernels then drop or add the
 * remainder term s) or the scan depth does; such graphs refuse to launch (FBP_EINVAL) and
 * must be captured again. */
int fbp_plan_set_coefficients(fbp_plan_t plan, const double* b, const double* a);

/* Row filter alone (Sec. 3, eq 12-13): every linogram row (b, q, t) is read over its window
 * of N cyclic shifts, run through the causal and the anticausal recursion with zero state
 * outside the window, summed, scaled by c_t and written to the same shifts of `lino_out`.
 * In-place (lino_out == lino_in) is allowed.  batch == 0 is a no-op. */
int fbp_filter(fbp_plan_t plan, const float* lino_in, float* lino_out, int32_t batch);

/* Back projection alone (Sec. 4.5, eq 19-22): img = sum over the four classes of the
 * transposed dyadic FHT of the class, mapped back to the image frame.  No filtering.
 * `lino` and `img` must not overlap. */
int fht_backproject(fbp_plan_t plan, const float* lino, float* img, int32_t batch);

/* Forward projection by the dyadic FHT (eq 16-17): lino[b][q][t][s] = sum over image rows of
 * the class-q frame along the dyadic pattern (t, s) (row-sum normalisation, no k_t).  Exact
 * adjoint of fht_backproject.  `img` and `lino` must not overlap. */
int fht_forward(fbp_plan_t plan, const float* img, float* lino, int32_t batch);

/* The method end to end (Sec. 3, eq 9-13, then Sec. 4.4-4.5, eq 19-22): fbp_filter then
 * fht_backproject, with the filter fused into the first back-projection pass (the linogram
 * is read once).  `lino` is not modified. */
int fbp_reconstruct(fbp_plan_t plan, const float* lino, float* img, int32_t batch);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): fbp_reconstruct with its inter-pass scratch taken
 * from a fixed array inside the library, FBP_NOALLOC_SCRATCH_BYTES per device, which each
 * device holds from the library's load until the process ends, instead of from the plan.
 * The call allocates nothing and records no timing events; create the plan beforehand (with
 * FBP_NO_SCRATCH it holds no scratch of its own).  The batch runs in chunks of at most
 * FBP_NOALLOC_SCRATCH_BYTES / (16 N^2 bytes x buffers) slices, buffers = 1 for a schedule of
 * two passes and 2 for three or more; a size whose single slice needs more than the array
 * (N = 4096) gives FBP_ERANGE before anything is launched.  Results are bit-identical to
 * fbp_reconstruct.  Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (other streams, host threads or plans) race on it and must be serialised by the caller.
 * FBP_EDEVICE if the array's address could not be resolved when the plan was made. */
int fbp_reconstruct_noalloc(fbp_plan_t plan, const float* lino, float* img, int32_t batch);

/* Gradient of a loss with respect to the recursive-filter coefficients, for learning them:
 * `lino` is the filter input and `grad_out` dL/d(fbp_filter output), both [batch][4][N][N].
 * Writes grad [groups][2][order] (device, float64): dL/db_k then dL/da_k per group, summed over
 * the batch and the group's rows in a fixed order (deterministic).  Adjoint-state form: the
 * gradient of a recursion is an opposite-direction recursion of the output gradient, run in
 * the same chunked scan as the filter.  N <= 2048. */
int fbp_filter_coef_grad(fbp_plan_t plan, const float* lino, const float* grad_out,
                         double* grad, int32_t batch);

/* Host-side fit of the recursive ramp pair (Sec. 3): minimise the squared error between the
 * impulse response of eq 9 and the causal half h+ of eq 10 over n = 0..length-1 by the
 * Nelder-Mead simplex method (a parameterised through reflection coefficients, so the fit is
 * always stable; b by linear least squares for each a).  flags bit 0 (FBP_FIT_DC_ZERO):
 * constrain sum(b) = 0 (zero response at zero frequency, as the ramp has).  flags bit 1
 * (FBP_FIT_FREQUENCY, not in the paper): fit the pair's frequency response
 * 2 Re(B(e^{iw}) / A(e^{iw})) to the ramp's |w| / (2 pi) in relative squared error at 256
 * frequencies spaced evenly in log w over [pi / length, pi] (the low frequencies the
 * time-domain criterion barely weighs).  Writes b[order], a[order] and the relative error of
 * the fit (L2 over the impulse response; RMS over the frequency grid with bit 1).
 * Deterministic.  No GPU needed. */
#define FBP_FIT_DC_ZERO    1u
#define FBP_FIT_FREQUENCY  2u
int fbp_fit_ramp_iir(int32_t order, int32_t length, uint32_t flags, double* b, double* a,
                     double* rel_err);

/* Direct FBP comparator on a uniform parallel-beam sinogram (Sec. 2, eq 3-5 with the exact
 * ramp of eq 7-8): sino [batch][n_angles][n_det], angle i = i pi / n_angles (unit normal
 * (cos, sin)), detector j at signed distance j - n_det/2 + 1/2 from the image centre.  Each
 * row is filtered by the full-length FIR and weighted pi / n_angles into `work`
 * ([batch][n_angles][n_det] floats, caller-owned), then back-projected with linear
 * interpolation into img [batch][n][n].  Theta(n_angles n^2) per slice. */
int fbp_direct_parallel(const float* sino, float* work, float* img, int32_t batch, int32_t n,
                        int32_t n_angles, int32_t n_det, void* stream);

/* Direct FBP on the linogram itself (Sec. 2-3: the exact ramp of eq 7-8 in place of the
 * recursive pair, exact line positions in place of dyadic patterns): every row (q, t) is read
 * over the same window as fbp_filter, filtered by the full-length FIR, scaled by c_t into
 * `work` ([batch][4N][N] floats, window order), and back-projected with linear interpolation at
 * the exact intercept of each pixel's line; the four classes are summed.  The accuracy yardstick
 * of the method (and the training target of the learned filter).  Theta(N^3) per slice. */
int fbp_direct_linogram(const float* lino, float* work, float* img, int32_t batch, int32_t n,
                        void* stream);

/* The two halves of fbp_direct_parallel, for timing them apart. */
int fbp_direct_filter(const float* sino, float* work, int32_t batch, int32_t n_angles,
                      int32_t n_det, void* stream);
int fbp_direct_backproject(const float* work, float* img, int32_t batch, int32_t n,
                           int32_t n_angles, int32_t n_det, void* stream);

/* ---- scanner input (Sec. 4.2, eq 14) ----------------------------------------------------- */
/* Resample a parallel-beam sinogram onto the four linogram line classes.  sino is
 * [batch][n_angles][n_det] float32: angle i has unit normal (cos, sin) of i * pi / n_angles,
 * detector j sits at signed distance j - n_det/2 + 1/2 (pixels) from the image centre.  Every
 * linogram line (class q, slope index t, shift s; the layout above) is looked up by its normal
 * angle in [0, pi) and its signed distance, linearly in angle and in detector position
 * (bilinear), zero off the detector; angle pi continues at angle 0 with the detector mirrored.
 * The two lines of a cell (shift s and its fold s - N) are summed.  Values stay line
 * integrals: the 1/k_t sample spacing of eq 15 is taken care of by the filter's row scale.
 * lino is [batch][4][n][n], 16-byte aligned.  n a power of two in [4, 4096], n_angles >= 1,
 * 1 <= n_det <= 65536, n_angles * n_det <= 2^29, else FBP_EINVAL.  The per-row geometry is built
 * once per (n, n_angles, n_det, device) in device memory kept until the process ends.  Runs on
 * `stream`. */
int fbp_resample_sinogram(const float* sino, float* lino, int32_t batch, int32_t n,
                          int32_t n_angles, int32_t n_det, void* stream);

/* The method from scanner data: fbp_resample_sinogram into `work` ([batch][4][N][N],
 * caller-owned scratch, 16-byte aligned), then fbp_reconstruct into img, on the plan's stream. */
int fbp_reconstruct_sinogram(fbp_plan_t plan, const float* sino, float* work, float* img,
                             int32_t batch, int32_t n_angles, int32_t n_det);

/* ---- kernel timing -------------------------------------------------------------------- */
/* Kernel kinds reported by fbp_plan_profile_read. */
#define FBP_KERNEL_FIRST   0  /* first back-projection pass (with the filter in reconstruct) */
#define FBP_KERNEL_MIDDLE  1  /* middle back-projection passes (N >= 2048)                   */
#define FBP_KERNEL_LAST_V  2  /* last pass, classes 0 + 1 into image rows                    */
#define FBP_KERNEL_LAST_H  3  /* last pass, classes 2 + 3 added into image columns          */
#define FBP_KERNEL_FORWARD 4  /* forward-transform passes                                    */
#define FBP_KERNEL_FILTER  5  /* filter alone                                                */
#define FBP_KERNEL_LAST    6  /* last pass of 5 levels, N >= 256: all four classes at once,   */
                              /* over 128 x 128 image tiles (takes the place of LAST_V + _H) */
#define FBP_KERNEL_KINDS   7

/* enable != 0: clear and start recording a HIP event pair around every kernel the plan launches
 * (on the plan's stream, so the events time exactly that launch); enable == 0: stop.  Costs
 * two event records per launch and no synchronisation. */
int fbp_plan_profile(fbp_plan_t plan, int32_t enable);

/* Synchronise the recorded events, write per-kind total milliseconds and launch counts
 * (arrays of FBP_KERNEL_KINDS entries) and clear the record. */
int fbp_plan_profile_read(fbp_plan_t plan, double* total_ms, int32_t* launches);

/* ---- learned residual correction ------------------------------------------------------ */
/* A small residual network after the reconstruction, out = img + conv3(relu(conv2(relu(conv1(
 * img))))), 3x3 convolutions with zero padding, 16 hidden channels: the learned part that
 * corrects what the low-order recursive filter leaves.  Convolutions run on the matrix cores
 * with BF16 operands and FP32 accumulation.  Images with one channel are FP32 [b][y][x];
 * 16-channel activations are BF16 NHWC [b][y][x][16] (uint16_t storage).  Supported
 * (cin, cout): (1, 16), (16, 16), (16, 1).  The kernels move BF16 activations, gradients and
 * packed weights 8 or 16 bytes at a time: such a buffer off a 16-byte boundary gives
 * FBP_EINVAL before any launch. */

/* Pack FP32 weights w[cout][cin][3][3] into the matrix-core operand order (fbp_cnn_packed_elems
 * (cin) BF16 values; for transpose_flip, fbp_cnn_packed_elems(cout)).  transpose_flip packs the
 * weights of the convolution that gives the gradient with respect to the input (channels
 * swapped, taps mirrored). */
int fbp_cnn_pack(const float* w, uint16_t* packed, int32_t cin, int32_t cout,
                 int32_t transpose_flip, void* stream);
int32_t fbp_cnn_packed_elems(int32_t cin);

/* One convolution: cout == 16 writes out16 = relu?(conv + bias) times (mask > 0) when mask is
 * given (the ReLU derivative of the layer below, for the backward pass); cout == 1 writes
 * out32 = conv + bias + resid (resid optional, and may be out32 itself).  bias may be NULL.
 * w must be a multiple of 16.  The output must not overlap the input (the kernels read a halo
 * of input pixels that other blocks write): FBP_EINVAL before any launch. */
int fbp_cnn_conv(int32_t cin, int32_t cout, const float* in32, const uint16_t* in16,
                 const uint16_t* wpacked, const float* bias, const uint16_t* mask,
                 const float* resid, uint16_t* out16, float* out32, int32_t relu, int32_t batch,
                 int32_t h, int32_t w, void* stream);

/* The whole network at inference in one launch: out = img + conv3(relu(conv2(relu(conv1(img) +
 * b1)) + b2)) + b3 for FP32 images [batch][h][w] (any h, w >= 1), with w1, w2, w3 packed by
 * fbp_cnn_pack ((1, 16), (16, 16), (16, 1)) and biases b1[16], b2[16], b3[1].  The hidden
 * activations stay on chip (BF16, as fbp_cnn_conv stores them); for a finite image the result
 * equals the three fbp_cnn_conv calls bit for bit.  out must not overlap img. */
int fbp_cnn_forward(const float* img, const uint16_t* w1, const float* b1, const uint16_t* w2,
                    const float* b2, const uint16_t* w3, const float* b3, float* out,
                    int32_t batch, int32_t h, int32_t w, void* stream);

/* Weight and bias gradients, out[cout * cin * 9 + cout] (FP32): dw[co][ci][tap] =
 * sum_p dz[p][co] in[p + off(tap)][ci], db[co] = sum_p dz[p][co]; dz has cout channels and in
 * cin.  `partial` is caller-owned scratch of fbp_cnn_wgrad_partial_floats floats, 8-byte
 * aligned (FBP_EINVAL otherwise); the block sums are added in a fixed order, in FP64
 * (deterministic).  w must be a multiple of 64. */
int64_t fbp_cnn_wgrad_partial_floats(int32_t cin, int32_t cout, int32_t batch, int32_t h,
                                     int32_t w);
int fbp_cnn_wgrad(int32_t cin, int32_t cout, const float* dz32, const uint16_t* dz16,
                  const float* in32, const uint16_t* in16, float* partial, float* out,
                  int32_t batch, int32_t h, int32_t w, void* stream);

/* Human-readable text of an error code (static storage). */
const char* fbp_strerror(int code);

/* Number of HBM passes and fused levels per pass the plan uses (for reports): writes up to
 * `cap` entries into levels[] and returns the pass count, or a negative error. */
int fbp_plan_passes(fbp_plan_t plan, int32_t* levels, int32_t cap);

/* ---- pass schedule (fusion depth) ----------------------------------------------------- */
/* The back projection runs the log2 N butterfly levels of the transposed dyadic FHT (eq 19-21,
 * Sec. 4.4) in a few HBM passes, each fusing a run of consecutive levels in on-chip memory.
 * Every level performs the same pairwise additions whichever pass runs it, so the grouping
 * and the column-tile width change the speed, never the result: images are bit-identical
 * across schedules.
 *
 * fbp_plan_set_schedule replaces the grouping of fbp_reconstruct and fht_backproject:
 * levels[0 .. passes-1] >= 1 must sum to log2 N (else FBP_EINVAL).  Pass 0, which also runs
 * the filter, holds 2^levels[0] full rows in LDS (levels[0] <= first_max of
 * fbp_plan_schedule_info, else FBP_ERANGE).  For N >= 256 the later passes work on tiles of
 * 2^levels[i] rows by 2^log2w columns plus a halo; 6 <= log2w <= min(10, log2 N), 0 keeps the
 * current width, and a tile that does not fit the LDS gives FBP_ERANGE.  A last pass of 5
 * levels runs over 128 x 128 image tiles whatever the width (the width still applies to the
 * middle passes and to a last pass of other depth).  Below N = 256 every
 * pass holds full rows.  fht_forward keeps the plan's initial schedule.  When the new schedule
 * needs more scratch than the plan holds, the call synchronises the plan's stream and
 * allocates it (FBP_ENOMEM on failure, the schedule unchanged).  Graphs captured before the
 * call refuse to launch (FBP_EINVAL) and must be captured again. */
int fbp_plan_set_schedule(fbp_plan_t plan, const int32_t* levels, int32_t passes, int32_t log2w);

/* Current column-tile width (log2) and the most levels pass 0 can fuse; either pointer may be
 * NULL. */
int fbp_plan_schedule_info(fbp_plan_t plan, int32_t* log2w, int32_t* first_max);

/* How the plan's row filter runs (Sec. 3, eq 9-13), any pointer may be NULL: `chunk` the
 * samples per chunk of the chunked recursion; `scan_levels` the levels of the chunk-state
 * scan its coefficients need (0 .. 7, the largest over the angle groups; the scan stops at the
 * first level j where ||Phi^(chunk 2^j)|| / (1 - ||Phi^chunk||), infinity norm, is at most
 * 2^-30, and runs every level when ||Phi^chunk|| >= 1); `first_levels` the same for the
 * chunks of the fused first back-projection pass, which are 32 samples at N = 4096 and the
 * filter's own (first_levels == scan_levels) at every other size; `remainder` 1 when the numerator's taps do not sum to zero within rounding and the
 * kernels add the remainder term s of B(z) = (1 - z^-1) C(z) + s, else 0.  Each follows the
 * last fbp_plan_set_coefficients. */
int fbp_plan_filter_info(fbp_plan_t plan, int32_t* chunk, int32_t* scan_levels,
                         int32_t* first_levels, int32_t* remainder);

/* ---- mixed batches and captured execution ------------------------------------------------ */
typedef struct fbp_graph_s* fbp_graph_t;

/* Reconstruct `count` sub-batches in one call (eq 9-13 then eq 19-22 per slice, as
 * fbp_reconstruct): sub-batch i is batch[i] slices of plans[i]'s size, linogram lino[i] and
 * image img[i] in the layouts above.  The plans may differ in N, order and coefficients, which
 * makes a batch of mixed sizes one call.  Everything runs on `stream` (a HIP stream, NULL for
 * the null stream) in sub-batch order; a plan that is profiling records its events there.
 * All arguments are checked before anything is launched: count < 0, a NULL array, a NULL
 * plan, a NULL or unaligned buffer of a non-empty sub-batch or plans on different devices give
 * FBP_EINVAL, a batch above its plan's max_batch FBP_ERANGE.  count == 0 does nothing. */
int fbp_reconstruct_many(const fbp_plan_t* plans, const float* const* lino, float* const* img,
                         const int32_t* batch, int32_t count, void* stream);

/* Capture the work of fbp_reconstruct_many with the same arguments into an executable HIP graph
 * (*out), so that one fbp_graph_launch replays every kernel of every sub-batch with a single
 * host call.  Sub-batches of distinct plans become parallel branches of the graph (each plan
 * owns its scratch); sub-batches that share a plan run in order.  The graph keeps the buffer
 * pointers given here and the plans' internal buffers: the plans must outlive it, and a
 * launch must not overlap other work on the same plans.  Coefficient updates
 * (fbp_plan_set_coefficients) are seen by later launches; a schedule change is not (the launch
 * then fails with FBP_EINVAL).  Profiling events are not captured.  The capture uses streams
 * and events of its own, destroyed before it returns.  FBP_EDEVICE if capture or
 * instantiation fails.  count == 0 gives a graph whose launches do nothing. */
int fbp_graph_create(const fbp_plan_t* plans, const float* const* lino, float* const* img,
                     const int32_t* batch, int32_t count, fbp_graph_t* out);

/* Enqueue one replay of the graph on `stream` (NULL: the null stream); returns without
 * synchronising. */
int fbp_graph_launch(fbp_graph_t graph, void* stream);

/* Free the graph (NULL is a no-op).  Synchronise any stream it was launched on first. */
int fbp_graph_destroy(fbp_graph_t graph);

#ifdef __cplusplus
}
#endif
#endif /* FHTFBP_H */
