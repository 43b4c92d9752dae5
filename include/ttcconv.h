/*
 * ttcconv.h -- C ABI of the MI355X (gfx950) library for direct n-D convolution,
 * image pyramids, first-difference derivative cubes and multi-scale
 * time-to-contact (TTC) / focus-of-expansion (FOE) estimation.
 *
 * Method: "Accelerated Convolutions for Efficient Multi-Scale Time to Contact
 * Computation in Julia" (Amini, Horn, Edelman).  Each entry point names the
 * passage of the paper that defines what it computes.
 *
 * Conventions shared by every entry point
 *  - Every buffer is owned by the caller.  Data pointers inside tc_tensor and
 *    the workspace are DEVICE pointers unless stated otherwise; descriptor
 *    structs themselves (tc_tensor, tc_seq) are read on the host during the
 *    call and may be freed when it returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Every
 *    launch is asynchronous on that stream; no entry point synchronises except
 *    tc_ttc_solve_batched and tc_ttc_plan_destroy, which say so.
 *  - No entry point allocates or frees device memory.
 *  - A negative return value other than TC_EDEVICE means the arguments were
 *    rejected and nothing was launched.  TC_EDEVICE reports a launch the
 *    runtime refused; in calls made of several launches, the ones before it
 *    may have run.  No C++ exception crosses this interface.
 *  - Strides are in elements and row-major (the last dimension is the
 *    fastest).  A stride of 0 on a dimension of extent > 1 is rejected.
 */
#ifndef TTCCONV_H
#define TTCCONV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes.  Positive values are per-result statuses (tc_ttc_level.status). */
enum {
  TC_OK = 0,
  TC_SINGULAR = 1,   /* the 3x3 normal matrix is rank deficient (e.g. a linear-ramp video) */
  TC_NEED_PREV = 2,  /* a stream has no previous frame yet (serving) */
  TC_NONFINITE = 3,  /* a sum is NaN or infinite (non-finite input) */
  TC_EINVAL = -1,    /* bad argument (NULL pointer, bad mode, too many levels, ...) */
  TC_ESHAPE = -2,    /* inconsistent shapes or strides */
  TC_EDTYPE = -3,    /* unsupported dtype combination */
  TC_EOVERFLOW = -4, /* an exact integer result could exceed int32 */
  TC_ENOMEM = -5,    /* workspace too small */
  TC_EDEVICE = -6    /* HIP error or a device other than gfx950 */
};

/* Element types. */
enum { TC_U8 = 0, TC_F16 = 1, TC_F32 = 2, TC_I32 = 3, TC_F64 = 4 };

/* Convolution output modes. */
enum { TC_FULL = 0, TC_SAME = 1, TC_VALID = 2 };

#define TC_MAX_DIMS 8
#define TC_MAX_LEVELS 4
#define TC_NUM_SUMS 10

/* A strided n-D array.  `data` is a device pointer (ignored by the pure
 * shape queries). */
typedef struct {
  void* data;
  int32_t dtype;
  int32_t ndim;
  int64_t shape[TC_MAX_DIMS];
  int64_t stride[TC_MAX_DIMS];
} tc_tensor;

/* Human-readable name of a return code or status.  Never NULL. */
const char* tc_status_str(int status);

/* Library version as major*10000 + minor*100 + patch. */
int tc_version(void);

/* Checks that HIP device `device` is a gfx950 and returns its number of
 * compute units in *n_cu (may be NULL).  TC_EDEVICE otherwise. */
int tc_device_check(int device, int* n_cu);

/* ------------------------------------------------------------------------
 * Direct n-D convolution
 *
 * Discrete Derivatives section, the spatial convolution equation; the paper
 * writes the sum as a correlation over the image extent, and it is read here
 * as true convolution over the kernel extent (the routine the paper's
 * Benchmarking subsection compares with), for arrays of any rank
 * (Accelerating Convolutions: n-dimensional convolution):
 *
 *     y[n] = sum_m x[m] * k[n - m],  zero outside the extents of x and k.
 *
 * Modes: TC_FULL (extent N+K-1), TC_SAME (extent N, starting at (K-1)/2 of
 * the full result), TC_VALID (extent |N-K|+1, starting at min(N,K)-1; needs
 * N >= K in every dimension or K >= N in every dimension).  The kernel may be
 * larger than x (full mode is commutative).
 *
 * dtypes (x, k -> y): F32,F32->F32; F16,F32->F32; U8,I32->I32 (exact).  x
 * and k have the same rank 1..8.  x and y may be strided; k must be
 * contiguous and at most 2^20 elements, and is read from DEVICE memory.  y
 * must not overlap x or k.  Float results are accumulated in FP32 (the order
 * of the taps is not specified).  Launches only: no entry point here reads
 * the kernel back to the host.
 *
 * tc_conv_nd: the direct kernels.  F32 and F16 inputs only: an I32 kernel is
 * rejected with TC_EINVAL, because its exactness bound is a property of the
 * taps that only the caller can state without a device-to-host read; integer
 * convolutions go through tc_conv_nd_ex.
 *
 * tc_conv_nd_ex: the same convolution with a choice of method (the hybrid of
 * the Accelerating Convolutions section: direct for small kernels, FFT from
 * a kernel-size threshold; the separable form of the Future Work section):
 *   method TC_CONV_DIRECT  the direct kernels;
 *          TC_CONV_FFT     the FFT branch (F32, rank 2 or 3, padded extents
 *                          within the transform limits; needs the workspace
 *                          of tc_conv_workspace_size, TC_ENOMEM if smaller);
 *          TC_CONV_AUTO    the FFT branch when it applies, the kernel's longest
 *                          side is >= fft_threshold (0: the library's measured
 *                          crossover for the rank) and the workspace is large
 *                          enough; else,
 *                          when k_host is given and k is a square F32 2-D
 *                          kernel of 3, 5, 7, 9, 11 or 15 taps that passes the
 *                          rank-one test of tc_conv_kernel_rank1 with tolerance
 *                          2^-20, the separable kernel with the factors passed
 *                          by value; else the direct kernels.
 *   k_abs_sum  U8,I32 only: sum over the kernel of |k|, a HOST-side value the
 *          caller guarantees.  Rejected with TC_EOVERFLOW unless
 *          255 * k_abs_sum <= 2^31-1 (then every partial sum fits int32 and the
 *          result is exact); TC_EINVAL when neither k_abs_sum >= 0 nor k_host
 *          is given.  A wrong value voids the exactness guarantee.
 *   k_host optional HOST copy of k (same dtype and contiguous layout), read
 *          during the call only: gives k_abs_sum for I32 kernels and enables
 *          the separable test.  NULL when not available.
 *   workspace, workspace_bytes  DEVICE scratch for the FFT branch (may be NULL
 *          and 0 when only the direct or separable paths may run).
 *   band_rows  output rows per wave of the row-streaming direct kernels (2-D
 *          images and 3-D kernels other than 3 x 3 x 3, kernels of 2, 3, 5 or 7
 *          taps per side): 2, 4 or 8, or 0 for the library's tuned default.
 *          Every value gives the same result bit for bit (the summation order
 *          of an output does not depend on it); TC_EINVAL for other values.
 *   reserved  must be 0 (TC_EINVAL otherwise).
 * opts may be NULL: TC_CONV_AUTO with no workspace and no host copy, i.e. the
 * direct kernels (which reject I32 kernels as above).
 *
 * tc_conv_workspace_size: bytes of device workspace tc_conv_nd_ex needs for
 * these shapes with `method` (0 when no FFT branch applies, or for
 * TC_CONV_DIRECT; for TC_CONV_FFT an error when the FFT branch does not apply).
 * ------------------------------------------------------------------------ */
enum { TC_CONV_AUTO = 0, TC_CONV_DIRECT = 1, TC_CONV_FFT = 2 };
typedef struct {
  int32_t method;
  int32_t fft_threshold;
  int64_t k_abs_sum;
  const void* k_host;
  void* workspace;
  size_t workspace_bytes;
  int32_t band_rows;
  int32_t reserved;  /* 0 */
} tc_conv_opts;

int tc_conv_out_shape(const tc_tensor* x, const tc_tensor* k, int32_t mode, int64_t* out_shape);
int tc_conv_nd(const tc_tensor* x, const tc_tensor* k, int32_t mode, const tc_tensor* y, void* stream);
int tc_conv_workspace_size(const tc_tensor* x, const tc_tensor* k, int32_t mode, int32_t method, size_t* ws_bytes);
int tc_conv_nd_ex(const tc_tensor* x, const tc_tensor* k, int32_t mode, const tc_tensor* y,
                  const tc_conv_opts* opts, void* stream);

/* ------------------------------------------------------------------------
 * Separable kernels
 *
 * Future Work section: a kernel that is the outer product of two vectors,
 * k[a][b] = u[a] v[b] (directional derivatives, Gaussian smoothing, block
 * averages), can be applied as two one-dimensional convolutions, 2K instead
 * of K^2 multiply-adds per output.
 *
 * tc_conv_kernel_rank1: HOST arrays.  k is KH x KW, row-major.  Returns 1 and
 * writes u[KH], v[KW] (FP32) when every |k[a][b] - u[a] v[b]| <= tol * max|k|
 * (checked in double with the FP32 factors), 0 when k has no such
 * factorisation (or holds a non-finite value), TC_EINVAL on bad arguments.
 *
 * tc_conv_nd_separable: y = x (*) (u v^T) with the modes and output extents of
 * tc_conv_nd for a K x K kernel.  x and y are 2-D F32 with unit stride along
 * their rows (the row stride is free); u and v are contiguous 1-D F32 of the
 * same length K in {3, 5, 7, 9, 11, 15}, in DEVICE memory.  Both passes run
 * in one kernel (no workspace, no intermediate image).  TC_EINVAL for other
 * K, TC_ESHAPE / TC_EDTYPE as tc_conv_nd.
 * ------------------------------------------------------------------------ */
int tc_conv_kernel_rank1(const float* k, int32_t KH, int32_t KW, double tol, float* u, float* v);
int tc_conv_nd_separable(const tc_tensor* x, const tc_tensor* u, const tc_tensor* v, int32_t mode,
                         const tc_tensor* y, void* stream);

/* ------------------------------------------------------------------------
 * FFT branch of 2-D and 3-D convolution
 *
 * Convolutions section: by the convolution theorem y = F^-1(F(x) F(k)), the
 * route the paper's hybrid FastConv takes for kernels above a size threshold
 * (Accelerating Convolutions); the Future Work section's n-dimensional
 * extension, here for rank 2 and rank 3.  The result, modes and output
 * extents are those of tc_conv_nd for F32 x and k of equal rank (2 or 3).
 * Each axis is zero-padded to the smallest 2^a 3^b 5^c that holds the full
 * output (x extent + k extent - 1), at most 4096 (TC_ESHAPE beyond); x and k
 * are transformed (mixed-radix Stockham, radix 2, 3, 4 and 5, FP32, twiddles
 * rounded from FP64), multiplied, transformed back and cut to the mode.  x and
 * y may be strided; k is contiguous device memory.  ws: device workspace of
 * tc_conv_fft_workspace_size bytes (three complex volumes of the padded size
 * and one twiddle table per axis; TC_ENOMEM if smaller).  Error: norm-wise,
 * about 2^-24 * (the transform's stage count) * ||x||_2 ||k||_1 per output (not
 * the element-wise bound of the direct path).  Launches only.
 *
 * tc_conv2d_fft_workspace_size / tc_conv2d_fft: the same for rank 2 only
 * (TC_ESHAPE for other ranks).
 * ------------------------------------------------------------------------ */
int tc_conv_fft_workspace_size(const tc_tensor* x, const tc_tensor* k, int32_t mode, size_t* ws_bytes);
int tc_conv_fft(const tc_tensor* x, const tc_tensor* k, int32_t mode, const tc_tensor* y, void* ws,
                size_t ws_bytes, void* stream);
int tc_conv2d_fft_workspace_size(const tc_tensor* x, const tc_tensor* k, int32_t mode, size_t* ws_bytes);
int tc_conv2d_fft(const tc_tensor* x, const tc_tensor* k, int32_t mode, const tc_tensor* y, void* ws,
                  size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Image pyramid
 *
 * Time to Contact, Results: down-sampling by a block-averaging filter,
 * repeated for several consecutive levels.  Read as the 2x2 block mean with
 * no further low-pass filter; odd extents are floored:
 *
 *     P_{l+1}[i][j] = (P_l[2i][2j] + P_l[2i][2j+1] + P_l[2i+1][2j] + P_l[2i+1][2j+1]) / 4
 *
 * `frame` is a 2-D U8, F16 or F32 image (strided).  `out` points to an array
 * of (levels - 1) 2-D F32 tensors (host array of descriptors, device data),
 * out[l-1] receiving level l with extent floor(H/2^l) x floor(W/2^l).
 * levels is 1..16; level levels-1 must be at least 1x1.  Exact for U8 frames.
 * ------------------------------------------------------------------------ */
int tc_pyramid_shape(int64_t H, int64_t W, int32_t level, int64_t* Hl, int64_t* Wl);
int tc_image_pyramid(const tc_tensor* frame, int32_t levels, const tc_tensor* out, void* stream);

/* ------------------------------------------------------------------------
 * First-difference derivative cube of one frame pair
 *
 * Discrete Derivatives section: the one-pixel forward difference (mask
 * [-1, 1]) and its 2x2 form (1/2)[[-1, 1], [-1, 1]] for E_x (transpose for
 * E_y), extended over the two frames of a pair:
 *
 *   E_x(i,j) = 1/4 sum_{a,c} [P_c(i+a,j+1) - P_c(i+a,j)]
 *   E_y(i,j) = 1/4 sum_{b,c} [P_c(i+1,j+b) - P_c(i,j+b)]
 *   E_t(i,j) = 1/4 sum_{a,b} [P_1(i+a,j+b) - P_0(i+a,j+b)]
 *
 * for 0 <= i <= H-2, 0 <= j <= W-2 (x = column, y = row).  prev and next are
 * 2-D U8/F16/F32 images of the same shape and dtype.  ex, ey, et are
 * (H-1) x (W-1): F32 outputs receive E (FP32, exact for U8 and rendered-F16
 * data); I32 outputs (U8 input only) receive the exact numerators 4*E.
 * ------------------------------------------------------------------------ */
int tc_horn_derivs(const tc_tensor* prev, const tc_tensor* next, const tc_tensor* ex, const tc_tensor* ey,
                   const tc_tensor* et, void* stream);

/* ------------------------------------------------------------------------
 * Image gradient, magnitude and direction
 *
 * Discrete Derivatives section: the gradient's magnitude |E| = sqrt(E_x^2 +
 * E_y^2) and its direction, the four-quadrant inverse tangent of (E_y, E_x)
 * in [-pi, pi], at every position of a mask; Convolutions section: the masks.
 * The figure that gives the masks is missing from the text, so they take their
 * textbook coefficients, scaled so that the ramp E = x has E_x = 1:
 *   TC_STENCIL_FD2       (1/2)[[-1, 1], [-1, 1]] and its transpose (the
 *                        Discrete Derivatives mask; 2x2 Prewitt)
 *   TC_STENCIL_ROBERTS   E(i+1,j+1) - E(i,j) and E(i+1,j) - E(i,j+1), / sqrt(2)
 *                        (axes turned by 45 degrees)
 *   TC_STENCIL_PREWITT3  rows [-1, 0, 1] / 6 and the transpose
 *   TC_STENCIL_SOBEL3    rows [-1, 0, 1] weighted 1, 2, 1, / 8, and the transpose
 * Masks are applied as written (no flip) where they fit: outputs are
 * (H-1) x (W-1) for the 2x2 masks and (H-2) x (W-2) for the 3x3 ones, x = column.
 * `image` is a 2-D U8, F16 or F32 image (strided); ex, ey, mag, dir are 2-D
 * F32 tensors of the output extent, each optional (NULL descriptor or NULL
 * data: not computed).  Computed in FP32 (integer mask weights summed first,
 * one scale).
 * ------------------------------------------------------------------------ */
#define TC_STENCIL_FD2 0
#define TC_STENCIL_ROBERTS 1
#define TC_STENCIL_PREWITT3 2
#define TC_STENCIL_SOBEL3 3
int tc_gradient(const tc_tensor* image, int32_t stencil, const tc_tensor* ex, const tc_tensor* ey,
                const tc_tensor* mag, const tc_tensor* dir, void* stream);

/* ------------------------------------------------------------------------
 * Time to contact and focus of expansion
 *
 * Time to Contact, Formulation: with the radial gradient G = x E_x + y E_y,
 * least squares of A E_x + B E_y + C G + E_t over every derivative cube gives
 * the 3x3 normal equations
 *
 *   [S(ExEx) S(ExEy) S(GEx)] [A]     [S(ExEt)]
 *   [S(ExEy) S(EyEy) S(GEy)] [B] = - [S(EyEt)]
 *   [S(GEx)  S(GEy)  S(GG) ] [C]     [S(GEt) ]
 *
 * and then x0 = -A/C, y0 = -B/C, TTC = 1/C.  Results subsection: the same is
 * done on each pyramid level, and the multi-scale estimate descends while the
 * TTC estimate keeps decreasing.
 *
 * Readings: x, y are cube centres in base-image pixels from the base-image
 * centre (x right, y down): a cube of level l between pixels (i,j) and
 * (i+1,j+1) sits at x = 2^l (j+1) - W/2, y = 2^l (i+1) - H/2.  Spatial
 * derivatives are per base pixel, so A, B, x0, y0 are in base pixels and C,
 * TTC per frame at every level.  C > 0 for an approaching camera.  The 3x3
 * system is solved in FP64 by Gaussian elimination with partial pivoting on
 * the equilibrated matrix D M D (D = diag(M_ii^-1/2)); it is TC_SINGULAR when
 * a diagonal entry is not positive or an equilibrated pivot is below 1e-6.
 * Multi-scale: an estimate that is singular, non-finite or not positive counts
 * as +infinity; descend from level 0 while the next level's estimate is
 * smaller; stop at the first non-decrease.
 *
 * Precision: frames are U8 or F16; derivatives are formed in FP32 (exact for
 * U8 and rendered-F16 frames at levels 0..3), products are FP32, each wave
 * sums a block of cubes in FP32 and the blocks are combined with TwoSum
 * (hi, lo) compensation; only the 3x3 solve is FP64.
 * ------------------------------------------------------------------------ */

/* The ten sums, in this order, in base-pixel units:
 *   S(ExEx), S(ExEy), S(EyEy), S(GEx), S(GEy), S(GG), S(ExEt), S(EyEt), S(GEt), S(EtEt) */
typedef struct {
  double sums[TC_NUM_SUMS];
  double A, B, C;
  double ttc, x0, y0;
  double resid;   /* sum of (A Ex + B Ey + C G + Et)^2 at the solution */
  int64_t n;      /* number of cubes summed */
  int32_t level;  /* pyramid level (0 = base) */
  int32_t status; /* TC_OK, TC_SINGULAR or TC_NONFINITE; A..resid are NaN unless TC_OK */
} tc_ttc_level;

/* The multi-scale choice for one frame pair. */
typedef struct {
  double ttc, x0, y0;
  double A, B, C;
  int32_t level;  /* selected level */
  int32_t status; /* status of the selected level */
} tc_ttc_pick;

/* A video stream of n_frames frames of H x W pixels.  Frame k starts at
 * frame0 + k * frame_stride elements and row i of it at + i * row_stride.
 * Pairs (k, k+1), k = 0 .. n_frames-2, are processed; a frame is read by the
 * two pairs it belongs to, whose work runs side by side (the second read is
 * normally served by the caches).  A single pair of unrelated frames is a stream with
 * n_frames = 2 and frame_stride = next - prev (in elements, may be negative). */
typedef struct {
  const void* frame0;
  int64_t frame_stride;
  int64_t row_stride;
  int32_t H, W;
  int32_t n_frames;
  int32_t levels;
} tc_seq;

typedef struct tc_ttc_plan tc_ttc_plan;

/* Validates a batch of streams (all of dtype U8 or F16, all with the same
 * number of levels 1..TC_MAX_LEVELS, every level at least 2x2, H and W at most
 * 2^20, row_stride >= W, frame0 aligned to the element size) and builds its
 * work tables in pinned host memory.  Streams whose frames and rows start on
 * 8-pixel boundaries are read with vector loads, others element by element.
 * Host-only; *plan must be released with tc_ttc_plan_destroy.
 * Output layout: stream-major, then pair, then level: stream s, pair p,
 * level l is levels_out[pair_base(s) * L + p * L + l] and picks_out[pair_base(s) + p],
 * pair_base(s) = sum over earlier streams of (n_frames - 1). */
int tc_ttc_plan_create(const tc_seq* seqs, int32_t n_seqs, int32_t dtype, tc_ttc_plan** plan);

/* Launch shape of the fused pass.  band_rows: base rows of each band a wave
 * walks for one frame pair (a multiple of 16 from 16 to 256; a wave holds one
 * to four bands of column strips side by side, the strip width chosen per
 * stream; taller bands walk fewer halo rows per owned row and give fewer,
 * longer work items); groups_per_cu:
 * work-groups (one wave each) of the persistent grid per compute unit
 * (1..256).  The sums depend on band_rows through their blocking (not on
 * groups_per_cu); a fixed tuning gives bit-identical results for a stream
 * whatever else is in the batch. */
typedef struct {
  int32_t band_rows;
  int32_t groups_per_cu;
} tc_ttc_tuning;
/* The built-in tuning for (dtype, levels), chosen by the tuning sweep of the
 * fused pass on MI355X. */
int tc_ttc_tuning_default(int32_t dtype, int32_t levels, tc_ttc_tuning* out);
/* tc_ttc_plan_create with an explicit tuning (NULL = the built-in one). */
int tc_ttc_plan_create_ex(const tc_seq* seqs, int32_t n_seqs, int32_t dtype, const tc_ttc_tuning* tuning,
                          tc_ttc_plan** plan);
/* Re-plans an existing plan for a new batch (same dtype and levels) in place:
 * the pinned table is reused when it is large enough (re-allocated otherwise).
 * For serving loops that plan every tick.  The plan's previous upload must
 * have completed (the table is overwritten), and the workspace size may change
 * (query it again with tc_ttc_plan_info). */
int tc_ttc_plan_reset(tc_ttc_plan* plan, const tc_seq* seqs, int32_t n_seqs);
/* Workspace bytes the plan needs, the total number of pairs and the number
 * of tc_ttc_level records (pairs * levels). */
int tc_ttc_plan_info(const tc_ttc_plan* plan, size_t* ws_bytes, int64_t* n_pairs, int64_t* n_level_records);
/* Asynchronously copies the plan's work tables into the workspace on
 * `stream`; the plan must stay alive until the stream has passed the copy. */
int tc_ttc_plan_upload(const tc_ttc_plan* plan, void* ws, size_t ws_bytes, void* stream);
/* Launches the fused pass (pyramid + derivative cube + products + block
 * sums, persistent, each frame read once) and the finishing pass
 * (compensated block reduction, FP64 solve, multi-scale choice).  Launches
 * only: may be captured in a HIP graph.  Reads the frames through the
 * pointers given at plan creation. */
int tc_ttc_plan_run(const tc_ttc_plan* plan, void* ws, size_t ws_bytes, tc_ttc_level* levels_out,
                    tc_ttc_pick* picks_out, void* stream);
/* The two launches of tc_ttc_plan_run separately: phase 1 is the fused pass
 * (writes the per-wave partial sums into the workspace), phase 2 the finishing
 * pass (reads them, writes levels_out and picks_out; may be NULL in phase 1).
 * Phase 3 runs both.  For timing or overlapping the phases on a stream. */
#define TC_PHASE_FUSED 1
#define TC_PHASE_FINISH 2
int tc_ttc_plan_run_phase(const tc_ttc_plan* plan, void* ws, size_t ws_bytes, tc_ttc_level* levels_out,
                          tc_ttc_pick* picks_out, int32_t phase, void* stream);
/* Frees the plan (synchronises the device first). */
void tc_ttc_plan_destroy(tc_ttc_plan* plan);

/* The multi-scale choice re-applied to level records already in device
 * memory (levels_out of a run: n_pairs x levels records, pair-major) into
 * picks_out[n_pairs].  TC_SELECT_DECREASING_TTC is the Results subsection's
 * rule as every run applies it (descend while the TTC estimate keeps
 * decreasing); TC_SELECT_MIN_RESIDUAL reads "improved" as a better fit: the
 * level with a valid TTC and the smallest residual per cube (resid / n), the
 * lower level on a tie, level 0 when none is valid.  levels_per_pair is 1..16
 * (TC_EINVAL otherwise, or for another rule); both arrays are device memory
 * owned by the caller.  Launches only (no allocation, no synchronisation). */
#define TC_SELECT_DECREASING_TTC 0
#define TC_SELECT_MIN_RESIDUAL 1
int tc_ttc_reselect(const tc_ttc_level* levels, int64_t n_pairs, int32_t levels_per_pair, int32_t rule,
                    tc_ttc_pick* picks_out, void* stream);

/* Create + upload + run + stream synchronise + destroy, for one-off calls. */
int tc_ttc_solve_batched(const tc_seq* seqs, int32_t n_seqs, int32_t dtype, void* ws, size_t ws_bytes,
                         tc_ttc_level* levels_out, tc_ttc_pick* picks_out, void* stream);

/* ------------------------------------------------------------------------
 * Time to contact with another derivative stencil or a pyramid low-pass
 *
 * Convolutions section: the centred 3x3 Prewitt and Sobel masks as the
 * derivative stencil; Time to Contact, Results: a low-pass filter after each
 * block mean.  The same least-squares estimate and multi-scale rule as
 * tc_ttc_solve, through materialised levels (a comparison path: each level
 * image is written once and read back).
 *
 * stencil: TC_STENCIL_FD2 (the 2x2x2 cube of tc_ttc_solve, estimates between
 *   pixels, (H_l-1)(W_l-1) of them), TC_STENCIL_PREWITT3 or TC_STENCIL_SOBEL3:
 *   E_x = (M_x * P0 + M_x * P1) / 2 with M_x the smoothing [1,1,1]/3 or
 *   [1,2,1]/4 across x times the centred difference [-1,0,1]/2 along x (E_y
 *   transposed), E_t = the 2-D smoothing s s^T applied to P1 - P0, at every
 *   pixel with a full 3x3 neighbourhood ((H_l-2)(W_l-2) estimates), centred at
 *   x = 2^l (j + 1/2) - W/2.  TC_STENCIL_ROBERTS is rejected (TC_EINVAL).
 * lowpass: TC_LOWPASS_NONE, or TC_LOWPASS_BINOMIAL3: after each 2x2 block mean
 *   the level is filtered by [1,2,1]/4 along rows and columns with clamped
 *   borders (level 0 is not filtered; level sizes are unchanged).
 * prev, next: 2-D U8, F16 or F32 frames of one shape (strided); every level
 * must hold at least 2x2 (cube) or 3x3 pixels (TC_ESHAPE otherwise).  ws: device
 * workspace of tc_ttc_variant_workspace_size bytes (TC_ENOMEM if smaller).
 * levels_out[levels], pick_out[1]: device memory.  Derivatives are FP32, G,
 * products and sums FP64 (deterministic order).  Launches only.
 * ------------------------------------------------------------------------ */
#define TC_LOWPASS_NONE 0
#define TC_LOWPASS_BINOMIAL3 1
int tc_ttc_variant_workspace_size(int64_t H, int64_t W, int32_t levels, int32_t stencil, int32_t lowpass,
                                  size_t* ws_bytes);
int tc_ttc_solve_variant(const tc_tensor* prev, const tc_tensor* next, int32_t levels, int32_t stencil,
                         int32_t lowpass, void* ws, size_t ws_bytes, tc_ttc_level* levels_out, tc_ttc_pick* pick_out,
                         void* stream);

/* Workspace bytes for tc_ttc_solve on an H x W pair with `levels` levels. */
int tc_ttc_workspace_size(int64_t H, int64_t W, int32_t levels, size_t* ws_bytes);
/* One frame pair (2-D U8 or F16 tensors of equal shape): levels_out[levels]
 * and pick_out[1] in device memory.  Launches only (no host copy). */
int tc_ttc_solve(const tc_tensor* prev, const tc_tensor* next, int32_t levels, void* ws, size_t ws_bytes,
                 tc_ttc_level* levels_out, tc_ttc_pick* pick_out, void* stream);

/* ------------------------------------------------------------------------
 * tc_ttc_solve without a workspace, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.
 *
 * Same arguments (minus ws), results and errors as tc_ttc_solve; the partial
 * sums go to a scratch array of TC_NOALLOC_SCRATCH_BYTES (4 MiB) held in the
 * library's device memory, one copy per GPU, kept until the process ends.  A
 * pair whose workspace (tc_ttc_workspace_size) exceeds that is rejected with
 * TC_ENOMEM before anything is launched (square frames up to 14448 x 14448
 * with 4 levels, 28912 x 28912 with one).  The first call on a device looks up the array's address on
 * the current device (the stream must belong to it); nothing is allocated or
 * freed, by this call or its kernels.  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (two streams, or two host threads)
 * race and must be ordered by the caller.  No part of the array needs to
 * start at zero (each call writes every partial it reads).  Launches only.
 * ------------------------------------------------------------------------ */
#define TC_NOALLOC_SCRATCH_BYTES (4u << 20)
int tc_ttc_solve_noalloc(const tc_tensor* prev, const tc_tensor* next, int32_t levels, tc_ttc_level* levels_out,
                         tc_ttc_pick* pick_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TTCCONV_H */
