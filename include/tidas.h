/*
 * tidas.h -- C ABI of the MI355X (gfx950) tiDAS library.
 *
 * Implements the hot path of "tiDAS: a time invariant approximation of the
 * Delay and Sum algorithm for biomedical ultrasound PSF reconstructions"
 * (arXiv 2507.15464):
 *
 *   das_beamform         exact Delay-and-Sum (Sec. 2, eqn:appF)
 *   tidas_build_kernels  per-depth-row kernels derived from DAS
 *                        (Sec. 2.2 eq:PSF; Sec. 2.3 eqn:tDAS, eqn:theta;
 *                        Sec. 3.1-3.2 FWHM correction window)
 *   tidas_apply          the time-invariant line model (Sec. 2.4, eqn:line_conv)
 *   tidas_adjoint        its transpose
 *   tidas_simulate_rf    Born-approximation RF synthesis (Sec. 2, eqn:SRX),
 *                        the input generator of the path
 *   tidas_apply_ex, tidas_adjoint_ex, tidas_deconvolve, tidas_operator_norm_sq
 *                        fused forms and the Tikhonov deconvolution built on
 *                        the line model (abstract; Sec. 1; Sec. 4)
 *   tidas_prepare, tidas_apply_prepared, tidas_adjoint_prepared
 *                        the line model with its kernel bank converted once
 *                        into the form its matrix-core kernels read
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units are SI (m, s, Hz, rad).  Device arrays are float32, C-order and
 * contiguous.  Layouts:
 *   RF channel data   [B][A][C][T]  frames x angles x elements x samples
 *   images, maps      [B][Z][X]     frames x depth rows x lateral columns
 *   kernel bank       [Z][K]        one K-tap kernel per OUTPUT depth row
 * Geometry: element n (0 <= n < C) sits at x_n = (n - (C-1)/2) * pitch,
 * depth 0; pixel (i, j) sits at (x0 + j dx, z0 + i dz).  A plane wave of angle
 * a reaches (x, z) at (x sin a + z cos a) / c; RF sample k is taken at time
 * t0 + k / fs.  Receive apodization is a Hann window of half width
 * z / (2 F) (weight 0.5 (1 + cos(pi d / (z / 2F))), zero outside).  Channel
 * data are read with linear interpolation, zero outside [0, T-1].
 *
 * Pointers marked DEV are device pointers owned by the caller; HOST pointers
 * are read during the call only.  The library keeps no pointer after a call
 * returns.  Work is enqueued on `stream` (a hipStream_t; NULL = the legacy
 * default stream) and is asynchronous: execution errors surface at the
 * caller's next synchronisation.  Outputs must not overlap inputs.
 *
 * Device scratch.  Entry points that need scratch memory take (workspace,
 * workspace_bytes) and have a size query named <entry point>_workspace_bytes:
 * workspace DEV, 256-byte aligned, at least the queried size, owned by the
 * caller and not retained; or workspace = NULL with workspace_bytes = 0, in
 * which case the call allocates the scratch stream-ordered (hipMallocAsync /
 * hipFreeAsync on `stream`; TIDAS_ENOMEM possible).  With a caller workspace
 * no call below allocates device memory, except the unprepared line-model
 * calls (tidas_apply, tidas_adjoint and their _ex forms), which keep their
 * signatures and convert the bank into band images in a stream-ordered
 * temporary; tidas_prepare with a caller buffer (tidas_prepared_bytes) and
 * tidas_apply_noalloc are their allocation-free forms.
 *
 * Return codes: 0 = OK; TIDAS_EINVAL (-1) invalid argument, checked before
 * any work is enqueued, in which case nothing is written; TIDAS_EHIP (-2) a
 * HIP runtime or launch error; TIDAS_ENOMEM (-3) a temporary device
 * allocation failed; TIDAS_EUNSUPPORTED (-4) a valid request this build does
 * not handle.  tidas_last_error() returns a thread-local message describing
 * the last non-zero status of the calling thread.
 */
#ifndef TIDAS_H
#define TIDAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TIDAS_OK 0
#define TIDAS_EINVAL (-1)
#define TIDAS_EHIP (-2)
#define TIDAS_ENOMEM (-3)
#define TIDAS_EUNSUPPORTED (-4)

#define TIDAS_MODE_EXACT 0 /* kernel = DAS PSF of a unit scatterer (Sec. 2.2 eq:PSF)        */
#define TIDAS_MODE_PAPER 1 /* kernel = theta x fixed-delay response (Sec. 2.3, eqn:theta)  */
#define TIDAS_MODE_LINE 2  /* kernel = theta x fixed-delay line on the RF (Sec. 2.4)       */
#define TIDAS_MODE_LATERAL 3 /* lateral profile of the row's PSF (separable 2-D extension) */

/* Linear array: element count C >= 1, pitch > 0, speed of sound c > 0 (Sec. 2.1). */
typedef struct tidas_array {
    int32_t n_elem;
    double pitch;
    double c;
} tidas_array;

/* Transmit and sampling.  n_angles >= 1 plane waves whose angles (radians)
 * are read from the HOST array `angles`; sampling rate fs > 0; time of RF
 * sample 0, t0; pulse p(t) = exp(-t^2 / (2 s^2)) cos(2 pi fc t) for
 * |t| <= 4 s, zero beyond, with the envelope FWHM 2 sqrt(2 ln 2) s spanning
 * `cycles` periods of fc (fc > 0, cycles > 0).  The pulse is used only where
 * echoes are synthesised (kernel building, RF synthesis). */
typedef struct tidas_tx {
    int32_t n_angles;
    const double* angles; /* HOST [n_angles] */
    double fs;
    double t0;
    double fc;
    double cycles;
} tidas_tx;

/* Receive: F-number of the Hann aperture (> 0). */
typedef struct tidas_rx {
    double fnumber;
} tidas_rx;

/* Image grid: nz >= 1 depth rows, nx >= 1 lateral columns; pixel (i, j) at
 * (x0 + j dx, z0 + i dz); dz > 0 and dx > 0. */
typedef struct tidas_grid {
    int32_t nz, nx;
    double z0, dz, x0, dx;
} tidas_grid;

/* Library version string (static storage). */
const char* tidas_version(void);

/* Message for the last non-zero status returned on the calling thread. */
const char* tidas_last_error(void);

/*
 * Debug builds (the library compiled with -DTIDAS_DEBUG: libtidas_debug.so)
 * check inside the kernels what the derivations promise and record failures
 * as bits, without trapping:
 *   TIDAS_DBG_NONFINITE_IN  a non-finite input (RF sample, map value or
 *                           kernel tap) entered DAS or the line model
 *   TIDAS_DBG_STUDY_SPAN    the single-point study skipped a non-zero echo
 *                           sample (its support table was wrong)
 * tidas_debug_flags synchronises the device and writes the OR of the bits
 * recorded since the last reset to *flags (HOST); reset != 0 clears them.
 * A release build writes 0 and returns TIDAS_EUNSUPPORTED.
 */
#define TIDAS_DBG_NONFINITE_IN 2u
#define TIDAS_DBG_STUDY_SPAN 4u
int32_t tidas_debug_flags(uint32_t* flags, int32_t reset);

/*
 * Exact Delay-and-Sum, Sec. 2 eqn:appF: every pixel gets its own delay
 * profile.  For each frame b
 *   image[b][i][j] = sum_a sum_n w(x_j - x_n, z_i) *
 *                    L(rf[b][a][n], (tau_n(x_j, z_i; a) - t0) * fs)
 * with tau_n = (x sin a + z cos a) / c + sqrt((x - x_n)^2 + z^2) / c, the
 * angles coherently compounded.  rf is DEV [n_frames][A][C][n_samples],
 * image DEV [n_frames][nz][nx] (overwritten).  n_frames >= 1,
 * n_samples >= 2.  All frames share one geometry.  workspace DEV (device
 * scratch convention above): with eight or more frames of one angle or of
 * eleven the call reads the RF through a frame-interleaved copy, four frames
 * per 16-byte load ([ceil(n_frames / 4)][A][C][n_samples][4] floats);
 * das_beamform_workspace_bytes gives its size (0: no scratch needed).
 */
int32_t das_beamform(const tidas_array* array, const tidas_tx* tx, const tidas_rx* rx,
                     const tidas_grid* grid, const float* rf, int32_t n_samples,
                     int32_t n_frames, float* image, void* workspace, size_t workspace_bytes,
                     void* stream);
size_t das_beamform_workspace_bytes(int32_t n_angles, int32_t n_elem, int32_t n_samples, int32_t n_frames);

/*
 * The paper's time-invariant beamformer applied to the RF (Sec. 2.3 eqn:tDAS:
 * the delays of one point serve a whole line; Sec. 2.4 eqn:line_conv: fixed
 * parameters along the line, scaled by the weights Theta).  Row i reads every
 * element with the receive law frozen at the depth of its reference row
 * r = ref_row[i], in every column:
 *   image[b][i][j] = theta[i] * sum_a sum_n w(x_j - x_n, z_r) *
 *       L(rf[b][a][n], (tau_tx(x_j, z_i; a) + z_i / c - D_n(x_j, z_r) - t0) * fs),
 *   D_n(x, z) = (z - sqrt((x - x_n)^2 + z^2)) / c   (eqn:delay at lateral x),
 * w and L as in das_beamform.  With ref_row[i] = i and theta = 1 this is
 * das_beamform.  ref_row DEV int32 [nz] or NULL (each row its own
 * reference); entries are clamped into [0, nz).  theta DEV [nz] or NULL
 * (ones), e.g. the weights tidas_build_kernels returns in paper mode.  rf,
 * image and n_frames as in das_beamform; image must not alias an input.
 * Waves whose rows share one reference (one law per neighbourhood or per
 * line) evaluate the law once per element for all their rows.  workspace
 * as in das_beamform (eight or more frames of one plane wave read the RF
 * through the same interleaved copy); tidas_beamform_workspace_bytes gives
 * its size.
 */
int32_t tidas_beamform(const tidas_array* array, const tidas_tx* tx, const tidas_rx* rx,
                       const tidas_grid* grid, const float* rf, int32_t n_samples, int32_t n_frames,
                       const int32_t* ref_row, const float* theta, float* image, void* workspace,
                       size_t workspace_bytes, void* stream);
size_t tidas_beamform_workspace_bytes(int32_t n_angles, int32_t n_elem, int32_t n_samples, int32_t n_frames);

/*
 * Per-depth-row kernel bank of the line model, evaluated on the centre line
 * x = 0 from the echo of a unit scatterer (computed analytically in float64
 * over n_samples RF samples, zero outside the record).  h = (K-1)/2.
 *
 * mode TIDAS_MODE_EXACT (Sec. 2.2, eq:PSF):
 *   kernels[i][m+h] = DAS of a unit scatterer at (0, z_i), evaluated at the
 *   pixel (0, z_i + m dz); the grid's x0, dx and nx are not used.
 * mode TIDAS_MODE_PAPER (Sec. 2.3 eqn:tDAS, eqn:diff, eqn:theta; Sec. 3.1-3.2):
 *   the receive delays and weights are frozen at the depth of row
 *   r = ref_row[i] (ref_row = NULL: r = i).  With the fixed-delay line
 *   F_r[S](z) = sum_a sum_n w(-x_n, z_r) L(S[a][n], (t(z; a) - D_n(z_r) - t0) fs),
 *   t(z; a) = z cos(a) / c + z / c and D_n the delay law of eqn:delay,
 *     h_r[m]   = F_r[unit echo at z_r](z_r + m dz),
 *     W_r      = FWHM of the envelope (|analytic signal|, DFT zero-padded to
 *                the first power of two >= twice the length) of the DAS PSF
 *                of the unit echo at z_r on the fine axis z_r + q c/(2 fs),
 *                |q| <= ceil(8 s fs),
 *     theta_i  = sum a b / sum a^2 over the fine points z_i + q c/(2 fs),
 *                |q| <= floor(W_r / (2 c/(2 fs))), with a = F_r[unit echo at
 *                z_i] and b = DAS of the unit echo at z_i (first line of
 *                eqn:theta, time domain), 0 when sum a^2 = 0,
 *     kernels[i][m+h] = theta_i * h_r[m].
 * mode TIDAS_MODE_LINE (Sec. 2.4, eqn:line_conv: Theta times the fixed-delay
 *   beamformer of the RF, expressed on the reflectivity by Born linearity):
 *   theta_i, r and W_r as in paper mode, and
 *     kernels[i][m+h] = theta_i * F_r[unit echo at z_i - m dz](z_i).
 * mode TIDAS_MODE_LATERAL (the separable 2-D extension; a 2-D model is future
 *   work in the conclusion, Sec. 4): the lateral profile through the scatterer
 *   of the same unit echo, normalised at the scatterer,
 *     kernels[i][m+h] = DAS(unit echo at (0, z_i)) at (m dx, z_i) / its value at (0, z_i)
 *   (0 when that value is 0), for tidas_apply_lateral.
 * kernels DEV [nz][K]; theta DEV [nz] or NULL (exact and lateral modes write 1).
 * ref_row HOST [nz] with 0 <= ref_row[i] < nz, or NULL.  K odd, >= 1.
 * Paper and line modes need scratch (reference responses and the row ->
 * reference map, tidas_build_kernels_workspace_bytes; exact and lateral modes
 * need none) and upload the map from a host copy that a host function queued
 * on `stream` releases: the call does not wait for the stream.
 */
size_t tidas_build_kernels_workspace_bytes(int32_t nz, int32_t K, int32_t mode);
int32_t tidas_build_kernels(const tidas_array* array, const tidas_tx* tx, const tidas_rx* rx,
                            const tidas_grid* grid, int32_t n_samples, int32_t K, int32_t mode,
                            const int32_t* ref_row, float* kernels, float* theta, void* workspace,
                            size_t workspace_bytes, void* stream);

/*
 * The tiDAS line model, Sec. 2.4 eqn:line_conv, applied to a reflectivity
 * map along depth in every lateral column, kernel chosen by the output row:
 *   image[b][i][j] = sum_{m=-h..h} kernels[i][m+h] * refl[b][i-m][j],
 * refl taken as zero outside [0, Z).  kernels DEV [Z][K], K odd >= 1;
 * refl, image DEV [B][Z][X], B, Z, X >= 1.
 */
int32_t tidas_apply(const float* kernels, int32_t K, const float* refl, int32_t B, int32_t Z,
                    int32_t X, float* image, void* stream);

/*
 * Transpose of tidas_apply:
 *   refl_bar[b][s][j] = sum_{m=-h..h} kernels[s+m][m+h] * image_bar[b][s+m][j],
 * terms with s + m outside [0, Z) dropped.  Shapes as tidas_apply.
 */
int32_t tidas_adjoint(const float* kernels, int32_t K, const float* image_bar, int32_t B,
                      int32_t Z, int32_t X, float* refl_bar, void* stream);

/*
 * Fused forms of the line model and its adjoint (same operators as above):
 *   image    = alpha * A(refl)       + beta * base
 *   refl_bar = alpha * A^T(image_bar) + beta * base
 * base is DEV [B][Z][X] or NULL (then beta is ignored).  base may alias the
 * output (each element is read before it is written) but neither may alias
 * the operator's input.  alpha, beta finite.  These carry the residual and
 * the update of gradient-based reconstruction through the line model without
 * extra passes over memory.
 */
int32_t tidas_apply_ex(const float* kernels, int32_t K, const float* refl, int32_t B, int32_t Z, int32_t X,
                       float alpha, float beta, const float* base, float* image, void* stream);
int32_t tidas_adjoint_ex(const float* kernels, int32_t K, const float* image_bar, int32_t B, int32_t Z, int32_t X,
                         float alpha, float beta, const float* base, float* refl_bar, void* stream);

/*
 * Lateral pass of the separable 2-D extension: after the line model's depth
 * pass, each depth row is convolved along the lateral axis with its own
 * kernel (tidas_build_kernels, TIDAS_MODE_LATERAL):
 *   out[b][i][j] = sum_{m=-h..h} kernels_x[i][m+h] * in[b][i][j-m],
 * in taken as zero outside [0, X).  kernels_x DEV [Z][K], K odd, 1 <= K <= 1535;
 * in, out DEV [B][Z][X], out must not alias an input.  With exact depth
 * kernels the two passes reproduce DAS along an on-axis scatterer's own row.
 */
int32_t tidas_apply_lateral(const float* kernels_x, int32_t K, const float* in, int32_t B, int32_t Z, int32_t X,
                            float* out, void* stream);

/*
 * Gradient of the line model in its kernels.  The model (Sec. 2.4,
 * eqn:line_conv) is linear in the per-row kernels, which the conclusion
 * (Sec. 4) treats as learnable weights; for image_bar = dL/d(image):
 *   kernels_bar[i][m+h] = sum_b sum_j image_bar[b][i][j] * refl[b][i-m][j],
 * refl taken as zero outside [0, Z) (those taps get 0).  refl, image_bar DEV
 * [B][Z][X]; kernels_bar DEV [Z][K], overwritten, must not alias an input.
 * K odd >= 1; B, Z, X >= 1; EUNSUPPORTED when (Z + 2 K + 512) X 4 bytes
 * reach 2^31.  Matrix-core products: split-bfloat16 (each value cut exactly
 * into three bfloat16 parts, six products, float32 sums) when X % 4 == 0 and
 * both inputs are 16-byte aligned, float32 otherwise; partial sums over
 * fixed ranges of (frame, column) added in double in a fixed order (bit-
 * reproducible on one device type); the workspace holds the partial sums
 * (tidas_kernel_grad_workspace_bytes, for the current device: about 2 x
 * compute units x 128 Z K / ceil(Z / 128) bytes).
 * Non-finite inputs: the float32 kernel propagates Inf and NaN as float32
 * arithmetic does; on the split-bfloat16 path an infinite input gives NaN
 * (its parts are Inf - Inf).
 */
size_t tidas_kernel_grad_workspace_bytes(int32_t K, int32_t B, int32_t Z, int32_t X);
int32_t tidas_kernel_grad(int32_t K, const float* refl, const float* image_bar, int32_t B, int32_t Z, int32_t X,
                          float* kernels_bar, void* workspace, size_t workspace_bytes, void* stream);

/*
 * Which kernel tidas_kernel_grad runs for X columns and the two input
 * pointers (a diagnostic, enqueues nothing, pointers are not dereferenced):
 * TIDAS_KGRAD_SPLIT_BF16 when X % 4 == 0 and both pointers are 16-byte
 * aligned, TIDAS_KGRAD_FP32 otherwise; TIDAS_EINVAL for X < 1.
 */
#define TIDAS_KGRAD_SPLIT_BF16 1
#define TIDAS_KGRAD_FP32 2
int32_t tidas_kernel_grad_kernel(int32_t X, const void* refl, const void* image_bar);

/*
 * tidas_apply for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same operator, kernels and results (bit for bit) as tidas_apply, with the
 * band images the split-bfloat16 kernels read prepared in a library-owned
 * device array of TIDAS_NOALLOC_SCRATCH_BYTES (8 MiB) on each GPU, held until
 * the process ends, instead of a temporary allocation; no call allocates or
 * frees anything.  The array belongs to the current device (which must be
 * the stream's device); every call on one GPU shares it, so calls that
 * overlap on one GPU (concurrent streams or threads) race and must be
 * serialised by the caller.  A bank whose band images exceed the array (one
 * operator mode at K taps and Z rows: about 1.1 MB per 1024 rows at K = 129)
 * returns TIDAS_EUNSUPPORTED before anything is enqueued; other arguments
 * as tidas_apply.
 */
#define TIDAS_NOALLOC_SCRATCH_BYTES ((size_t)8 << 20)
int32_t tidas_apply_noalloc(const float* kernels, int32_t K, const float* refl, int32_t B, int32_t Z, int32_t X,
                            float* image, void* stream);

/*
 * Which line-model kernel tidas_apply / tidas_adjoint (and their fused and
 * prepared forms) run for K taps, B frames of Z x X (16-byte aligned
 * buffers): a diagnostic for callers and tests, enqueues nothing.
 *   TIDAS_LINE_FOUR_BLOCK  split-bfloat16 matrix cores, 128 x 256 tiles (K <= 161,
 *                          at least one tile per compute unit)
 *   TIDAS_LINE_TWO_BLOCK   split-bfloat16 matrix cores, 64 x 256 tiles (K <= 321)
 *   TIDAS_LINE_FP32_MATRIX float32 matrix cores (larger K)
 *   TIDAS_LINE_VECTOR      vector ALU
 * TIDAS_EINVAL for even or non-positive K or sizes, TIDAS_EUNSUPPORTED when no
 * kernel takes K.  The four forms give the same results to float32 rounding;
 * the two split-bfloat16 tiles give the same bits.
 */
#define TIDAS_LINE_FOUR_BLOCK 1
#define TIDAS_LINE_TWO_BLOCK 2
#define TIDAS_LINE_FP32_MATRIX 3
#define TIDAS_LINE_VECTOR 4
int32_t tidas_line_kernel(int32_t K, int32_t B, int32_t Z, int32_t X);

/*
 * Prepared kernel bank.  The line model's kernels (Sec. 2.4, eqn:line_conv)
 * depend on the geometry only, so a caller that applies one bank to many
 * frames can convert it once: tidas_prepare writes, for the forward operator
 * and its adjoint, the banded matrix of every 64-row tile of the bank and (K
 * <= 161) of every 128-row tile, with each float32 tap cut exactly into three
 * bfloat16 parts (the forms the split-bfloat16 matrix-core kernels of
 * tidas_apply read; tidas_apply builds the one it needs in a temporary buffer
 * on every call).  tidas_apply_prepared and tidas_adjoint_prepared then give
 * the same results as tidas_apply_ex and tidas_adjoint_ex on that bank, bit
 * for bit (every line-model kernel sums a row's taps in the same order).
 *
 * tidas_prepared_bytes: size of the prepared form for K taps and Z rows; 0
 * when K is even, < 1, or too large for the matrix-core tiles (K > 321).
 * tidas_prepare: kernels DEV [Z][K] -> prepared DEV, >= tidas_prepared_bytes
 * bytes, 16-byte aligned, owned by the caller, valid until the bank changes.
 * TIDAS_EUNSUPPORTED when tidas_prepared_bytes is 0 for a valid odd K.
 * tidas_apply_prepared / tidas_adjoint_prepared: the fused forms above with
 * the prepared bank of the same K and Z in place of the kernels;
 * TIDAS_EUNSUPPORTED when the frame is too large for the matrix-core tiles
 * (then use tidas_apply_ex / tidas_adjoint_ex).
 */
size_t tidas_prepared_bytes(int32_t K, int32_t Z);
int32_t tidas_prepare(const float* kernels, int32_t K, int32_t Z, void* prepared, size_t bytes, void* stream);
int32_t tidas_apply_prepared(const void* prepared, int32_t K, const float* refl, int32_t B, int32_t Z, int32_t X,
                             float alpha, float beta, const float* base, float* image, void* stream);
int32_t tidas_adjoint_prepared(const void* prepared, int32_t K, const float* image_bar, int32_t B, int32_t Z,
                               int32_t X, float alpha, float beta, const float* base, float* refl_bar, void* stream);

/*
 * Tikhonov-regularised deconvolution through the line model (the paper
 * proposes the convolutional form as a foundation for deconvolution: abstract,
 * Sec. 1, Sec. 4).  Minimises 1/2 ||A r - y||^2 + lam/2 ||r||^2 by `iters`
 * gradient steps from r_0 = 0:
 *   r_{t+1} = r_t - eta (A^T (A r_t - y) + lam r_t),
 * computed as r_{t+1} = N r_t + c with the step operator N = (1 - eta lam) I
 * - eta A^T A (a bank of 2K - 1 taps built in float64) and c = eta A^T y,
 * r_1 = c: one launch per step, or, when the bank of N^2 (4K - 3 taps) fits
 * the split-bfloat16 tile (K <= 81), one launch per two steps
 * (r_{t+2} = N^2 r_t + N c + c); kernels too long for the tile (K > 161)
 * take two fused launches per step as written.  y, r, work DEV [B][Z][X],
 * pairwise distinct; r receives the result, work is scratch.  lam >= 0,
 * eta > 0 (for convergence eta < 2 / (||A||^2 + lam); see
 * tidas_operator_norm_sq).  The step operators, their band images and c (and
 * N c + c) live in the workspace (tidas_deconvolve_workspace_bytes: about 2
 * frames plus 60 Z K bytes; 0 for kernels too long for the tile).
 */
size_t tidas_deconvolve_workspace_bytes(int32_t K, int32_t B, int32_t Z, int32_t X);
int32_t tidas_deconvolve(const float* kernels, int32_t K, const float* y, int32_t B, int32_t Z, int32_t X,
                         float lam, float eta, int32_t iters, float* r, float* work, void* workspace,
                         size_t workspace_bytes, void* stream);

/*
 * Largest eigenvalue of A^T A for the Z x Z column operator of the line model
 * (= squared largest singular value), by `iters` steps of power iteration
 * from the all-ones vector.  work DEV with room for 3 Z + 4 floats; the
 * workspace holds the bank's band images (tidas_operator_norm_sq_workspace_bytes,
 * 0 when the bank takes the float32 path); *out is a HOST double, written
 * after the call synchronises the stream (the result is a host value).
 */
size_t tidas_operator_norm_sq_workspace_bytes(int32_t K, int32_t Z);
int32_t tidas_operator_norm_sq(const float* kernels, int32_t K, int32_t Z, int32_t iters, float* work, double* out,
                               void* workspace, size_t workspace_bytes, void* stream);

/*
 * Ragged batches.  Each frame has its own image grid and buffers; the array,
 * transmit and receive set-up (and, for the line model, K) are shared.  One
 * persistent launch covers the tiles of all frames (tiles are dealt to the
 * 8 XCDs in contiguous chunks so a frame's data stays in one L2).
 */
typedef struct tidas_frame {
    tidas_grid grid;       /* this frame's image grid */
    const float* rf;       /* DEV [A][C][n_samples]: DAS input (ignored by the line model) */
    const float* kernels;  /* DEV [nz][K]: line-model kernel bank (ignored by DAS) */
    const float* in;       /* DEV [nz][nx]: line-model reflectivity (ignored by DAS) */
    float* out;            /* DEV [nz][nx]: output image */
} tidas_frame;

/* Launch-shape variants the batch entry points accept (chosen by an autotuner):
 *   DAS:        variant v -> wave tile of 1 x 64, 2 x 32 or 4 x 16 pixels
 *               (depth x lateral, v / 6), 4 or 8 waves per workgroup stacked
 *               in depth (v & 1), and 2, 4 or 8 workgroups per compute unit
 *               ((v % 6) >> 1)
 *   line model: variants 0-5: persistent workgroups over the 64-row tiles of
 *               all frames (split-bfloat16 two-block tile: 1, 2, 3, 4, 6 or 8
 *               workgroups per compute unit; for K > 321 the float32 matrix
 *               tile: prefetch depth 4, 8 or 16 steps (v % 3) and 2 or 4
 *               workgroups per compute unit (v / 3));
 *               variant 6 (TIDAS_APPLY_BATCH_FOUR_BLOCK, K <= 161): the band
 *               images of every frame prepared once in the workspace, then
 *               one workgroup per 128-row tile of every frame on the
 *               four-block tile, walking the frame's 256-column tiles; it
 *               needs tidas_apply_batch_workspace_bytes and a 256-byte
 *               aligned workspace.  Every variant gives the same bits. */
#define TIDAS_DAS_BATCH_VARIANTS 18
#define TIDAS_APPLY_BATCH_VARIANTS 7
#define TIDAS_APPLY_BATCH_FOUR_BLOCK 6

/* Device workspace (bytes) a batch of n_frames needs: the frame table. */
size_t tidas_batch_workspace_bytes(int32_t n_frames);

/* Device workspace (bytes) tidas_apply_batch needs for these frames and K
 * with any variant: the frame table and, when K <= 161, the four-block band
 * images of every frame (one operator mode: about 1 MB per 1024 rows at
 * K = 129, 0.8 MB at K = 65).  0 for invalid arguments. */
size_t tidas_apply_batch_workspace_bytes(const tidas_frame* frames, int32_t n_frames, int32_t K);

/*
 * DAS of a ragged batch: frames[f].out = DAS(frames[f].rf) on frames[f].grid
 * (definition of das_beamform).  frames HOST [n_frames] (validated, then
 * copied into `workspace`, DEV, 16-byte aligned, >= tidas_batch_workspace_bytes
 * bytes; the copy is staged before the call returns).  variant in
 * [0, TIDAS_DAS_BATCH_VARIANTS).
 */
int32_t das_beamform_batch(const tidas_array* array, const tidas_tx* tx, const tidas_rx* rx, int32_t n_samples,
                           const tidas_frame* frames, int32_t n_frames, void* workspace, size_t workspace_bytes,
                           int32_t variant, void* stream);

/*
 * Line model of a ragged batch: frames[f].out = A_f(frames[f].in) with the
 * frame's own [nz][K] bank (definition of tidas_apply).  Workspace of
 * tidas_apply_batch_workspace_bytes (variants 0-5 need only the table,
 * tidas_batch_workspace_bytes); variant in [0, TIDAS_APPLY_BATCH_VARIANTS).  TIDAS_EUNSUPPORTED if a frame
 * exceeds the tile path's limits (then use tidas_apply per frame).
 */
int32_t tidas_apply_batch(const tidas_frame* frames, int32_t n_frames, int32_t K, void* workspace,
                          size_t workspace_bytes, int32_t variant, void* stream);

/*
 * The four-block batch (variant TIDAS_APPLY_BATCH_FOUR_BLOCK) split in two,
 * for a batch applied many times (the banks depend on the geometry only):
 * tidas_apply_batch_prepare uploads the frame table and prepares every
 * frame's band images in `workspace` (tidas_apply_batch_workspace_bytes
 * bytes, 256-byte aligned); tidas_apply_batch_prepared then runs the line
 * model of the batch with one launch and no upload.  The workspace then
 * holds the frames' bank, input and output pointers: the prepared call must
 * get the same frames (it recomputes only the launch size from them) and the
 * banks must be unchanged since the prepare call; the outputs are the same
 * bits as tidas_apply_batch.  EUNSUPPORTED for K > 161 or more than 65535
 * tiles of 128 rows.
 */
int32_t tidas_apply_batch_prepare(const tidas_frame* frames, int32_t n_frames, int32_t K, void* workspace,
                                  size_t workspace_bytes, void* stream);
int32_t tidas_apply_batch_prepared(const tidas_frame* frames, int32_t n_frames, int32_t K, const void* workspace,
                                   size_t workspace_bytes, void* stream);

/*
 * Exact-mode row kernels for independent draws (the surrogate's training data
 * and error judge).  Row i uses params[i] = (depth z, F-number, plane-wave
 * angle [rad], centre frequency [Hz]) (DEV float64 [N][4]), one transmit
 * angle, the pulse of `cycles` periods at that frequency and n_samples
 * samples at fs from t0:
 *   out[i][m+h] = DAS, at (0, z + m dz), of a unit scatterer at (0, z)
 * (the exact mode of tidas_build_kernels for that single row).  scale DEV [N]
 * or NULL receives s_i = max(sum_n w(-x_n, z), 1), the row's aperture weight
 * sum, against which the surrogate learns normalised kernels; with
 * normalise != 0, out[i] is divided by s_i.
 */
int32_t tidas_kernels_at(const tidas_array* array, double fs, double t0, double cycles, int32_t n_samples, double dz,
                         const double* params, int32_t N, int32_t K, int32_t normalise, float* out, float* scale,
                         void* stream);

/*
 * Kernel-surrogate MLP (an extension; the paper treats the weights Theta as
 * learned, Sec. 4): widths[5] = {4, 256, 256, 256, K}, GELU after the first
 * three linear layers.  Parameters are one flat float32 buffer (DEV [P],
 * P = tidas_mlp_param_count): for each layer W [out][in] then b [out]; a
 * bfloat16 copy (DEV uint16 [P], round to nearest even) feeds the matrix
 * cores.  Inputs x DEV float32 [rows][4] are normalised features in [-1, 1]
 * (tidas_mlp_features).  Every GEMM takes bfloat16 operands and accumulates
 * in float32; activations and back-propagated gradients are rounded to
 * bfloat16 before each GEMM.  `work` is DEV, 256-byte aligned, of
 * tidas_mlp_workspace_bytes(widths, N) bytes.
 */
int64_t tidas_mlp_param_count(const int32_t* widths /* HOST [5] */);
size_t tidas_mlp_workspace_bytes(const int32_t* widths /* HOST [5] */, int32_t N);

/* x [N][4] = 2 (params - lo) / (hi - lo) - 1 per column; params DEV float64
 * [N][4]; lo, hi HOST [4] with lo < hi. */
int32_t tidas_mlp_features(const double* params, int32_t N, const double* lo, const double* hi, float* x,
                           void* stream);

/* params16 = bfloat16(params), n values. */
int32_t tidas_mlp_to_bf16(const float* params, int64_t n, uint16_t* params16, void* stream);

/* y [N][K] = MLP(x), each row times scale[row] (scale DEV [N] or NULL). */
int32_t tidas_mlp_forward(const int32_t* widths, const uint16_t* params16, const float* params, const float* x,
                          int32_t N, const float* scale, float* y, void* work, size_t work_bytes, void* stream);

/* One training step on N rows gathered from the dataset (x DEV [n_rows][4],
 * target DEV [n_rows][K]) through idx (DEV int32 [N], values clamped to
 * [0, n_rows); NULL = rows 0..N-1): forward, loss = mean (y - target)^2
 * written to *loss (DEV float), and the gradient of the loss with respect to
 * every parameter written to grad (DEV float32 [P]). */
int32_t tidas_mlp_train_step(const int32_t* widths, const uint16_t* params16, const float* params, const float* x,
                             const float* target, int32_t n_rows, const int32_t* idx, int32_t N, float* grad,
                             float* loss, void* work, size_t work_bytes, void* stream);

/* Adam (bias-corrected, step >= 1) on the float32 master parameters with
 * moments m, v (DEV [P]); refreshes the bfloat16 copy. */
int32_t tidas_mlp_adam(const int32_t* widths, float* params, const float* grad, float* m, float* v,
                       uint16_t* params16, float lr, float beta1, float beta2, float eps, int32_t step, void* stream);

/*
 * Error measure for reports and for the surrogate's error judge:
 * out[0] = sum (a - b)^2, out[1] = sum b^2 over n float32 values (DEV a, b),
 * accumulated in float64; work DEV double [2]; out HOST double [2], written
 * after the call synchronises the stream.
 */
int32_t tidas_sq_norms(const float* a, const float* b, int64_t n, double* work, double* out, void* stream);

/*
 * Born-approximation RF synthesis, Sec. 2 eqn:SRX with linear superposition:
 *   rf[a][n][k] = sum_s amp[s] * p(t0 + k/fs - tau_n(x_s, z_s; a))
 * evaluated in float64, accumulated exactly in 64-bit fixed point (2^e units
 * per unit amplitude, n_scat max|amp| 2^e < 2^61: each term carries an
 * absolute error below 2^-(e+1)) and rounded once to float32.  The integer sum
 * does not depend on the order of the additions, so the record is the same
 * bits on every call.  scat is DEV [n_scat][3] float64 rows (x, z,
 * amplitude); rf DEV [A][C][n_samples] (overwritten).  n_scat >= 0.  The
 * workspace holds the accumulator (tidas_simulate_rf_workspace_bytes:
 * A*C*n_samples + 1 eight-byte values).
 */
size_t tidas_simulate_rf_workspace_bytes(int32_t n_angles, int32_t n_elem, int32_t n_samples);
int32_t tidas_simulate_rf(const tidas_array* array, const tidas_tx* tx, const double* scat,
                          int32_t n_scat, int32_t n_samples, float* rf, void* workspace, size_t workspace_bytes,
                          void* stream);

/*
 * The paper's single-point study (Sec. 3.1-3.3), float64 throughout.  An
 * unsteered beam focused on the probe axis (Sec. 2.1) at the depth of point
 * focal_index of the axial points z_s = z_first + s z_step (s < P =
 * n_points, Sec. 3.1: one point is the transmit focus): the n_tx centremost
 * elements fire at T_m = (z_f - sqrt(x_m^2 + z_f^2)) / c, unit weights (see
 * tidas_kossoff_tx_count for the aperture of Sec. 3.1).  For a unit
 * scatterer at every point s its echo, sampled on the record of n_samples
 * samples (tx: fs, t0, fc, cycles; its angle list must be the single angle
 * 0), is beamformed on the probe axis at the depths z_s + q dzf, dzf =
 * c / (2 fs), |q| <= line_half: by DAS (transmit arrival z / c, dynamic
 * receive law, Hann aperture of F-number rx->fnumber) giving b_s, and, for
 * the delay curve of every point r, by the time-invariant line (receive
 * delays D_n(z_r) of eqn:delay and the aperture of depth z_r for every
 * depth, Sec. 2.3 eqn:tDAS) giving a_rs.  Outputs, DEV float64 [P][P] with
 * entry [r][s]:
 *   theta      = sum_B a b / sum_B a^2 (0 when sum_B a^2 = 0)  (eqn:theta, line 1)
 *   err_local  = ||theta a - b||^2 over B / ||b||^2 over B    (Sec. 3.3, near the peak)
 *   err_global = ||theta a - b||^2 / ||b||^2 over the line     (Sec. 3.3, whole signal)
 * (errors 0 where ||b|| = 0), with the window B: |q| <= floor(W / (2 dzf)),
 * W the FWHM of the envelope of the focal point's DAS line measured on
 * |q| <= ceil(8 sigma fs) (Sec. 3.1-3.2); window DEV double [1] receives W in
 * metres (or NULL).  stats DEV float64 [P][4] (or NULL): per point s the
 * envelope peak of b_s, that of theta[focal][s] a_{focal,s}, and the two
 * envelopes' FWHMs in metres, all on |q| <= stats_half <= 511 (Sec. 3.2).
 * workspace DEV of at least tidas_point_study_workspace_bytes(C, P,
 * n_samples, line_half) bytes (echoes [P][C][n_samples] float64, their
 * supports, the DAS lines).  EINVAL: invalid descriptors, a steered or
 * multi-angle tx, n_tx outside [1, C] or with C - n_tx odd, n_samples < 2,
 * P < 1, z_first <= 0, z_step <= 0 when P > 1, focal_index outside [0, P),
 * line_half < 0, stats_half outside [0, 511] with stats, null or overlapping
 * outputs, a null or short workspace.  EUNSUPPORTED: C > 512, P > 65535, or
 * a pulse longer than the 1023-sample FWHM axis.
 */
size_t tidas_point_study_workspace_bytes(int32_t n_elem, int32_t n_points, int32_t n_samples, int32_t line_half);
int32_t tidas_point_study(const tidas_array* array, const tidas_tx* tx, const tidas_rx* rx, int32_t n_tx,
                          int32_t n_samples, int32_t n_points, double z_first, double z_step, int32_t focal_index,
                          int32_t line_half, int32_t stats_half, double* theta, double* err_local,
                          double* err_global, double* stats, double* window, void* workspace,
                          size_t workspace_bytes, void* stream);

/*
 * Transmit aperture of the single-point study (Sec. 3.1: Kossoff's
 * criterion with parameter `ratio`, 0.6 in the paper), read as the width D
 * whose near-field length D^2 / (4 lambda) puts the focus z_focus at `ratio`
 * of it: D = sqrt(4 lambda z_focus / ratio), lambda = c / fc.  Returns the
 * element count nearest D / pitch with the parity of n_elem (a set symmetric
 * about the probe centre), clamped to [1 (odd n_elem) or 2, n_elem]; or
 * TIDAS_EINVAL.  Host arithmetic only.
 */
int32_t tidas_kossoff_tx_count(const tidas_array* array, double fc, double z_focus, double ratio);

#ifdef __cplusplus
}
#endif

#endif /* TIDAS_H */
