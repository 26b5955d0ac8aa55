/*
 * tp.h -- C ABI of libtp.so, the MI355X (gfx950) filtered-backprojection hot path
 * for parallel-beam tomography (arXiv 2209.08450, "TomocuPy").
 *
 * Path: raw projections + dark/flat fields --(tp_normalize)--> sinogram
 *       --(tp_filter)--> ramp-filtered rows --(tp_backproject)--> slices,
 * fused as tp_fbp_chunk; tp_radon is the exact transpose of tp_backproject.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Device pointers are caller-owned; the library never frees or retains them
 *   beyond the call.  `stream` is a hipStream_t passed as void* (NULL = the
 *   null stream).  Every compute call only enqueues work on `stream` and
 *   returns; results are visible after the caller synchronises that stream.
 * - Arguments are validated on the host before anything is enqueued.  On a
 *   bad argument a call returns TP_EINVAL (or TP_EUNSUPPORTED for a valid but
 *   unimplemented choice), enqueues nothing, and tp_last_error() describes
 *   the problem.  A failed launch returns TP_EHIP.  No call aborts, exits or
 *   lets a C++ exception escape.
 * - Geometry: detector column j sits at detector coordinate j; the rotation
 *   axis is at `center` (in columns).  Voxel (ix, iy) of an N x N slice is
 *   centred at x = ix - floor(N/2), y = iy - floor(N/2) (ix is the fast,
 *   contiguous axis), and projects at angle theta to s = x cos + y sin + center.
 *   Detector rows (slices) are independent.
 * - Layouts (row-major, last index fastest):
 *     raw projections  uint16 [n_angles][rows][n_det]   (projection-major, as recorded)
 *     dark / flat      uint16 [frames][rows][n_det]
 *     sinogram, rows   [rows][n_angles][n_det]           (sinogram-major)
 *     volume           float  [rows][N][N]
 * - Hot calls (normalize/filter/backproject/radon/fbp_chunk) never allocate
 *   device memory once their tables exist (tp_plan_create builds the
 *   geometry and filter tables of a plan; tp_filter_prepare those of a
 *   standalone filter length), so they may be captured into a HIP graph.
 */
#ifndef TP_H
#define TP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TP_OK = 0,
    TP_EINVAL = -1,        /* invalid argument; nothing enqueued */
    TP_EUNSUPPORTED = -2,  /* valid request this build does not implement */
    TP_EHIP = -3,          /* a HIP runtime call or kernel launch failed */
    TP_ENOMEM = -4         /* device allocation failed (table building only) */
} tp_status;

/* Storage type of sinograms and filtered rows.  Arithmetic is FP32 for all. */
typedef enum { TP_F32 = 0, TP_F16 = 1, TP_BF16 = 2 } tp_dtype;

/* Row filter: the band-limited ramp |w| (w in cycles/pixel, |w| <= 1/2) times
 * a window W(x), x = 2|w| (the paper's filter choices, Section 2.4; Parzen is
 * its default and is used for every result of Section 3).  The paper gives no
 * formulas; the textbook windows are:
 *   TP_RAMP:   W = 1;
 *   TP_SHEPP:  W = sinc(x/2) = sin(pi x/2)/(pi x/2)  (taps 2/(pi^2 (1 - 4m^2)));
 *   TP_PARZEN: W = 1 - 6x^2 + 6x^3 for x <= 1/2, 2(1 - x)^3 for 1/2 < x <= 1. */
typedef enum { TP_RAMP = 0, TP_SHEPP = 1, TP_PARZEN = 2 } tp_filter_kind;

/* Scan geometry (paper Section 2.4: angles, rotation axis, detector width). */
typedef struct {
    int32_t n_angles;       /* N_theta >= 1 */
    int32_t n_det;          /* detector columns n >= 1 (filter length limit: n <= 8192) */
    int32_t n_vox;          /* reconstructed slice is n_vox x n_vox; 0 => n_det */
    double center;          /* rotation axis in detector columns (any value; rays off
                               the detector contribute zero) */
    const double* angles;   /* HOST pointer to n_angles radians, read during
                               tp_plan_create only */
} tp_geometry;

/* A plan owns device-side tables for one geometry on the device that is
 * current when it is created: FP32 (cos, sin) per angle and, per 32-voxel
 * tile edge, the detector coordinate of the tile origin computed in FP64 and
 * split into an integer and an FP32 fraction, plus the ramp filter's tables
 * for pad length 2^ceil(log2(2 n_det)).  Use a plan only on that device.
 *
 * Why a handle: the paper's reconstruction is configured once per scan (the
 * angles, rotation axis and detector width of Section 2.4) and then run chunk
 * after chunk (Section 2.3), with FFT plans built once and reused per chunk
 * (Section 2.2).  The plan is that once-per-scan state: its tables are built
 * here, outside any graph capture, and every chunk call reads them.
 *
 * tp_plan_create: g as above (angles read during the call only); *out
 * receives the plan.  Errors: TP_EINVAL (null pointers, non-positive sizes,
 * non-finite angles or centre, |center| > 1e6), TP_EUNSUPPORTED (pad length
 * above 16384 or n_vox above 32768), TP_ENOMEM / TP_EHIP from the device.
 * If tp_tune_load has loaded a table holding this device and shape, the
 * plan starts from the recorded backprojection tilings (else the defaults
 * below). */
typedef struct tp_plan tp_plan;

tp_status tp_plan_create(const tp_geometry* g, tp_plan** out);
/* Frees the plan's tables, including those built later on first use (the
 * Fourier path's per window and truncation radius, laminography's per tilt,
 * centre_v and slice count: about 2 MB each at 2048 angles x 2048 voxels).
 * Those are kept until this call, since graph-captured launches refer to
 * them; the caller must ensure no enqueued work still uses them. */
tp_status tp_plan_destroy(tp_plan* plan);

/* Tuning of the backprojection kernel for one storage type of its input
 * (results are bitwise identical for every legal choice: each slice always
 * sums its angles in order).
 *   slices_per_block in {1, 2, 4, 8, 16}: slices sharing one coordinate evaluation;
 *   angles_per_block in {8, 16, 32, 64}: angles staged in LDS per step;
 *   the staged block, angles x 48 bins x pitch (slices x 4 bytes, 2 for F16,
 *   plus 16 when that is 64 or more), must fit in 160 KiB.  Defaults: F16
 *   (16, 16); F32 and BF16 (16, 8). */
tp_status tp_plan_set_tuning(tp_plan* plan, tp_dtype storage, int32_t slices_per_block,
                             int32_t angles_per_block);
tp_status tp_plan_get_tuning(const tp_plan* plan, tp_dtype storage, int32_t* slices_per_block,
                             int32_t* angles_per_block);

/* Build and cache the filter tables of one pad length and window on the
 * current device (the paper builds its FFT plans once and runs them per
 * chunk, Section 2.2; the windows are the filter choices of Section 2.4), for
 * tp_filter / tp_fbp_chunk calls that will be graph-captured; a plan prepares
 * the ramp of its own pad length.  pad_len: power of two in [2, 16384].
 * Errors: TP_EINVAL (pad_len), TP_EUNSUPPORTED (kind), TP_ENOMEM / TP_EHIP. */
tp_status tp_filter_prepare(int32_t pad_len, tp_filter_kind kind);

/* Everything the hot calls of one plan need for one filter window and one
 * storage type, built before the first chunk (FFT plans created once and
 * executed per chunk, paper Section 2.2; the filter and 16-bit storage
 * choices of Section 2.4): the window's tables at the plan's pad length and
 * the dynamic-LDS limit of the backprojection kernel that the plan's current
 * tiling for `storage` selects.  After it, tp_fbp_chunk and tp_backproject
 * with that (kind, storage) allocate nothing and make no one-time runtime
 * call, so they may be graph-captured.  Call it again after
 * tp_plan_set_tuning.  The plan's device must be current.  Errors: TP_EINVAL
 * (null plan, bad storage, another device current), TP_EUNSUPPORTED (kind),
 * TP_ENOMEM / TP_EHIP from the device. */
tp_status tp_prepare(const tp_plan* plan, tp_filter_kind kind, tp_dtype storage);

/* Loads the autotuner's table of backprojection tilings (the tile parameters
 * of the backprojection; the paper's per-chunk kernels take their sizes from
 * the chunk and detector, Section 2.3) from a JSON file: an object mapping
 * "<device name>|<f32|f16|bf16>|na=<angles>|n=<columns>|N=<voxels>|rows=<rows>"
 * to objects whose "choice" member is [slices_per_block, angles_per_block]
 * (other members are ignored; several row counts of one shape keep the
 * largest).  Plans created afterwards on a matching device and shape start
 * from these tilings.  Tilings never change results (every legal tiling gives
 * bitwise-identical output), only speed.  json_path NULL clears the table.
 * Host only (no device call).  Errors: TP_EINVAL for an unreadable file,
 * malformed JSON, a malformed key or an illegal tiling; the previous table is
 * then kept. */
tp_status tp_tune_load(const char* json_path);
/* Host only: the tiling the loaded table holds for (device_name, storage,
 * n_angles, n_det, n_vox; n_vox 0 => n_det).  TP_EINVAL if none (or null
 * arguments). */
tp_status tp_tune_lookup(const char* device_name, tp_dtype storage, int32_t n_angles, int32_t n_det, int32_t n_vox,
                         int32_t* slices_per_block, int32_t* angles_per_block);

/* Releases what the library caches across plans: the filter tables of every
 * (device, pad length, window) on every device, and the tuning table.  Plans
 * point at those tables, so every plan must have been destroyed first
 * (TP_EINVAL otherwise, nothing freed), and no enqueued work may still read
 * them.  Later calls rebuild what they need.  Errors: TP_EINVAL (plans
 * alive), TP_EHIP (a device call failed; the cache is emptied regardless). */
tp_status tp_shutdown(void);

/* Host only, no device needed: the FP64 filter response the device tables are
 * rounded from, H[k] = sum_{m=-L/2}^{L/2-1} h[m] exp(-2 pi i k m / L), where
 * h[m] = integral over |w| <= 1/2 of |w| W(2|w|) exp(2 pi i w m) dw.
 * H: HOST array of pad_len doubles, written.  pad_len: power of two in
 * [2, 16384].  Errors: TP_EINVAL (null H, bad pad_len), TP_EUNSUPPORTED
 * (unknown kind). */
tp_status tp_filter_response(int32_t pad_len, tp_filter_kind kind, double* H);

/* --------------------------------------------------------------------------
 * Dark/flat correction and negative logarithm (paper Section 2.2):
 *   D = mean over frames of dark, F = mean over frames of flat   (per pixel)
 *   sino[r][a][j] = -ln( max( (P[a][r][j] - D) / max(F - D, 1), 1e-6 ) )
 * proj:  dev, element (a, r, j) at proj[a*proj_stride + r*n_det + j];
 *        proj_stride 0 => n_rows*n_det (contiguous).
 * dark/flat: dev, frame f row r at ptr[f*frame_stride + r*n_det]; frame_stride
 *        0 => n_rows*n_det.  n_dark, n_flat >= 1, each <= 256 (exact sums).
 * sino:  dev [n_rows][n_angles][n_det] of out_dtype (RNE rounding for F16/BF16).
 * workspace: dev, >= tp_normalize_workspace_bytes(n_rows, n_det) bytes,
 *        256-byte aligned; holds D and 1 / max(F - D, 1) between two kernels
 *        (the normaliser multiplies by the stored reciprocal).
 * ------------------------------------------------------------------------ */
size_t tp_normalize_workspace_bytes(int32_t n_rows, int32_t n_det);
tp_status tp_normalize(const uint16_t* proj, int64_t proj_stride,
                       const uint16_t* dark, int32_t n_dark,
                       const uint16_t* flat, int32_t n_flat, int64_t frame_stride,
                       int32_t n_angles, int32_t n_rows, int32_t n_det,
                       tp_dtype out_dtype, void* sino,
                       void* workspace, size_t workspace_bytes, void* stream);

/* --------------------------------------------------------------------------
 * tp_normalize without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same operation, arguments, layouts and results as
 * tp_normalize; D and 1/max(F - D, 1) live instead in a file-scope device
 * array of 2 x TP_NOALLOC_MAX_PIXELS floats (64 MiB), one per GPU, kept until
 * the process ends.  Its address is looked up on the first call on each
 * device (that device must be current); the call allocates nothing.
 * Limit: n_rows * n_det <= TP_NOALLOC_MAX_PIXELS (e.g. 2048 rows of a
 * 4096-column detector); larger calls return TP_EINVAL, enqueue nothing.
 * Every call on one GPU shares that array: calls that can overlap on one
 * device (different streams, or host threads without ordering) race and may
 * produce wrong sinograms.  Nothing in the array needs clearing: each call
 * writes every entry it reads.
 * ------------------------------------------------------------------------ */
#define TP_NOALLOC_MAX_PIXELS (8388608LL)
tp_status tp_normalize_noalloc(const uint16_t* proj, int64_t proj_stride,
                               const uint16_t* dark, int32_t n_dark,
                               const uint16_t* flat, int32_t n_flat, int64_t frame_stride,
                               int32_t n_angles, int32_t n_rows, int32_t n_det,
                               tp_dtype out_dtype, void* sino, void* stream);

/* --------------------------------------------------------------------------
 * Filter of detector rows by FFT (paper Section 2.2, padding per Section 3):
 * each row p[0..n) is padded to L by replicating its end values, with the data
 * at offset floor((L - n)/2); y = IFFT(H . FFT(u)), H = tp_filter_response of
 * (L, kind) (ramp: h[0] = 1/4, h[odd m] = -1/(pi^2 m^2)); q[j] = y[off + j].
 * sino: dev [n_lines][n_det] of in_dtype;  filt: dev [n_lines][n_det] of
 * out_dtype; filt may equal sino only when in_dtype == out_dtype (in place),
 * otherwise the ranges must not overlap.  pad_len 0 => 2^ceil(log2(2 n_det));
 * else a power of two with n_det <= pad_len <= 16384.
 * ------------------------------------------------------------------------ */
tp_status tp_filter(const void* sino, tp_dtype in_dtype, void* filt, tp_dtype out_dtype,
                    int64_t n_lines, int32_t n_det, int32_t pad_len, tp_filter_kind kind,
                    void* stream);

/* --------------------------------------------------------------------------
 * Backprojection with linear interpolation ("LineRec", paper Sections 2.2, 3):
 *   vol[r][iy][ix] (+)= scale * sum_a ( (1-w) Q(j0) + w Q(j0+1) ),
 *   s = x cos(theta_a) + y sin(theta_a) + center, j0 = floor(s), w = s - j0,
 *   Q(j) = filt[r][a][j] for 0 <= j < n_det, else 0.
 * FBP uses scale = pi / n_angles; the adjoint of tp_radon uses scale = 1.
 * filt: dev [n_rows][n_angles][n_det] of in_dtype.  vol: dev float
 * [n_rows][N][N]; accumulate 0 overwrites, 1 adds.  Arithmetic is FP32 with
 * the detector coordinate split into an FP64-derived integer part and an
 * FP32 offset below 64 columns.
 * ------------------------------------------------------------------------ */
tp_status tp_backproject(const tp_plan* plan, const void* filt, tp_dtype in_dtype,
                         int32_t n_rows, float scale, float* vol, int32_t accumulate,
                         void* stream);

/* --------------------------------------------------------------------------
 * Forward projection (the operator the paper's iterative reconstruction
 * methods need alongside the backprojector, Sections 1 and 5; not defined in
 * the paper, so it is read as the exact transpose of tp_backproject with
 * scale 1):
 *   sino[r][a][j] = sum over voxels of vol[r][iy][ix] * ( (1-w)[j0 == j] + w[j0+1 == j] )
 * with (j0, w) computed by the same FP32 formula as tp_backproject, so
 * <R x, y> = <x, R^T y> holds up to FP32 summation rounding.  Gather form
 * (each output summed by one thread in a fixed order): deterministic.  Inputs
 * are finite.
 * vol: dev float [n_rows][N][N];  sino: dev float [n_rows][n_angles][n_det],
 * overwritten; 1 <= n_rows <= 65535.
 * workspace: dev, 256-byte aligned, not overlapping vol or sino, at least
 * tp_radon_workspace_bytes(plan, n_rows) bytes (a transposed copy of vol, so
 * that angles whose rays run closer to the y axis also read contiguous
 * memory; 0 bytes, and workspace may be NULL, when every angle has
 * |cos| >= |sin|).  Its contents are scratch.
 * ------------------------------------------------------------------------ */
size_t tp_radon_workspace_bytes(const tp_plan* plan, int32_t n_rows);
tp_status tp_radon(const tp_plan* plan, const float* vol, int32_t n_rows, float* sino,
                   void* workspace, size_t workspace_bytes, void* stream);

/* --------------------------------------------------------------------------
 * One chunk of rows through the whole path (paper Section 2.2: dark/flat
 * correction, -log, filtering, backprojection; Section 2.3: the path runs per
 * chunk of detector rows): normalise -> filter -> backproject.
 *   vol = (pi / n_angles) R^T ( H * normalize(proj, dark, flat) )
 * The -log sinogram never leaves the chip: the filter kernel normalises raw
 * counts in registers, filters in FP32 and stores only the filtered rows, in
 * `storage` precision, into the workspace.  Inputs as for tp_normalize
 * (n_angles, n_det from the plan); vol: dev float [n_rows][N][N] (overwritten).
 * kind: filter window at the plan's pad length 2^ceil(log2(2 n_det)); windows
 * other than TP_RAMP build their tables on first use (tp_filter_prepare first
 * when the call will be graph-captured; else TP_EUNSUPPORTED during capture).
 * workspace: dev, 256-byte aligned, >= tp_fbp_workspace_bytes(plan, n_rows, storage).
 * ------------------------------------------------------------------------ */
size_t tp_fbp_workspace_bytes(const tp_plan* plan, int32_t n_rows, tp_dtype storage);
tp_status tp_fbp_chunk(const tp_plan* plan,
                       const uint16_t* proj, int64_t proj_stride,
                       const uint16_t* dark, int32_t n_dark,
                       const uint16_t* flat, int32_t n_flat, int64_t frame_stride,
                       int32_t n_rows, tp_filter_kind kind, tp_dtype storage,
                       void* workspace, size_t workspace_bytes,
                       float* vol, void* stream);

/* As tp_fbp_chunk, and additionally records caller-created hipEvent_t handles
 * (passed as void*) on `stream`: events[0] before the dark/flat means,
 * events[1] before the fused normalise+filter, events[2] before the
 * backprojection, events[3] after it.  Any entry may be NULL; events may be
 * NULL.  For per-stage timing (the paper's timeline breakdown, Section 2.3). */
tp_status tp_fbp_chunk_events(const tp_plan* plan,
                              const uint16_t* proj, int64_t proj_stride,
                              const uint16_t* dark, int32_t n_dark,
                              const uint16_t* flat, int32_t n_flat, int64_t frame_stride,
                              int32_t n_rows, tp_filter_kind kind, tp_dtype storage,
                              void* workspace, size_t workspace_bytes,
                              float* vol, void* stream, void* const* events);

/* As tp_fbp_chunk_events with a choice of output precision (paper, Section 3:
 * in the 16-bit mode the reconstructed volumes are stored in 16 bits, half
 * the memory and storage traffic).  vol_dtype TP_F32: vol is dev float
 * [n_rows][N][N], exactly tp_fbp_chunk_events.  TP_F16: vol is dev IEEE half
 * [n_rows][N][N], each voxel the FP32 result rounded once to nearest; needs
 * storage TP_F16 (TP_EUNSUPPORTED otherwise, nothing enqueued).  Other
 * vol_dtype values return TP_EINVAL. */
tp_status tp_fbp_chunk_out(const tp_plan* plan,
                           const uint16_t* proj, int64_t proj_stride,
                           const uint16_t* dark, int32_t n_dark,
                           const uint16_t* flat, int32_t n_flat, int64_t frame_stride,
                           int32_t n_rows, tp_filter_kind kind, tp_dtype storage,
                           void* workspace, size_t workspace_bytes,
                           tp_dtype vol_dtype, void* vol, void* stream, void* const* events);

/* --------------------------------------------------------------------------
 * Fourier-domain filtered backprojection ("FourierRec"; paper, Section 2.2:
 * the backprojection evaluated with exponential interpolation kernels in the
 * frequency domain, and Section 3, where it is the reference method).
 *
 * What it computes: for every slice,
 *   vol(x, y) = (pi / n_angles) * sum_a y_a(x cos(theta_a) + y sin(theta_a) + center + off)
 * where y_a is the real trigonometric interpolant of the padded, filtered row
 * (pad length L = 2^ceil(log2(2 n_det)), edge padding, data at
 * off = (L - n_det) / 2, both Nyquist terms at half weight): the same
 * normalise -> pad -> filter steps as tp_fbp_chunk, then band-limited instead
 * of linear interpolation along each ray (x = ix - N/2, y = iy - N/2).
 *
 * How: two slices travel as the real and imaginary parts of one complex row.
 * Each row's spectrum (FFT, times the filter response and the phase of the
 * axis position) is a line of samples through the origin of the 2-D frequency
 * plane (Fourier slice theorem).  A deterministic gather resamples those polar
 * samples onto a Cartesian grid of M = max(L, 2^ceil(log2(2N))) points per
 * side with a truncated Gaussian, a 2-D inverse FFT returns to image space and
 * division by the Gaussian's transform undoes the resampling kernel
 * (unequally spaced FFT with oversampling >= 2).  half_width is the Gaussian's
 * truncation radius in grid points (0 selects 6; 3..8 allowed): relative error
 * about exp(-2.2 half_width) of the exact sum, plus FP32 rounding.
 *
 * Inputs as for tp_fbp_chunk (raw counts, strides, dark/flat frames; n_angles,
 * n_det from the plan); vol: dev float [n_rows][N][N] (overwritten);
 * kind: filter window (tables built on first use, see tp_fourier_prepare).
 * workspace: dev, 256-byte aligned, not overlapping the inputs or vol.
 * tp_fourier_workspace_bytes(plan, n_rows) bytes process every pair of rows in
 * one pass; a smaller workspace (at least tp_fourier_workspace_bytes(plan, 2))
 * processes the rows in several passes of as many pairs as fit.  Its contents
 * are scratch.  Errors: TP_EINVAL for bad arguments (checked before any
 * launch), TP_EUNSUPPORTED for M > 16384 or tables missing during capture.
 * ------------------------------------------------------------------------ */
size_t tp_fourier_workspace_bytes(const tp_plan* plan, int32_t n_rows);
/* Builds the Fourier path's tables for (plan, kind, half_width) outside any
 * graph capture (they are otherwise built on first use). */
tp_status tp_fourier_prepare(const tp_plan* plan, tp_filter_kind kind, int32_t half_width);
tp_status tp_fourier_fbp_chunk(const tp_plan* plan,
                               const uint16_t* proj, int64_t proj_stride,
                               const uint16_t* dark, int32_t n_dark,
                               const uint16_t* flat, int32_t n_flat, int64_t frame_stride,
                               int32_t n_rows, tp_filter_kind kind, int32_t half_width,
                               void* workspace, size_t workspace_bytes,
                               float* vol, void* stream);
/* As tp_fourier_fbp_chunk, recording caller-created hipEvent_t handles on
 * `stream` for per-stage timing of the first pass: events[0] before the
 * dark/flat means, [1] before the spectra, [2] before the gather onto the
 * Cartesian grid, [3] before the inverse FFT along grid rows, [4] before the
 * inverse FFT along columns (with deconvolution), [5] after it (end of the
 * first pass).  Any entry may be NULL; events may be NULL. */
tp_status tp_fourier_fbp_chunk_events(const tp_plan* plan,
                                      const uint16_t* proj, int64_t proj_stride,
                                      const uint16_t* dark, int32_t n_dark,
                                      const uint16_t* flat, int32_t n_flat, int64_t frame_stride,
                                      int32_t n_rows, tp_filter_kind kind, int32_t half_width,
                                      void* workspace, size_t workspace_bytes,
                                      float* vol, void* stream, void* const* events);
/* As tp_fourier_fbp_chunk_events, with the slices stored as `vol_dtype`:
 * TP_F32, or TP_F16 for 16-bit volumes (paper, Section 3: FP16
 * reconstructions take half the memory; each voxel's FP32 result is rounded
 * once to nearest even, so the FP16 slices equal the FP32 slices rounded).
 * vol: device buffer of n_rows * N * N elements of that type.  Any other
 * vol_dtype fails with TP_EUNSUPPORTED before anything is enqueued. */
tp_status tp_fourier_fbp_chunk_out(const tp_plan* plan,
                                   const uint16_t* proj, int64_t proj_stride,
                                   const uint16_t* dark, int32_t n_dark,
                                   const uint16_t* flat, int32_t n_flat, int64_t frame_stride,
                                   int32_t n_rows, tp_filter_kind kind, int32_t half_width,
                                   void* workspace, size_t workspace_bytes,
                                   tp_dtype vol_dtype, void* vol, void* stream, void* const* events);

/* --------------------------------------------------------------------------
 * Log-polar-based filtered backprojection ("LpRec"; paper, Section 2.2: the
 * backprojection over equally spaced angles as a convolution in log-polar
 * coordinates, with spline interpolations to and from the log-polar grid in
 * the image domain; Section 3 lists it with cubic splines).  The paper gives
 * no grids or spline details; the reading built here:
 *
 * Target: the same sum as tp_fourier_fbp_chunk (every padded filtered row
 * read along each ray by its trigonometric interpolant, scale pi / n_angles),
 * approximated; the plan's angles must be theta_0 + a pi / n_angles.
 *
 * Method, per slice: (1) each padded filtered row is represented by a periodic
 * quintic B-spline through its trigonometric interpolant at half-sample
 * spacing (filter, spline prefilter and 2x resampling in one spectrum
 * multiply); (2) the angles are split into `spans` groups of n_span =
 * ceil(n_angles / spans) slots, each rotated to centre on zero, and the image
 * is moved by a0 = (1 + eps) R / cos(phi_max) (R: farthest voxel centre from
 * the axis + 2) so every ray offset s of an image point is >= eps R; with
 * x = e^rho (cos psi, sin psi) the span's backprojection is
 *   F(psi, rho) = dtheta sum_k G_k(rho + log cos(psi - phi_k)),
 *   G_k(sigma) = spline_a(e^sigma - a0 cos(phi_k) + center + off);
 * (3) G_k is sampled at sigma_j = sigma0 + j delta (Ns points, raised-cosine
 * taper at both ends); (4) the convolution is evaluated exactly for the
 * sampled band by FFTs: a shift over sigma, a linear convolution over the
 * fine angle psi_m = phi_0 + m dtheta / M; (5) quintic B-spline prefilters in
 * both transform domains give spline coefficients of F on the grid, which
 * (6) is evaluated at every voxel; the spans are summed.
 *
 * Accuracy: set by the grid resolution at the image's far side, os (grid
 * steps delta and dtheta / M at most 1 / (os (a0 + R)); the power-of-two
 * lengths usually give more), and by the row splines: at the defaults,
 * relative L2 against the exact sum of 9e-4 on the 12-bit 2048 x 2048
 * phantom scan (2048 angles) and 6e-4 on 256-column scans; see
 * tp_lprec_grid_query for the grid a call uses.
 *
 * Parameters: spans in 2..4 (0: 3), os in [0.25, 8] (0: 1.0), eps in
 * [0.05, 4] (0: 1.0).  Ns and NA (the angle FFT length) are powers of two
 * in [1024, 16384] and the pad length at most 8192, else TP_EUNSUPPORTED.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t spans, n_span;   /* spans and angle slots per span */
    int32_t Ns;              /* sigma samples (FFT length) */
    int32_t M;               /* fine angle steps per angle step */
    int32_t NA;              /* angle FFT length (>= rows + M (n_span - 1)) */
    int32_t D;               /* kernel length rows + M (n_span - 1) */
    int32_t rows, m_lo;      /* stored fine-angle rows m_lo .. m_lo + rows - 1 */
    int32_t d_lo;            /* first kernel index (m_lo - M (n_span - 1)) */
    int32_t j_lo, nj;        /* stored sigma window j_lo .. j_lo + nj - 1 */
    double os, eps;          /* the parameters used (defaults filled in) */
    double dtheta, R, phi0;  /* pi / n_angles, image radius, first slot offset */
    double a0, s_min, s_max; /* origin shift, least and largest ray offset */
    double delta, sigma0;    /* sigma step and origin */
    double dpsi;             /* dtheta / M */
} tp_lprec_grid;

/* Host only: the grid the sizing rule picks for n_angles x n_vox^2. */
tp_status tp_lprec_grid_query(int32_t n_angles, int32_t n_vox, int32_t spans, double os, double eps,
                              tp_lprec_grid* out);
/* Workspace for n_rows rows in one pass (0 on an unsupported plan).  A
 * smaller workspace (at least that of 2 rows) runs several passes. */
size_t tp_lprec_workspace_bytes(const tp_plan* plan, int32_t n_rows, int32_t spans, double os, double eps);
/* Builds the tables for (plan, kind, spans, os, eps) outside graph capture. */
tp_status tp_lprec_prepare(const tp_plan* plan, tp_filter_kind kind, int32_t spans, double os, double eps);
/* Inputs as for tp_fbp_chunk; vol: dev float [n_rows][N][N] (overwritten);
 * workspace: dev, 256-byte aligned, scratch.  Errors as above, TP_EINVAL for
 * bad arguments (checked before any launch). */
tp_status tp_lprec_fbp_chunk(const tp_plan* plan,
                             const uint16_t* proj, int64_t proj_stride,
                             const uint16_t* dark, int32_t n_dark,
                             const uint16_t* flat, int32_t n_flat, int64_t frame_stride,
                             int32_t n_rows, tp_filter_kind kind, int32_t spans, double os, double eps,
                             void* workspace, size_t workspace_bytes,
                             float* vol, void* stream);
/* As tp_lprec_fbp_chunk, recording caller-created hipEvent_t handles for the
 * first pass: [0] before the dark/flat means, [1] before the row splines,
 * [2] before the log-radial resampling and its FFT, [3] before the angle
 * convolution, [4] before the inverse sigma FFT, [5] before the evaluation at
 * the voxels, [6] after it.  Any entry may be NULL; events may be NULL. */
tp_status tp_lprec_fbp_chunk_events(const tp_plan* plan,
                                    const uint16_t* proj, int64_t proj_stride,
                                    const uint16_t* dark, int32_t n_dark,
                                    const uint16_t* flat, int32_t n_flat, int64_t frame_stride,
                                    int32_t n_rows, tp_filter_kind kind, int32_t spans, double os, double eps,
                                    void* workspace, size_t workspace_bytes,
                                    float* vol, void* stream, void* const* events);

/* --------------------------------------------------------------------------
 * Laminographic backprojection (paper, Section 2.2: the direct line-integral
 * backprojector is kept because it also serves laminography, where the
 * rotation axis is tilted with respect to the beam).  Geometry (a reading:
 * the paper does not define it): axis tilted by `tilt` = phi in (0, pi) from
 * the beam, phi = pi/2 being tomography; voxel (x, y, z) of the
 * [n_slices][N][N] volume (x = ix - N/2, y = iy - N/2, z = iz - n_slices/2)
 * is seen at detector column u = x cos + y sin + center (the plan's axis) and
 * row v = (-x sin + y cos) cos(phi) + z sin(phi) + center_v, and
 *   vol = scale * sum_a bilinear(filt_a, v, u),  zero off the detector.
 * filt: dev [n_angles][det_rows][n_det] in in_dtype (projections filtered
 * along detector rows, e.g. by tp_filter); vol: dev float [nz][N][N] receives
 * slices z0 .. z0 + nz - 1 (overwritten).  Tables are built on first use per
 * (tilt, center_v, n_slices) (tp_lamino_prepare first when the call will be
 * graph-captured; else TP_EUNSUPPORTED during capture).  TP_EINVAL for bad
 * arguments, checked before any launch.
 * ------------------------------------------------------------------------ */
tp_status tp_lamino_prepare(const tp_plan* plan, double tilt, double center_v, int32_t n_slices);
tp_status tp_lamino_backproject(const tp_plan* plan, const void* filt, tp_dtype in_dtype, int32_t det_rows,
                                double tilt, double center_v, int32_t n_slices, int32_t z0, int32_t nz,
                                float scale, float* vol, void* stream);

/* --------------------------------------------------------------------------
 * Storage reads and writes of the chunk pipeline (paper, Section 2.3: chunks
 * are read from the storage drive and reconstructed chunks written back by
 * their own threads, in parallel, overlapped with transfers and computation).
 * Host-only calls: plain host pointers (pinned or pageable), blocking, safe to
 * call from several threads at once on different buffers.  A failing call
 * returns TP_EINVAL with the reason in tp_io_last_error() (thread-local,
 * separate from tp_last_error); nothing is partially reported as success.
 * Files are raw little-endian arrays (they stand in for the paper's HDF5
 * datasets and TIFF slices).  When every file offset, length and the buffer
 * are 4096-byte aligned the file is opened with O_DIRECT (bypassing the page
 * cache), else buffered; buffers the kernel cannot pin for a direct transfer
 * (EFAULT, such as the GPU runtime's pinned host memory) go through per-thread
 * aligned bounce buffers, and filesystems that refuse direct transfers
 * (EINVAL) get buffered I/O.  n_threads: 1..64 threads issue the pieces.
 * ------------------------------------------------------------------------ */
/* Reads detector rows [z0, z1) of a projection-major file holding, after
 * header_bytes, [n_outer][n_rows][n_det] elements of elem_bytes each (n_outer
 * = angles, or dark/flat frames) into dst [n_outer][z1 - z0][n_det]: n_outer
 * pieces of (z1 - z0) * n_det elements. */
tp_status tp_io_read_rows(const char* path, int64_t header_bytes, int32_t n_outer, int32_t n_rows, int32_t n_det,
                          int32_t z0, int32_t z1, int32_t elem_bytes, void* dst, int32_t n_threads);
/* Writes n_slices slices of slice_bytes each from src to the file (which must
 * exist, see tp_io_create) at header_bytes + first_slice * slice_bytes: one
 * piece per slice.  Writeback of the range to the drive is started before
 * returning (not waited for), so a later flush finds little left to write. */
tp_status tp_io_write_slices(const char* path, int64_t header_bytes, int64_t first_slice, int32_t n_slices,
                             int64_t slice_bytes, const void* src, int32_t n_threads);
/* Creates (or truncates) the file and sets its size to `bytes`. */
tp_status tp_io_create(const char* path, int64_t bytes);
/* Thread-local description of the last failing tp_io_* call on this thread. */
const char* tp_io_last_error(void);

/* --------------------------------------------------------------------------
 * Measurement instruments for the roofline report (not part of the paper's
 * method): the rates a kernel of this library can reach on this device, as
 * the denominators beside the vendor peaks.
 * tp_peak_copy: copies `bytes` (a positive multiple of 16; both buffers dev,
 *   16-byte aligned, not overlapping) with 16-byte loads and stores on
 *   `stream`; time it with events to get the copy rate (2 x bytes moved).
 * tp_peak_valu: `blocks` work-groups of 256 threads each run 16 independent
 *   multiply-add chains of one instruction form for `iters` steps and store
 *   one float per thread to out (dev, blocks x 256 floats); *flop receives
 *   the flop count (2 per FMA, 4 per dot2).  Forms: TP_VALU_FMA_F32
 *   (v_fma_f32, VGPR operands), TP_VALU_FMA_F32_SGPR (one operand from a
 *   scalar register), TP_VALU_FMA_MIX_F16 (v_fma_mix_f32, an FP16 operand),
 *   TP_VALU_DOT2_F16 (v_dot2_f32_f16: two FP16 products into an FP32 sum).
 * tp_peak_fma: tp_peak_valu with TP_VALU_FMA_F32.
 * tp_peak_lds: `blocks` work-groups of 256 threads each issue 16 x iters
 *   conflict-free 16-byte LDS reads and store one word per thread to out
 *   (dev, blocks x 256 words); *bytes receives the bytes read.
 *   blocks in [1, 2^20], iters in [1, 2^24] for all of them.
 * Errors: TP_EINVAL for bad arguments (nothing enqueued), TP_EHIP.
 * ------------------------------------------------------------------------ */
#define TP_VALU_FMA_F32 0
#define TP_VALU_FMA_F32_SGPR 1
#define TP_VALU_FMA_MIX_F16 2
#define TP_VALU_DOT2_F16 3
tp_status tp_peak_copy(const void* src, void* dst, int64_t bytes, void* stream);
tp_status tp_peak_valu(int32_t form, float* out, int32_t blocks, int32_t iters, int64_t* flop, void* stream);
tp_status tp_peak_fma(float* out, int32_t blocks, int32_t iters, int64_t* flop, void* stream);
tp_status tp_peak_lds(uint32_t* out, int32_t blocks, int32_t iters, int64_t* bytes, void* stream);

/* Thread-local description of the last non-OK status returned on this thread. */
const char* tp_last_error(void);
/* Library version string. */
const char* tp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TP_H */
