/*
 * pxst.h -- C interface of libpxst, the gfx950 (MI355X) implementation of the
 * data-parallel reconstruction loop of Ptychographic X-ray Speckle Tracking.
 *
 * The paper (speckle-tracking: a software suite for PXST) states the problem as
 * frames I[n, i, j], a white-field W[i, j], a pixel mask M[i, j], a pixel map
 * u[2, i, j] (reference-plane coordinates sampled on the detector grid) and sample
 * translations dx[n, 2], related by the discrete forward model of Sec. 2.1, Eq. 3:
 *
 *     I[n, i, j] ~ W[i, j] * I_ref[u[0, i, j] - dx[n, 0], u[1, i, j] - dx[n, 1]].
 *
 * Conventions used by every call:
 *   - axis 0 = detector slow scan ("ss", x, i); axis 1 = fast scan ("fs", y, j);
 *   - all arrays are C row-major;
 *   - the reference index of detector pixel (i, j) in frame n is
 *     u[:, i, j] - dx[n] - origin, with the integer origin of pxst_geom
 *     (the paper leaves the reference origin free; an integer keeps every
 *     fraction in u and dx);
 *   - units are reference pixels throughout;
 *   - a reference pixel is valid where its weight sum wsum > 0; lookups use the
 *     masked bilinear interpolation of Sec. 4 (unknown or out-of-grid corners are
 *     dropped and the remaining weights renormalised).
 *
 * Memory: every array pointer below is a DEVICE pointer owned by the caller.  The
 * library never allocates device memory: scratch space comes from the caller's
 * workspace (`ws`, `ws_bytes`), sized by pxst_workspace_bytes().  Host structs are
 * read only during the call.  Pointers must be aligned to their element size and
 * the workspace to 256 bytes.
 *
 * Execution: every call validates its arguments on the host first (no GPU work
 * is enqueued when validation fails, so nothing is written), then enqueues its
 * kernels on `stream` and returns without synchronising.  Results are valid once
 * the stream has been synchronised.  Calls that share a workspace must be ordered
 * on one stream.
 *
 * Errors: 0 on success, a negative PXST_E* code otherwise; pxst_last_error()
 * returns a thread-local message describing the last failure of this thread.
 */
#ifndef PXST_H
#define PXST_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PXST_ABI_VERSION 3

#define PXST_OK 0
#define PXST_EINVAL (-1)       /* null pointer, bad size or misaligned pointer        */
#define PXST_EWORKSPACE (-2)   /* workspace missing or smaller than required         */
#define PXST_EUNSUPPORTED (-3) /* valid but outside the implemented limits           */
#define PXST_EHIP (-4)         /* HIP runtime or launch failure                       */

/* Implemented limits: search half-widths 0..15 for the pixel map, 0..2 for
 * translations; at most 2^24 - 1 detector pixels per frame; reference at most
 * 16384 x 16384. */
#define PXST_MAX_PM_RADIUS 15
#define PXST_MAX_TR_RADIUS 2
#define PXST_MAX_FRAC_STEPS 15

/* Scan geometry. */
typedef struct {
    int32_t n_frames;          /* N >= 1                                            */
    int32_t det_ss, det_fs;    /* H, W: detector shape (slow scan, fast scan)       */
    int32_t ref_ss, ref_fs;    /* Rs, Rf: reference shape                           */
    int32_t org_ss, org_fs;    /* integer origin of the reference grid              */
} pxst_geom;

/* Search window: integer offsets k in [-r, r] per axis, step 1 (the searches of
 * Sec. 2.2.2 and Sec. 2.2.3 cover a fixed window around the current value).  refine != 0 adds the 3x3
 * paraboloid sub-pixel offset around the integer minimum. */
typedef struct {
    int32_t r_ss, r_fs;
    int32_t refine;
} pxst_window;

/* One scan: frames [N][H][W] uint16 photon counts, white-field [H][W] float32,
 * mask [H][W] uint8 (1 = good pixel, 0 = excluded), all device memory. */
typedef struct {
    const uint16_t* frames;
    const float* white;
    const uint8_t* mask;
    pxst_geom geom;
} pxst_scan;

/* Arithmetic of the reference update (Sec. 2.2.1), for the precision study:
 *   PXST_REF_EXACT  every term rounded to a power-of-two quantum (about 1e-9 of the
 *                   largest term) and summed exactly in float64; the reference is
 *                   stored as float32.  The default.
 *   PXST_REF_FP32   float32 numerator with compensated sums over frames, float64
 *                   weight sums; stored as float32.
 *   PXST_REF_BF16   as PXST_REF_EXACT, then every reference value rounded to the
 *                   nearest bfloat16 (ties to even); all later lookups see bfloat16
 *                   values (kept in float32 arrays). */
#define PXST_REF_EXACT 0
#define PXST_REF_FP32 1
#define PXST_REF_BF16 2

/* Main-loop options (Sec. 2.2): n_iter iterations of (i) reference update,
 * (ii) pixel-map update with window `pm`, then its regularisation when pm_sigma > 0
 * or pm_integrate != 0 (see pxst_regularise_pixel_map), (iii) translation update
 * with window `tr` when update_dx != 0, (iv) total error; ref_mode selects the
 * arithmetic of every reference update of the loop (PXST_REF_*).  pm_sigma: finite,
 * 0 <= pm_sigma with int(4 pm_sigma + 0.5) <= 256; pm_integrate: 0 or 1. */
typedef struct {
    int32_t n_iter;
    pxst_window pm;
    int32_t update_dx;
    pxst_window tr;
    int32_t ref_mode;
    float pm_sigma;
    int32_t pm_integrate;
} pxst_solve_opts;

/* Workspace bytes that every entry point below needs for this geometry and these
 * windows (opts may be NULL: reference update and error only).  With
 * opts->pm_integrate != 0 the workspace also holds the buffers of the map
 * integration (two H x W and the H x H and W x W float64 matrices), which
 * pxst_regularise_pixel_map with integrate != 0 requires.  Returns 0 and sets the
 * last error when the arguments are invalid. */
size_t pxst_workspace_bytes(const pxst_geom* geom, const pxst_solve_opts* opts);

/*
 * Reference update -- Sec. 2.2.1 with the bilinear splat of Sec. 4.
 *   ref[p]  = sum_{n,i,j} w_p M W I[n,i,j] / sum_{n,i,j} w_p M W^2
 *   wsum[p] = sum_{n,i,j} w_p M W^2
 * where w_p is the bilinear weight of reference pixel p for the point
 * u[:, i, j] - dx[n] - origin.  ref = 0 where wsum == 0.
 *   u    [2][H][W] float32 (in)      dx   [N][2] float32 (in)
 *   ref  [Rs][Rf]  float32 (out)     wsum [Rs][Rf] float64 (out)
 * Arithmetic PXST_REF_EXACT: numerator and weight terms rounded to power-of-two
 * quanta and summed exactly in float64, so the result is the same bits whatever the
 * order of the additions (deterministic).  pxst_update_reference_ex selects the
 * arithmetic (PXST_REF_*; EINVAL for another value).
 */
int pxst_update_reference(const pxst_scan* scan, const float* u, const float* dx,
                          float* ref, double* wsum, void* ws, size_t ws_bytes,
                          hipStream_t stream);
int pxst_update_reference_ex(const pxst_scan* scan, const float* u, const float* dx,
                             int32_t ref_mode, float* ref, double* wsum, void* ws,
                             size_t ws_bytes, hipStream_t stream);

/*
 * Pixel-map update -- Sec. 2.2.2 (brute-force search, normalised error, argmin,
 * optional quadratic refinement).  For every good pixel: c = round-half-up(u_in);
 * for each candidate c + k, k in the window (slow-scan offset outer, fast-scan
 * inner), over the frames whose lookup at c + k - dx[n] - origin is valid:
 *   err = sum (I - W g)^2,  var = sum (I - W)^2,  E = err / var
 * (E = 0 when var = err = 0 with a valid frame; +inf when no frame is valid or
 * var = 0 < err).  The first minimum is taken; with refine, the least-squares
 * paraboloid through the 3x3 errors around it adds an offset clamped to +-0.5
 * (only for an interior minimum with finite neighbours; a 3-point parabola when
 * one half-width is 0).
 *   ref [Rs][Rf] float32, wsum [Rs][Rf] float64, dx [N][2], u_in [2][H][W] (in)
 *   u_out [2][H][W] (out, may equal u_in)
 *   err_min [H][W] float32 (out, optional), argmin [H][W] int32 (out, optional):
 *   linear candidate index (k_ss + r_ss) * (2 r_fs + 1) + (k_fs + r_fs), or -1
 *   (and err_min = +inf, u unchanged) for bad pixels and pixels with no finite
 *   candidate.
 * Lookups are interpolated in float32.  For windows whose per-tile error table fits
 * the LDS (up to 21 x 21 candidates at 121 frames), the frame sums run as an exact
 * int8 contraction of the counts with a fixed-point reference (rounding 2^-22 of the
 * largest reference value) combined in float64; otherwise float32 compensated sums.
 */
int pxst_update_pixel_map(const pxst_scan* scan, const float* ref, const double* wsum,
                          const float* dx, const float* u_in, pxst_window window,
                          float* u_out, float* err_min, int32_t* argmin,
                          void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Pixel-map search on a fine grid -- Sec. 2.2.2: the error evaluated at non-integer
 * positions through the interpolation of Sec. 4, in place of the paraboloid.
 * For each good pixel the candidates are c + m / steps per axis, c = round-half-up(u_in),
 * m in [-(r steps + (steps-1)/2), r steps + (steps-1)/2] with r the window radius of
 * that axis (window.refine is ignored: no paraboloid); the error of a candidate is the
 * normalised error of pxst_update_pixel_map with every lookup at
 * (c + m/steps) - dx[n] - origin.  The first minimum in fine-grid order (slow axis
 * outer) is taken:
 *   u_out   [2][H][W] float32  c + m/steps at the minimum (u_in where none; may be u_in)
 *   err_min [H][W]    float32  its normalised error (+inf where none), may be NULL
 *   argmin  [H][W]    int32    fine index m0' * n1 + m1', m' = m + r steps + (steps-1)/2,
 *                              n1 = 2 (r_fs steps + (steps-1)/2) + 1; -1 where none; may be NULL
 * steps: odd, 1 <= steps <= PXST_MAX_FRAC_STEPS (PXST_EINVAL / PXST_EUNSUPPORTED).
 * Cost: steps^2 integer searches (the fine classes are integer searches with the
 * translations moved by -q/steps).  Same workspace and errors as pxst_update_pixel_map.
 */
int pxst_update_pixel_map_fractional(const pxst_scan* scan, const float* ref, const double* wsum,
                                     const float* dx, const float* u_in, pxst_window window,
                                     int32_t steps, float* u_out, float* err_min, int32_t* argmin,
                                     void* workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * Split-half analysis -- Sec. 2.3 (additional analysis): every pixel of every frame
 * belongs to one of two halves of the data set; a pixel map is searched from each half
 * against the same reference, and the per-axis differences of the two maps are
 * histogrammed as an estimate of the uncertainty.
 *   half   [N][H][W] uint8 (in)  0: the term belongs to half A, 1: to half B (the
 *                                 caller draws the assignment)
 *   u_a, u_b [2][H][W] float32 (out)  the search of pxst_update_pixel_map (window,
 *                                 refine) over the terms of half A / B only; pixels
 *                                 without a result keep u_in.  Must not alias u_in
 *                                 or each other.
 *   hist   [2][nbins] int32 (out, may be NULL)  per axis, counts of u_a - u_b over the
 *                                 good pixels with a result in both halves, in nbins
 *                                 equal bins over [-hist_range, hist_range] (the last
 *                                 bin includes its upper edge, values outside are not
 *                                 counted)
 * hist_range finite > 0 and 1 <= nbins <= 65536 when hist is given (PXST_EINVAL).
 * The halves give every pixel its own subset of frames, so this search runs on the
 * vector ALUs (no matrix-core contraction).  Same workspace as pxst_update_pixel_map.
 */
int pxst_split_half_pixel_map(const pxst_scan* scan, const float* ref, const double* wsum,
                              const float* dx, const float* u_in, pxst_window window,
                              const uint8_t* half, float* u_a, float* u_b, float hist_range,
                              int32_t nbins, int32_t* hist, void* workspace,
                              size_t workspace_bytes, hipStream_t stream);

/*
 * Defocus by registration -- Sec. 2.1 (fit_defocus_registration): a reference image is
 * built (Sec. 2.2.1, exact arithmetic) from the map of every candidate magnification,
 * and the candidate whose reference has the greatest contrast is chosen.
 *   scales  [n_cand][2] float32, HOST memory (in)  per-axis scale factors s of the
 *                       linear map u = c + s (x - c) of a magnification change on the
 *                       fixed reference grid (scan geometry), x the detector pixel
 *   centre_ss, centre_fs  the fixed point c; NaN: the detector centre ((H-1)/2, (W-1)/2)
 *   dx      [N][2] float32 (in)
 *   contrast [n_cand] float64 (out)  variance / mean^2 of the reference pixels with a
 *                       positive weight sum (0 when there are none)
 *   best    [1] int32 (out, may be NULL)  index of the first maximum of contrast
 * n_cand >= 1 and finite scales (PXST_EINVAL).  Uses the reference-update part of the
 * workspace; candidates run one after the other on `stream`.
 */
int pxst_defocus_sweep(const pxst_scan* scan, const float* dx, const float* scales, int32_t n_cand,
                       float centre_ss, float centre_fs, double* contrast, int32_t* best,
                       void* workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * Translation update -- Sec. 2.2.3.  For frame n and integer shift s in the
 * window, the candidate translation is dx_in[n] + s and its error integrates over
 * the good pixels with a valid lookup at u - (dx_in[n] + s) - origin:
 *   E_n(s) = sum (I - W g)^2 / sum (I - W)^2
 * with the same empty / zero-variance rules, first-minimum order and refinement
 * as the pixel map.  Frames with no finite candidate keep dx_in[n] (argmin -1).
 *   u [2][H][W], dx_in [N][2] (in); dx_out [N][2] (out, may equal dx_in)
 *   err_min [N] float32 (optional), argmin [N] int32 (optional)
 */
int pxst_update_translations(const pxst_scan* scan, const float* ref, const double* wsum,
                             const float* u, const float* dx_in, pxst_window window,
                             float* dx_out, float* err_min, int32_t* argmin,
                             void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Figures of merit -- Sec. 2.2.4 with the integrand of Eq. 2.
 *   sigma2[i,j]  = (1/N) sum_n M (I - W)^2
 *   eps[n,i,j]   = M (I - W g)^2 / sigma2  (valid lookup at u - dx[n] - origin and
 *                  sigma2 > 0; else 0)
 *   pixel_err [H][W] float32 = sum_n eps       (optional)
 *   frame_err [N] float64   = sum_{i,j} eps    (optional)
 *   total     [1] float64   = sum eps          (required)
 *   ref_err   [Rs][Rf] float32 (optional) = sum w_p M eps / sum w_p M, the error
 *                  mapped to the reference plane with the splat of Sec. 2.2.1
 * Pixel sums use compensated float32; frame and total sums are float64 and
 * reduced in a fixed order.
 */
int pxst_error(const pxst_scan* scan, const float* ref, const double* wsum, const float* u,
               const float* dx, float* pixel_err, double* frame_err, double* total,
               float* ref_err, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Figures of merit without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Computes what pxst_error computes for pixel_err, frame_err and total,
 * with the same kernels, bit for bit; the reference-plane error is not offered.
 * Scratch (the reference with its validity, sigma^2 and the partial sums:
 * 4 Rs Rf + 4 H W + 8 N ceil(H W / 256) + 8 N bytes, each section rounded up to 256)
 * comes from a fixed device array of PXST_NOALLOC_SCRATCH_BYTES (32 MiB) inside the
 * library, one copy per GPU it runs on, held until the process ends.  Geometries
 * that need more return PXST_EUNSUPPORTED before any GPU work.  The call allocates
 * nothing and needs no clearing between calls.  All calls on one GPU share its array:
 * calls that overlap on one GPU (other streams, other threads) race and must be
 * ordered by the caller.  Arguments, layout and the other errors as pxst_error.
 */
#define PXST_NOALLOC_SCRATCH_BYTES (32u << 20)
int pxst_error_noalloc(const pxst_scan* scan, const float* ref, const double* wsum, const float* u,
                       const float* dx, float* pixel_err, double* frame_err, double* total,
                       hipStream_t stream);

/*
 * Pixel-map regularisation -- Sec. 2.2.2, closing paragraphs: optionally a Gaussian
 * filter of the map ("sigma"), then optionally the irrotational constraint
 * ("integrate": the map is replaced by the gradient of its least-squares potential).
 *   filter     each component convolved along both axes with exp(-k^2/(2 sigma^2)),
 *              |k| <= int(4 sigma + 0.5), normalised to unit sum; the nearest pixel
 *              is repeated outside the detector; sigma = 0: no filter
 *   integrate  Phi minimises sum (Phi[i+1,j]-Phi[i,j]-(u0[i,j]+u0[i+1,j])/2)^2
 *              + sum (Phi[i,j+1]-Phi[i,j]-(u1[i,j]+u1[i,j+1])/2)^2 over all pixels
 *              (solved exactly: the normal equations are diagonal in the DCT-II
 *              basis); u becomes the gradient of Phi by central differences,
 *              second-order one-sided at the edges (first order along an axis of two
 *              pixels; an axis of one pixel keeps its component)
 * The filter runs first, then the integration.
 *   u_in  [2][H][W] float32 (in)     u_out [2][H][W] float32 (out; may equal u_in)
 * sigma: finite, >= 0, int(4 sigma + 0.5) <= 256 (else PXST_EINVAL /
 * PXST_EUNSUPPORTED); integrate: 0 or 1.  The workspace must come from
 * pxst_workspace_bytes with opts->pm_integrate = 1 when integrate = 1
 * (PXST_EWORKSPACE otherwise).  Ordered on `stream`; allocates nothing (the DCT
 * products run in the library's own kernels, the transform matrices generated on
 * the fly).
 */
int pxst_regularise_pixel_map(const pxst_geom* geom, const float* u_in, float* u_out, float sigma,
                              int32_t integrate, void* workspace, size_t workspace_bytes,
                              hipStream_t stream);

/*
 * Main loop -- Sec. 2.2.  For k = 0..n_iter-1:
 *   (ref, wsum) <- reference update from (u, dx)
 *   u           <- pixel-map update with opts->pm
 *   dx          <- translation update with opts->tr (if opts->update_dx)
 *   err_hist[k] <- total error of (ref, u, dx)
 * then a final reference update from the last (u, dx).
 *   u [2][H][W], dx [N][2]: in/out.  ref [Rs][Rf], wsum [Rs][Rf]: out.
 *   err_hist [n_iter] float64: out (optional).
 * Everything is ordered on `stream` without host synchronisation: iteration k's
 * error pass runs on a library-internal second stream of the device (created on first
 * use, default priority, kept until the process ends) while iteration k + 1 updates
 * the reference, and `stream` waits for it before the search of iteration k + 1 and
 * before the call's last work, so work enqueued on `stream` afterwards sees every
 * output.  Concurrent calls on one device are enqueued one after the other.  Since
 * the whole state is in the caller's buffers, calling again continues the iteration.
 */
int pxst_solve(const pxst_scan* scan, const pxst_solve_opts* opts, float* u, float* dx,
               float* ref, double* wsum, double* err_hist, void* ws, size_t ws_bytes,
               hipStream_t stream);

/*
 * Batched iteration for serving many reconstructions at once.  Each job carries
 * its own scan, options, state buffers and workspace (sized by
 * pxst_workspace_bytes for that job).  One call performs, for every job, the step
 * selected by its `iter` field:
 *   0 <= iter < n_iter : one main-loop iteration (reference, pixel map,
 *                        translations if enabled, error -> err_hist[iter]);
 *   iter == n_iter     : the final reference update.
 * Stages shared across jobs: the inverted maps and splat of the reference update
 * (exact arithmetic, also when rounded to bfloat16; one launch per kernel for the
 * jobs of each frame-chunking form), the summed-area tables of invalid reference
 * pixels, the pixel-map search (shared launches over (job, tile) items per group
 * of jobs with one window; a job large enough to fill the device runs in launches of
 * its own), the translation search (one launch per kernel per translation window)
 * and the error (one launch per kernel per reference-lookup form).  Per job: the
 * frame variance and search setup at iter == 0, the float32-gather reference
 * arithmetic, the bfloat16 rounding and the map regularisation.  A job's results do
 * not depend on which other jobs share the call: each kernel computes a job's items
 * exactly as in a call of its own.
 * `batch_ws` (device memory, at least pxst_batch_workspace_bytes(n_jobs) bytes)
 * receives the argument tables, copied from pinned host staging memory in one
 * transfer before the first launch.  Calls that share `batch_ws` must be ordered
 * (same stream, or synchronised); the library serialises the host side and waits
 * for the previous call's table copy before it reuses the staging memory, which it
 * allocates (pinned, grown on demand) and keeps until the process ends.
 * Errors: every job and the workspace sizes are validated, and every table is staged,
 * before anything is enqueued; a PXST_EINVAL / PXST_EUNSUPPORTED / PXST_EWORKSPACE
 * return therefore leaves every job untouched.  A PXST_EHIP return (a failed HIP
 * call) can come after some stages were enqueued: the states of all jobs of the call
 * are then undefined.
 */
typedef struct {
    pxst_scan scan;
    pxst_solve_opts opts;
    float* u;
    float* dx;
    float* ref;
    double* wsum;
    double* err_hist;
    int32_t iter;
    void* ws;
    size_t ws_bytes;
} pxst_job;

size_t pxst_batch_workspace_bytes(int32_t n_jobs);
int pxst_batch_iterate(const pxst_job* jobs, int32_t n_jobs, void* batch_ws,
                       size_t batch_ws_bytes, hipStream_t stream);

/* Kernel timing for benchmarks: when enabled, the library brackets each launch of
 * the named kernel family with HIP events on the launch stream and accumulates
 * their elapsed times (reading them synchronises on the recorded events).
 * Families: "pm_fast", "pm_edge", "pm_edge_mma", "pm_generic", "pm_planes" (the
 * operand planes the matrix-core searches read; no work units), "pm_frac" (a whole
 * fractional-step search), "pm_split" (both split-half searches), "defocus_sweep",
 * "ref_gather",
 * "tr_partial", "err_pixels", "pm_fast_int8_ops" (the interior-tile search on the
 * matrix cores, counting int8 operations), "reg_filter" and "reg_integrate" (the
 * map regularisation).  pxst_profile_read returns the total milliseconds, the
 * number of timed launches and the work units of the family (candidate evaluations;
 * int8 operations for "pm_fast_int8_ops"; output values times taps for
 * "reg_filter"; float64 operations of the transforms for "reg_integrate"), and
 * resets the family. */
int pxst_profile_enable(int32_t on);
int pxst_profile_read(const char* family, double* total_ms, int64_t* launches,
                      int64_t* work_units);
/* Restricts the timing to the families named in `families` (comma-separated, e.g.
 * "pm_fast"); NULL or "" selects every family again (the default).  A restricted
 * selection brackets only those families' launches and copies no device work
 * counters (their work units read as 0), so that timing perturbs the stream as
 * little as possible: each event record and counter copy holds the stream for a few
 * microseconds.  Always returns PXST_OK. */
int pxst_profile_select(const char* families);

const char* pxst_last_error(void);
int32_t pxst_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PXST_H */
