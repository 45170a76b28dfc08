/*
 * rmsynth.h -- C ABI of the MI355X (gfx950) RM-synthesis library librmsynth.so.
 *
 * The library evaluates the discrete Faraday-depth transform of rotation
 * measure synthesis (Sridhar, Heald & van der Hulst, "cuFFS", Section 2.2):
 *
 *   F_l(phi_k) = K sum_j w_j (Q_lj + i U_lj) exp(-2 i phi_k (lambda_j^2 - lambda0^2))
 *                                                                    eq. (11)
 *   K = 1 / sum_j w_j                                                eq. (13)
 *   Re F = Qt, Im F = Ut                                         eqs. (15)-(16)
 *   |F| = sqrt(Qt^2 + Ut^2)                                          eq. (17)
 *
 * for every line of sight (LOS) l of a Q/U cube and every phi_k of a grid
 * (eqs. (18)-(19)), together with the RM spread function R(phi), eq. (12),
 * and the per-LOS peak of |F| (phi_peak, |F|max, Qt and Ut at the peak).
 *
 * Conventions shared by every call
 *   - Return value: RMSYNTH_OK (0) or a negative rmsynth_status.  The reason
 *     of the last failure on the calling thread is in rmsynth_last_error().
 *   - Argument errors are detected and returned before anything is enqueued.
 *   - Device buffers are plain device pointers (e.g. from hipMalloc or a torch
 *     tensor's data pointer) owned by the caller; the library never frees or
 *     keeps them.  Host arrays passed to rmsynth_plan are copied.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *     is enqueued asynchronously on it; nothing synchronises.  A fault inside a
 *     kernel surfaces as RMSYNTH_EHIP from a later call or synchronisation.
 *   - A plan belongs to the device that was current when it was created; it
 *     must be used with that device current.  A plan is immutable after
 *     creation and may be used concurrently from several streams.
 *   - Output layout is phi-fastest: Fq[l * nphi + k].
 */
#ifndef RMSYNTH_H
#define RMSYNTH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rmsynth_plan_s* rmsynth_plan_t;

typedef enum {
    RMSYNTH_OK = 0,
    RMSYNTH_EINVAL = -1,        /* invalid argument                          */
    RMSYNTH_ENOMEM = -2,        /* device or host allocation failed          */
    RMSYNTH_EHIP = -3,          /* a HIP runtime call or kernel launch failed */
    RMSYNTH_EUNSUPPORTED = -4,  /* valid but not supported combination      */
    RMSYNTH_EWORKSPACE = -5     /* workspace too small                       */
} rmsynth_status;

typedef enum {
    RMSYNTH_LOS_MAJOR = 0,   /* Q[l * nchan + j]: frequency fastest            */
    RMSYNTH_FREQ_MAJOR = 1   /* Q[j * nlos + l]: LOS fastest (channel planes)  */
} rmsynth_layout;

typedef enum {
    RMSYNTH_FP32 = 0,        /* FP32 products, FP32 accumulation (FP32 MFMA)     */
    RMSYNTH_SPLIT_BF16 = 1,  /* x = hi + lo in bfloat16; hi*hi + hi*lo + lo*hi
                                on BF16 MFMA with FP32 accumulation             */
    RMSYNTH_SPLIT_FP16 = 2   /* same split in IEEE half precision               */
} rmsynth_precision;

/*
 * rmsynth_plan -- prepare the channel set and the Faraday-depth grid.
 * Passage: eqs. (11)-(13) and the definition of lambda0^2 (Section 2.2);
 * K, 2 phi and lambda^2 - lambda0^2 are computed once per data set
 * (Section 2.3).
 *   lambda2  [nchan] host, lambda_j^2 in m^2, finite.
 *   weights  [nchan] host, w_j >= 0 and finite; w_j = 0 flags channel j (its
 *            Q/U values, NaN included, then have no effect).  sum w > 0.
 *   phi      [nphi]  host, Faraday depths in rad m^-2, finite, any order.
 *   lambda0_sq  reference lambda^2; NaN selects the weighted mean
 *            K sum_j w_j lambda_j^2.
 *   out      receives the plan (destroy with rmsynth_destroy).
 * Limits: 1 <= nchan <= 65536, 1 <= nphi <= 1048576.
 * K and lambda0^2 are formed in FP64 on the host; the plan uploads the
 * FP64 tables the GPU phase generator needs (a few tens of KB).
 * Errors: EINVAL (bad sizes / values / NULL), ENOMEM, EHIP.
 */
int rmsynth_plan(const double* lambda2, const double* weights, int32_t nchan,
                 const double* phi, int32_t nphi, double lambda0_sq,
                 rmsynth_plan_t* out);

/*
 * rmsynth_plan_info -- scalars of a plan (any pointer may be NULL).
 *   K           eq. (13).
 *   lambda0_sq  the reference lambda^2 in use.
 *   fwhm_est    2 sqrt(3) / Delta lambda^2, eq. (20), Delta lambda^2 = span of
 *               lambda^2 over channels of non-zero weight.
 *   phimax_est  sqrt(3) / delta lambda^2, eq. (21), delta lambda^2 = widest gap
 *               between adjacent channel centres (all channels).
 *   nchan, nphi sizes of the plan.
 */
int rmsynth_plan_info(rmsynth_plan_t plan, double* K, double* lambda0_sq,
                      double* fwhm_est, double* phimax_est,
                      int32_t* nchan, int32_t* nphi);

/*
 * rmsynth_workspace_size -- device workspace rmsynth_execute needs for `nlos`
 * LOS in the given layout and precision.  FP32 and the bfloat16 split read
 * Q/U in place and need none (*bytes = 0).  The FP16 split keeps one FP32
 * power-of-two scale per LOS (so that every LOS uses the half range without
 * overflow): round_up(4 max(nlos, 1), 256) bytes.
 *
 * Workspaces in general (this call, rmsynth_execute_peaks_workspace_size and
 * rmsynth_search_workspace_size): the size returned covers the whole call.  A
 * smaller workspace, of at least the size the same query returns for
 * min(nlos, 128) LOS, is also accepted: the call then processes the LOS in
 * batches of as many multiples of 128 as it holds, with the same results.
 */
int rmsynth_workspace_size(rmsynth_plan_t plan, int64_t nlos, int32_t layout,
                           int32_t precision, size_t* bytes);

/*
 * rmsynth_rmsf -- the RM spread function on the plan's grid, eq. (12):
 *   R(phi_k) = K sum_j w_j exp(-2 i phi_k (lambda_j^2 - lambda0^2)).
 *   R_re, R_im  [nphi] device float, written.
 * FP64 argument reduction, FP32 sin/cos and accumulation.
 */
int rmsynth_rmsf(rmsynth_plan_t plan, float* R_re, float* R_im, void* stream);

/*
 * rmsynth_execute -- the Faraday-depth transform, eqs. (11), (15)-(17), for
 * nlos lines of sight.
 *   Q, U     device float, layout RMSYNTH_LOS_MAJOR: [nlos][nchan];
 *            RMSYNTH_FREQ_MAJOR: [nchan][nlos].  Read only.
 *   nlos     >= 0 (0 enqueues nothing).
 *   precision  rmsynth_precision.
 *   Fq, Fu   [nlos][nphi] device float, written: Re F and Im F.
 *   Fabs     [nlos][nphi] device float or NULL: |F| when non-NULL.
 *   workspace, workspace_bytes: device scratch of at least
 *            rmsynth_workspace_size() bytes (may be NULL when that is 0).
 * A LOS whose unflagged channels hold a non-finite value gets non-finite
 * outputs; other LOS are unaffected.  RMSYNTH_SPLIT_FP16 keeps a per-LOS
 * power-of-two scale in the workspace (any phi grid); the workspace is
 * overwritten, and calls that share one workspace must not overlap.
 * The split precisions use factored phase tables on a uniform phi grid, a
 * plan-time table of the whole split phase matrix on other grids when it
 * holds at most 256 MiB (nchan x nphi up to about 1.6e7), and generate the
 * phases per element beyond that; the results agree to the same bounds.
 * Errors: EINVAL (NULL buffers with nlos > 0, bad layout/precision, wrong
 * device current), EWORKSPACE, EHIP (launch failure).
 */
int rmsynth_execute(rmsynth_plan_t plan, const float* Q, const float* U, int64_t nlos,
                    int32_t layout, int32_t precision,
                    float* Fq, float* Fu, float* Fabs,
                    void* workspace, size_t workspace_bytes, void* stream);

/*
 * rmsynth_execute_peaks -- rmsynth_execute followed by rmsynth_peaks on its
 * outputs, in one call: arguments as there (Fq, Fu are written as by
 * rmsynth_execute; idx, phi_pk, amp, q_pk, u_pk as by rmsynth_peaks, idx
 * required, the others may be NULL).  With a split precision on a uniform phi
 * grid, or on an irregular one whose phase table the plan holds (see
 * rmsynth_execute), the transform kernels reduce |F|^2 per (LOS, phi tile) while the tile
 * is still in registers and a small kernel merges the tiles, so the outputs are
 * not read back; the results are identical to the two separate calls.
 *   workspace: rmsynth_execute_peaks_workspace_size() bytes (the FP16
 *   split's per-LOS scales, then 16 bytes per LOS and phi tile of 128), or
 *   less down to its value for 128 LOS (LOS batches, see above).
 * With Fq, Fu and Fabs all NULL the call is rmsynth_search without the
 * sub-grid outputs (F is never stored; workspace as rmsynth_search's).
 * Errors as rmsynth_execute.
 */
int rmsynth_execute_peaks(rmsynth_plan_t plan, const float* Q, const float* U, int64_t nlos,
                          int32_t layout, int32_t precision, float* Fq, float* Fu, float* Fabs,
                          int32_t* idx, float* phi_pk, float* amp, float* q_pk, float* u_pk,
                          void* workspace, size_t workspace_bytes, void* stream);

/* rmsynth_execute_peaks_workspace_size -- device workspace rmsynth_execute_peaks
 * needs for nlos LOS in the given layout and precision. */
int rmsynth_execute_peaks_workspace_size(rmsynth_plan_t plan, int64_t nlos, int32_t layout,
                                         int32_t precision, size_t* bytes);

/*
 * rmsynth_search -- the per-LOS peak of |F| (Section 2.2 after eq. (14)) of
 * the transform of eqs. (11), (15)-(16) without storing F: what
 * rmsynth_execute followed by rmsynth_peaks and rmsynth_peak_fit return, for
 * a cube whose F would not fit or is not wanted (a 2048^2 x 4001 F is 134 GB).
 *   Q, U, nlos, layout, precision  as rmsynth_execute.
 *   idx, phi_pk, amp, q_pk, u_pk   as rmsynth_peaks (idx required, the
 *            others may be NULL); bit-identical to execute + peaks with the
 *            same precision.
 *   phi_fit, amp_fit [nlos] device float or NULL: the sub-grid peak, as
 *            rmsynth_peak_fit (bit-identical to it on the stored F).
 *   workspace: rmsynth_search_workspace_size() bytes, or less down to its
 *            value for 128 LOS (LOS batches).  With a split precision on a
 *            uniform phi grid, or on an irregular one whose phase table the
 *            plan holds, the transform kernels reduce each (LOS, 64 phi) to a
 *            32-byte record while F is in registers (32 bytes per LOS and 64
 *            phi); other paths hold F of one batch in the workspace.
 * Errors as rmsynth_execute.
 */
int rmsynth_search(rmsynth_plan_t plan, const float* Q, const float* U, int64_t nlos,
                   int32_t layout, int32_t precision, int32_t* idx, float* phi_pk, float* amp,
                   float* q_pk, float* u_pk, float* phi_fit, float* amp_fit, void* workspace,
                   size_t workspace_bytes, void* stream);

/* rmsynth_search_workspace_size -- device workspace rmsynth_search needs for
 * the whole of nlos LOS in the given layout and precision. */
int rmsynth_search_workspace_size(rmsynth_plan_t plan, int64_t nlos, int32_t layout,
                                  int32_t precision, size_t* bytes);

/*
 * rmsynth_search_noalloc -- rmsynth_search for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same arguments without a workspace,
 * the same results bit for bit.  Its workspace is a fixed array of
 * rmsynth_search_noalloc_scratch_bytes() (64 MiB) inside the library, one
 * per device, held until the process ends; the LOS run in batches that fit
 * it.  The call itself allocates nothing (no hipMalloc, hipFree or
 * allocating library routine).
 *   All calls on one device share that device's array: calls that overlap
 *   on a device (several streams or threads) race and must be serialised by
 *   the caller.  No part of the array has to start at zero.
 * Errors as rmsynth_search; EINVAL when one batch of 128 LOS does not fit
 * the array (only the unfused paths, which hold F of a batch: nphi above
 * 65536 at FP32, or on an irregular grid too large for a phase table).
 */
int rmsynth_search_noalloc(rmsynth_plan_t plan, const float* Q, const float* U, int64_t nlos,
                           int32_t layout, int32_t precision, int32_t* idx, float* phi_pk,
                           float* amp, float* q_pk, float* u_pk, float* phi_fit, float* amp_fit,
                           void* stream);

/* rmsynth_search_noalloc_scratch_bytes -- size of rmsynth_search_noalloc's
 * per-device array. */
size_t rmsynth_search_noalloc_scratch_bytes(void);

/*
 * rmsynth_adjoint -- spectra from Faraday-depth components on the plan's
 * grid: eq. (4) (P(lambda^2) as the integral of F(phi) exp(2i phi lambda^2))
 * as a sum over the grid, referred to lambda0^2 as eq. (11) refers F:
 *   P_lj = sum_k C_lk exp(+2i phi_k (lambda_j^2 - lambda0^2)),
 * i.e. the adjoint of rmsynth_execute without its K w_j factor (a single
 * component C_k = 1 gives the unit-amplitude spectrum of a Faraday-thin
 * screen at phi_k, eqs. (1), (3)).  The model spectra of RM-CLEAN components, or of any
 * model Faraday dispersion function, come from here.
 *   Cq, Cu   [nlos][nphi] device float: Re and Im of the components.
 *   Pq, Pu   [nlos][nchan] device float (LOS-major): Re and Im of P.
 *   precision  any rmsynth_precision.  The split precisions take tables
 *            instead of per-element phase generation: channels uniform in
 *            lambda^2 (the factored tables of the forward transform), a
 *            uniform phi grid of at least 288 values (K-tiles of 96 phi
 *            combined by Horner's rule), otherwise the whole split phase
 *            matrix when it holds at most 256 MiB.
 *   workspace  rmsynth_adjoint_workspace_size() bytes (0 except FP16), or
 *            less down to its value for 128 LOS (batches).
 * Every channel gets a value (weights do not enter).  A LOS with a
 * non-finite component gets non-finite outputs.
 * Errors as rmsynth_execute.
 */
int rmsynth_adjoint(rmsynth_plan_t plan, const float* Cq, const float* Cu, int64_t nlos,
                    int32_t precision, float* Pq, float* Pu, void* workspace,
                    size_t workspace_bytes, void* stream);

/* rmsynth_adjoint_workspace_size -- device workspace rmsynth_adjoint needs
 * for the whole of nlos LOS. */
int rmsynth_adjoint_workspace_size(rmsynth_plan_t plan, int64_t nlos, int32_t precision,
                                   size_t* bytes);

/*
 * rmsynth_execute_nufft -- the Faraday-depth transform of eq. (11) on a
 * uniform phi grid evaluated by a non-uniform FFT, the FFT evaluation the
 * paper proposes in place of the direct sums of eqs. (15)-(16) (Section 4):
 * with phi_k = phi_c + (k - kc) dphi (kc = nphi / 2), F is a type-1
 * non-uniform DFT of c_j = K w_j P_j exp(-2i a_j phi_c) at the points
 * x_j = 2 a_j dphi (mod 2 pi), computed by gridding the c_j onto the
 * smallest power-of-two grid n >= 2 nphi with an exponential-of-semicircle
 * kernel 8 cells wide, an n-point FFT (FP32) and division by the kernel's
 * Fourier transform.  An approximation of eq. (11): about 1e-6 of max|F|
 * per LOS (the kernel width's truncation below 1e-7, the rest FP32).
 *   Q, U     [nlos][nchan] device float (LOS-major).
 *   Fq, Fu   [nlos][nphi] device float; Fabs [nlos][nphi] or NULL.
 * Needs a uniform phi grid with n <= 8192 (nphi <= 4096), nchan <= 4096 and
 * (n + nchan) * 8 bytes of LDS per workgroup; EUNSUPPORTED otherwise.  A LOS
 * whose unflagged channels hold a non-finite value gets non-finite outputs.
 */
int rmsynth_execute_nufft(rmsynth_plan_t plan, const float* Q, const float* U, int64_t nlos,
                          float* Fq, float* Fu, float* Fabs, void* stream);

/*
 * rmsynth_rmclean -- RM-CLEAN of each LOS's Faraday spectrum: the
 * deconvolution by the RMSF R(phi) of eq. (12) that Section 2.2 names (and the
 * paper leaves unsupported, Section 4), as Hogbom's iteration on a uniform
 * phi grid:
 *   r <- F;  C <- 0;  repeat at most max_iter times:
 *     p = the lowest index maximising |r_k|^2 (FP32);  stop if |r_p| < cutoff;
 *     c = gain r_p;  C_p += c;  r_k -= c R((k - p) dphi) for every k;
 *   restored_k = r_k + sum_m C_m G((k - m) dphi),
 *   G(x) = exp(-4 ln 2 x^2 / fwhm^2) (Gaussian restoring beam of peak 1).
 * R is evaluated on the doubled grid (k - p) dphi by the plan's phase
 * generator (FP64 argument reduction, FP32 accumulation); the loop runs in
 * FP32.
 *   Fq, Fu   [nlos][nphi] device float: the spectrum (rmsynth_execute).
 *   gain     in (0, 1];  cutoff >= 0 (same unit as F);  max_iter >= 0.
 *   fwhm     of the restoring beam in rad m^-2; <= 0 or NaN: the plan's
 *            fwhm_est (eq. (20)).
 *   rq, ru   [nlos][nphi] device float: the residual r (may be Fq, Fu:
 *            in place).
 *   cq, cu   [nlos][nphi] device float: the components C (zero elsewhere).
 *   Rq, Ru   [nlos][nphi] device float or both NULL: the restored spectrum.
 *   niter    [nlos] device int32 or NULL: iterations taken; -1 for a LOS
 *            whose F is not finite (its outputs are then all NaN).
 *   workspace  rmsynth_rmclean_workspace_size() bytes (the two tables).
 * Requires a uniform phi grid and nphi <= 4096 (EUNSUPPORTED otherwise).
 * Components, restored spectrum and workspace must not overlap other buffers.
 */
int rmsynth_rmclean(rmsynth_plan_t plan, const float* Fq, const float* Fu, int64_t nlos,
                    float gain, float cutoff, int32_t max_iter, double fwhm, float* rq, float* ru,
                    float* cq, float* cu, float* Rq, float* Ru, int32_t* niter, void* workspace,
                    size_t workspace_bytes, void* stream);

/* rmsynth_rmclean_workspace_size -- device workspace rmsynth_rmclean needs:
 * 12 (2 nphi - 1) bytes, rounded up. */
int rmsynth_rmclean_workspace_size(rmsynth_plan_t plan, size_t* bytes);

/*
 * rmsynth_peak_fit -- sub-grid Faraday depth and amplitude of each LOS's peak
 * (an extension: the paper reports phi_peak on the grid, Section 2.2 after
 * eq. (14)): the vertex of the parabola through |F| at idx - 1, idx, idx + 1
 * (any grid spacing), |F| being the FP64 square root of the FP32
 * Fq^2 + Fu^2 the peak search compares; the arithmetic is FP64.
 *   Fq, Fu   [nlos][nphi] device float; idx [nlos] device int32 (as written
 *            by rmsynth_peaks).
 *   phi_fit, amp_fit [nlos] device float (either may be NULL, not both):
 *            the vertex; the grid values phi[idx], |F|(idx) where a
 *            neighbour is off the grid or the parabola does not open
 *            downwards; NaN where idx = -1.
 */
int rmsynth_peak_fit(rmsynth_plan_t plan, const float* Fq, const float* Fu, const int32_t* idx,
                     int64_t nlos, float* phi_fit, float* amp_fit, void* stream);

/*
 * rmsynth_peaks -- per-LOS peak of |F| (the Faraday depth phi_peak where |F|
 * is largest, Section 2.2 after eq. (14)).
 *   Fq, Fu   [nlos][nphi] device float (as written by rmsynth_execute).
 *   idx      [nlos] device int32: smallest k maximising Fq^2 + Fu^2 (FP32);
 *            -1 if any |F| of that LOS is non-finite.
 *   phi_pk   [nlos] device float: phi[idx] (NaN when idx = -1).
 *   amp      [nlos] device float: |F| at idx.
 *   q_pk, u_pk [nlos] device float: Fq, Fu at idx.  Any of the five outputs
 *            except idx may be NULL.
 */
int rmsynth_peaks(rmsynth_plan_t plan, const float* Fq, const float* Fu, int64_t nlos,
                  int32_t* idx, float* phi_pk, float* amp, float* q_pk, float* u_pk,
                  void* stream);

/*
 * rmsynth_peak_angle -- polarization angle of each LOS's peak referred to
 * lambda^2 = 0 (eq. (14), read as half the phase of F(phi_peak) after undoing
 * the exp(2i phi_peak lambda0^2) the lambda0^2 term of eq. (11) puts on it;
 * for a Faraday-thin screen it is the screen's intrinsic angle chi0).
 *   phi_pk, q_pk, u_pk [nlos] device float, as written by rmsynth_peaks.
 *   chi0     [nlos] device float (output): radians in [0, pi); NaN where an
 *            input is not finite (LOS with idx = -1).
 * Evaluated in FP64 from the FP32 inputs and the plan's lambda0^2.  nlos >= 0.
 */
int rmsynth_peak_angle(rmsynth_plan_t plan, const float* phi_pk, const float* q_pk,
                       const float* u_pk, int64_t nlos, float* chi0, void* stream);

/* rmsynth_destroy -- free a plan's device tables (NULL is a no-op).  The caller
 * must make sure no enqueued work still uses the plan. */
void rmsynth_destroy(rmsynth_plan_t plan);

/* rmsynth_last_error -- message of the last failure on this thread ("" if none). */
const char* rmsynth_last_error(void);

/* rmsynth_version -- library version string. */
const char* rmsynth_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RMSYNTH_H */
