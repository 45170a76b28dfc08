/*
 * rmsynth_mlp.h -- learned gate for RM synthesis on AMD Instinct MI355X
 * (gfx950).
 *
 * The paper evaluates the Faraday dispersion function of eq. (15) for every
 * line of sight of the cube (Sect. 3).  When most lines of sight hold no
 * polarised source, a small network that looks at the Q/U spectrum can pick
 * the lines of sight worth the fine-grid synthesis; the others report the
 * network's estimate.  The network is not part of the paper: this header is
 * the boundary of that extension.  Every line of sight the gate passes is
 * synthesised by rmsynth_execute and searched by rmsynth_peaks, exactly as in
 * the ungated path.
 *
 * Network (per line of sight, nchan channels, weights w_j of the plan):
 *   x  = [w Q | w U] / rms(w Q, w U)              (2 nchan inputs)
 *   h1 = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),  o = W3 h2 + b3
 *   phi_hat = o[0] * phi_scale,  score = sigmoid(o[1])
 *   loss = mean over the batch of BCE(score, det) + det (o[0] - phi/phi_scale)^2
 * x, h1, h2, dz and the weights are rounded to IEEE half for the FP16 matrix
 * cores (FP32 accumulation); master weights and Adam moments are FP32.
 *
 * Canonical parameter vector (FP32, nparams = h1 (2 nchan + 1) + h2 (h1 + 1)
 * + 2 (h2 + 1)):  W1 [h1][2 nchan] row-major, b1 [h1], W2 [h2][h1], b2 [h2],
 * W3 [2][h2], b3 [2].
 *
 * Conventions as in rmsynth.h: Q/U and all outputs are device pointers in
 * LOS-major layout (Q[l][j]); calls are asynchronous on `stream` (a
 * hipStream_t, NULL = default stream) unless stated otherwise; argument
 * errors return synchronously with a message in rmsynth_last_error().  A
 * network object keeps its own activation buffers, so one object must not be
 * used from two streams at once.  The object lives on the device that was
 * current at creation; calls from another device return RMSYNTH_EINVAL.
 */
#ifndef RMSYNTH_MLP_H
#define RMSYNTH_MLP_H

#include "rmsynth.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rmsynth_mlp_s* rmsynth_mlp_t;

/*
 * rmsynth_mlp_create -- network for spectra of `nchan` channels with hidden
 * widths h1, h2 (multiples of 64, at most 4096).  `weights` (host, [nchan],
 * NULL = all ones; finite, >= 0) are the channel weights applied to the
 * inputs; zero-weight channels are ignored, as in the synthesis.
 * phi_scale > 0 scales the Faraday-depth output.  Weights are He-normal
 * from `seed`, biases zero, Adam moments zero.  Allocates device memory.
 */
int rmsynth_mlp_create(int32_t nchan, int32_t h1, int32_t h2, const float* weights,
                       float phi_scale, uint64_t seed, rmsynth_mlp_t* out);

/* rmsynth_mlp_num_params -- length of the canonical parameter vector. */
int rmsynth_mlp_num_params(rmsynth_mlp_t mlp, int64_t* nparams);

/* rmsynth_mlp_info -- the sizes a network was created with (any pointer may
 * be NULL): channels per spectrum, hidden widths, Faraday-depth scale of the
 * first output.  Host only; EINVAL when mlp is NULL. */
int rmsynth_mlp_info(rmsynth_mlp_t mlp, int32_t* nchan, int32_t* h1, int32_t* h2,
                     float* phi_scale);

/*
 * rmsynth_mlp_get_params / rmsynth_mlp_set_params -- copy the FP32 master
 * parameters to / from a HOST array of nparams floats in canonical order.
 * Synchronous (waits for the device).  set_params leaves the Adam moments
 * and step count unchanged and refreshes the half copies.
 */
int rmsynth_mlp_get_params(rmsynth_mlp_t mlp, float* params);
int rmsynth_mlp_set_params(rmsynth_mlp_t mlp, const float* params);

/*
 * rmsynth_mlp_grad -- loss and gradient of the mean loss over `batch` lines
 * of sight, without updating the parameters.
 *   Q, U       device [batch][nchan]
 *   phi_label  device [batch]  Faraday depth of the brightest component
 *   det_label  device [batch]  1 for a detection, 0 otherwise (values in [0, 1])
 *   grad       device [nparams], canonical order (output)
 *   loss       device [1] mean loss (output, may be NULL)
 * batch >= 1.  Grows the object's activation buffers when needed.
 */
int rmsynth_mlp_grad(rmsynth_mlp_t mlp, const float* Q, const float* U, int64_t batch,
                     const float* phi_label, const float* det_label, float* grad, float* loss,
                     void* stream);

/*
 * rmsynth_mlp_train_step -- one Adam step (beta1 0.9, beta2 0.999, eps 1e-8,
 * bias-corrected, learning rate lr > 0) on the gradient rmsynth_mlp_grad
 * computes; arguments as there.
 */
int rmsynth_mlp_train_step(rmsynth_mlp_t mlp, const float* Q, const float* U, int64_t batch,
                           const float* phi_label, const float* det_label, float lr, float* loss,
                           void* stream);

/*
 * rmsynth_mlp_infer -- phi_hat and detection score for nlos >= 0 lines of
 * sight (device [nlos] each).  A non-finite unflagged input gives NaN
 * outputs.  Hidden widths 256 and 256 run as one fused kernel per call (the
 * first call after a parameter change also rebuilds, on `stream`, the
 * object's copy of W1 and W2 in matrix-core fragment order); other widths
 * work in chunks through the object's buffers.  An object is not to be used
 * from several host threads at once.
 */
int rmsynth_mlp_infer(rmsynth_mlp_t mlp, const float* Q, const float* U, int64_t nlos,
                      float* phi_hat, float* score, void* stream);

/*
 * rmsynth_gate_workspace_size -- device workspace rmsynth_gate_execute needs
 * for `nlos` lines of sight with this plan.
 */
int rmsynth_gate_workspace_size(rmsynth_plan_t plan, rmsynth_mlp_t mlp, int64_t nlos,
                                size_t* bytes);

/*
 * rmsynth_gate_execute -- gated peak search.  For every line of sight the
 * network gives (phi_hat, score); the line of sight is GATED when
 * score >= tau, when either output is not finite, or when |phi_hat| lies
 * within one RMSF width (plan's 2 sqrt(3) / span of lambda^2) of the largest
 * |phi| of the plan's grid.  Gated lines of sight are gathered, synthesised
 * with rmsynth_execute (FP32 path) and searched with rmsynth_peaks; the
 * results are scattered back:
 *   idx[l], phi_pk[l], amp[l]: the peak of eq. (15) on the plan's grid
 *       (as rmsynth_peaks), for gated l;  idx = -1, phi_pk = phi_hat,
 *       amp = NaN for the others.
 *   gated[l]: 1 or 0.
 * The plan's nchan must equal the network's.  workspace: device memory of at
 * least rmsynth_gate_workspace_size() bytes.  Synchronises `stream` once
 * (to read the number of gated lines of sight).
 */
int rmsynth_gate_execute(rmsynth_plan_t plan, rmsynth_mlp_t mlp, const float* Q, const float* U,
                         int64_t nlos, float tau, int32_t* idx, float* phi_pk, float* amp,
                         int32_t* gated, void* workspace, size_t workspace_bytes, void* stream);

/*
 * rmsynth_gate_search -- rmsynth_gate_execute with the gated lines of sight
 * searched by rmsynth_search in the given precision (F never stored): gated
 * outputs are bit for bit those of rmsynth_search over the whole cube in that
 * precision, the others as rmsynth_gate_execute.  workspace: at least
 * rmsynth_gate_search_workspace_size() bytes.  Errors as rmsynth_gate_execute,
 * plus EINVAL for a bad precision.
 */
int rmsynth_gate_search(rmsynth_plan_t plan, rmsynth_mlp_t mlp, const float* Q, const float* U,
                        int64_t nlos, int32_t precision, float tau, int32_t* idx, float* phi_pk,
                        float* amp, int32_t* gated, void* workspace, size_t workspace_bytes,
                        void* stream);

/* rmsynth_gate_search_workspace_size -- device workspace rmsynth_gate_search
 * needs for `nlos` lines of sight in this precision. */
int rmsynth_gate_search_workspace_size(rmsynth_plan_t plan, rmsynth_mlp_t mlp, int64_t nlos,
                                       int32_t precision, size_t* bytes);

/*
 * Training data.  Synthetic spectra of the sky model of Section 2.1: a
 * Faraday-thin screen P0 exp(2i(chi0 + phi0 lambda^2)) (eqs. (1), (3)), two
 * such screens, or a Burn slab of width W, P0 exp(2i(chi0 + phic lambda^2))
 * sin(W lambda^2)/(W lambda^2) (eq. (4)), plus N(0, sigma^2) noise on every
 * channel and Stokes parameter.  P0, phi0, W are uniform over the given
 * ranges, chi0 uniform over [0, pi).  Draws come from Philox4x32-10 (Salmon
 * et al., SC 2011) addressed by (seed, global line-of-sight index), so a line
 * of sight has the same content whatever batch makes it:
 *   counters (0, g_lo, g_hi, 0) class, (1 + c, g_lo, g_hi, 0) component c,
 *   (m, g_lo, g_hi, 1) noise of channels 2m and 2m + 1;
 *   32-bit word x -> u = (floor(x / 2^9) + 1/2) 2^-23;
 *   class 0 (noise only) if u < frac_noise, 1 (one screen) if
 *   u < frac_noise + frac_thin1, 2 (two screens) if below that + frac_thin2,
 *   else 3 (slab);  component words -> P0, phi0, chi0, W in that order;
 *   noise by Box-Muller, (r cos t, r sin t) -> (Q, U), r = sqrt(-2 ln u0),
 *   t = 2 pi u1 for channel 2m and (u2, u3) for channel 2m + 1.
 * The model is evaluated in FP64 and rounded to FP32 once.  Labels come from
 * the transform itself: rmsynth_execute (FP32 path) on the plan's grid and
 * rmsynth_peaks; phi_label = phi at the peak, det_label = 1 iff the peak
 * |F| >= det_threshold (0 for a line of sight with non-finite input).
 */
typedef struct rmsynth_train_spec {
    double frac_noise, frac_thin1, frac_thin2;  /* class fractions; slabs get the rest */
    double p0_lo, p0_hi;                        /* polarised amplitude, >= 0 */
    double phi_lo, phi_hi;                      /* Faraday depth of the components */
    double w_lo, w_hi;                          /* slab width, > 0 */
    double sigma;                               /* noise per channel and Stokes, >= 0 */
    double det_threshold;                       /* detection threshold on the peak |F| */
} rmsynth_train_spec;

/* rmsynth_train_workspace_size -- workspace rmsynth_synth_training needs to
 * label nlos lines of sight (0 when no labels are asked for is also fine). */
int rmsynth_train_workspace_size(rmsynth_plan_t plan, int64_t nlos, size_t* bytes);

/*
 * rmsynth_synth_training -- lines of sight first_los .. first_los + nlos - 1
 * of the stream `seed`, on the plan's channels (its lambda^2).
 *   Q, U        device [nlos][nchan] float, written
 *   phi_label, det_label  device [nlos] float or both NULL (no labelling,
 *               no workspace needed)
 *   cls         device [nlos] int32 or NULL: class 0..3
 *   truth       device [nlos][4] float or NULL: (phi0, P0) of components 0
 *               and 1, NaN where absent
 * Errors: EINVAL (bad spec, NULL Q/U, first_los < 0), EWORKSPACE, EHIP.
 */
int rmsynth_synth_training(rmsynth_plan_t plan, const rmsynth_train_spec* spec, uint64_t seed,
                           int64_t first_los, int64_t nlos, float* Q, float* U, float* phi_label,
                           float* det_label, int32_t* cls, float* truth, void* workspace,
                           size_t workspace_bytes, void* stream);

/*
 * rmsynth_mlp_save / rmsynth_mlp_load -- binary file with the shape, channel
 * weights, phi_scale, master parameters, Adam moments and step count.  load
 * creates a new object on the current device.  Synchronous.
 */
int rmsynth_mlp_save(rmsynth_mlp_t mlp, const char* path);
int rmsynth_mlp_load(const char* path, rmsynth_mlp_t* out);

/* rmsynth_mlp_destroy -- frees the object (NULL is ignored). */
void rmsynth_mlp_destroy(rmsynth_mlp_t mlp);

#ifdef __cplusplus
}
#endif

#endif /* RMSYNTH_MLP_H */
