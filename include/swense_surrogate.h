/*
 * swense_surrogate.h - C ABI of the learned surrogate of the HOS step: a
 * spectral neural operator (Fourier neural operator) that maps the surface
 * state (eta, phis) at time t to its change over s HOS steps beyond the exact
 * linear propagator, with BF16 MFMA contractions and FP32 accumulation,
 * trained on the GPU on trajectories of the HOS step itself, and a rollout
 * that keeps the HOS step (Sec. 3.1.2) as its fallback and the judge of its
 * error.  The paper has no learned component: this part follows the
 * surrogate requirements of the project; its readings are listed with the
 * design notes.
 *
 * Conventions are those of swense.h (return codes, streams, ownership).
 *
 * Network, per sample on an n x n grid (x fastest), C channels:
 *   v_0 = W_0 x + b_0                               (lift, in -> C, pointwise)
 *   v_l = gelu(W_l v_{l-1} + b_l + K_l(v_{l-1}))     (l = 1..L)
 *   y   = Q_2 gelu(Q_1 v_L + c_1) + c_2              (projection C -> H -> 2)
 * K_l(v) is the truncated spectral convolution: vhat = rfft2(v) / n^2 on the
 * retained modes S = {(p, q): 0 <= p < P along x, -Q <= q <= Q along y},
 * per-mode complex channel mixing yhat_o = sum_i vhat_i R_l[s][i][o], the
 * p = 0 column projected onto Hermitian symmetry (q and -q averaged with
 * conjugation, q = 0 made real), and back: sum_S c_p Re(yhat e^{i k.x}) with
 * c_0 = 1, c_{p>0} = 2.  gelu is the tanh form.  Every GEMM input
 * (activations and weights, forward and backward) is rounded to BF16 (round
 * to nearest even); accumulation, activations between layers and the master
 * weights are FP32.
 *
 * Parameter vector (FP32, packed in this order, row-major):
 *   W_0 [C][in_channels], b_0 [C],
 *   for l = 1..L: W_l [C][C], b_l [C], R_l [nq][P][C][C] complex (re, im)
 *                 interleaved, mode index s = a P + p with a the position of q
 *                 in the order 0, 1, .., Q, -Q, .., -1 (nq = 2Q + 1),
 *   Q_1 [H][C], c_1 [H], Q_2 [2][H], c_2 [2].
 * Activations: [batch][channel][n][n] FP32 device arrays.
 */
#ifndef SWENSE_SURROGATE_H
#define SWENSE_SURROGATE_H

#include <stddef.h>

#include "swense.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct swense_fno_desc {
  int n;         /* grid points per axis: 64, 128, 256, 512 or 1024           */
  int channels;  /* C: even, 2..256                                           */
  int layers;    /* L: 1..32                                                  */
  int p_modes;   /* P: retained p in [0, P), 1 <= P < n/2                     */
  int q_modes;   /* Q: retained q in [-Q, Q], 2Q + 1 <= n/2                   */
  int hidden;    /* H: projection width                                       */
  int in_channels; /* input fields: 2 (eta, phis) or 4 (with their linear    */
                   /* propagation over the surrogate stride), 1..16          */
  int max_batch; /* largest batch passed to any call (sizes the workspaces)   */
} swense_fno_desc;

typedef struct swense_fno swense_fno; /* network + optimiser state (opaque) */

/* Number of FP32 parameters of the packed vector for descriptor d. */
size_t swense_fno_param_count(const swense_fno_desc* d);

/* Create a network with the packed parameters `params` (host FP32, copied).
 * The handle owns its device memory: FP32 master weights, their BF16 copy,
 * gradients, Adam moments and activation workspaces for max_batch samples.
 * stream: HIP stream of all later work (NULL = null stream).  Synchronises. */
int swense_fno_create(const swense_fno_desc* d, const float* params, void* stream, swense_fno** out);

/* Forward pass: x device [batch][in_channels][n][n] -> y device [batch][2][n][n].
 * Keeps the activations for a following swense_fno_backward.  Asynchronous. */
int swense_fno_forward(swense_fno* f, const float* x, float* y, int batch);

/* Relative L2 loss (mean over samples and the two channels of
 * ||y - t||^2 / ||t||^2) and its gradient gy (device, same layout as y).
 * Synchronises to return *loss. */
int swense_fno_loss(swense_fno* f, const float* y, const float* t, float* gy, int batch, float* loss);

/* Backward pass of the last forward (same batch and x): parameter gradients
 * into the handle's gradient vector (overwritten), input gradient into gx
 * (device [batch][in_channels][n][n], may be NULL).  Asynchronous. */
int swense_fno_backward(swense_fno* f, const float* x, const float* gy, float* gx, int batch);

/* One optimiser step on (x, t): forward, loss, backward, Adam (beta1 0.9,
 * beta2 0.999, eps 1e-8, learning rate lr) on the FP32 masters, BF16 copy
 * refreshed.  Synchronises to return *loss (may be NULL). */
int swense_fno_train_step(swense_fno* f, const float* x, const float* t, int batch, float lr, float* loss);

/* Copy out (host, param_count floats) what = 0: master weights, 1: gradients
 * of the last backward, 2: Adam first moments, 3: Adam second moments.
 * Synchronises. */
int swense_fno_get(swense_fno* f, int what, float* host);

/* Load a packed vector (host FP32): what = 0 the master weights (the BF16
 * copy is refreshed, the Adam state kept), 2 and 3 the Adam moments (restoring
 * a checkpoint).  Synchronises. */
int swense_fno_set(swense_fno* f, int what, const float* host);

/* Activations of the last forward pass, for checking a layer on its own
 * inputs (host): v_0 .. v_L and z_1 .. z_L ([batch][C][n][n] each, v_l the
 * input of layer l + 1 and z_l the pre-activation of layer l), then zq and h
 * ([batch][H][n][n]: the projection's pre-activation and its GELU), for the
 * last forward's batch, in that order: (2L + 1) batch C n^2 + 2 batch H n^2
 * floats.  Synchronises. */
int swense_fno_get_activations(swense_fno* f, float* host);

/* Intermediate gradients of the backward passes, for checking a layer on its
 * own upstream gradient: trace (device, caller-owned, at least
 * (L + 1) max_batch C n^2 + max_batch H n^2 floats; NULL: off) receives from
 * each later backward dL/dz_1 .. dL/dz_L and dL/dv_0 ([batch][C][n][n] each),
 * then dL/dzq ([batch][H][n][n]), in that order. */
int swense_fno_set_trace(swense_fno* f, float* trace);

const char* swense_fno_last_error(const swense_fno* f);
void swense_fno_destroy(swense_fno* f);

/* The contraction the network runs on: C = A B for row-major FP32 device
 * matrices A [M][K], B [K][N], C [M][N], with A and B rounded to BF16 (round
 * to nearest even) and FP32 accumulation on the matrix cores.  Asynchronous
 * on `stream`. */
int swense_gemm_bf16(int M, int N, int K, const float* A, const float* B, float* C, void* stream);

/* ---- rollout with the HOS step as fallback and judge ------------------ */

/* Surrogate call: with X = (eta, phis) the physical surface state of a square
 * realisation (nx = ny = n of the network), the network input is
 * x = (eta / sigma_eta, phis / sigma_phi), followed for a 4-channel network
 * by the same scaling of the base prediction B(X), and its output y gives
 *   X(t + s dt) = B(X(t)) + rho (sigma_eta y_0, sigma_phi y_1),
 * B either Lin_{s dt} or a coarse integrating-factor RK4 step over s dt
 * (base_substeps).  Lin_tau is the exact linear propagator, mode by mode with omega^2 = g k tanh(kh)
 * (deep water: g k): eta <- cos(w tau) eta + (k tanh(kh)/w) sin(w tau) phis,
 * phis <- cos(w tau) phis - (g/w) sin(w tau) eta; k = 0: phis <- phis - g tau
 * eta.  The mean of eta (k = 0) is kept from X(t): mass is conserved as in
 * the HOS step.  The linear part and the state stay FP64. */
typedef struct swense_surrogate_desc {
  int stride_s;       /* s: HOS steps replaced by one call (>= 1)                 */
  double sigma_eta;   /* input scale of eta                                       */
  double sigma_phi;   /* input scale of phis                                      */
  double rho;         /* output scale of the residual                             */
  double tol;         /* audit threshold: relative L2 error, max over eta, phis   */
  int audit_every;    /* A: every A-th surrogate call is re-run by HOS and judged */
  int cooldown;       /* calls advanced by HOS alone after a fallback             */
  double energy_tol;  /* guard on |E1 - E0| / |E0| per call (<= 0: off)           */
  int probation;      /* passed audits in a row required before network calls */
                      /* go unaudited between the A-th ones (0: none)          */
  int base_substeps;  /* base prediction B: 0 = Lin_{s dt} (exact linear        */
                      /* propagation); n > 0 = n integrating-factor RK4        */
                      /* substeps over s dt (swense_hos_step_exp)              */
  double drift_tol;   /* bound on the estimated error accumulated against     */
                      /* plain HOS since creation or the last reset (<= 0:   */
                      /* none): each unjudged call adds the largest judged   */
                      /* error so far; a call that would pass the bound, and */
                      /* every call after it, is advanced by HOS             */
  int base_only;      /* 1: each call is the base prediction B alone (the     */
                      /* network is not evaluated), judged the same way     */
} swense_surrogate_desc;

/* Counters accumulated by swense_surrogate_advance (zero them before use). */
typedef struct swense_surrogate_stats {
  long long calls;           /* calls requested                                   */
  long long surrogate_calls; /* calls advanced by the network                     */
  long long hos_calls;       /* calls advanced by HOS alone (cool-down)           */
  long long audits;          /* network calls re-run by HOS and compared          */
  long long fallbacks;       /* audits above tol or guard trips: HOS state kept   */
  long long guard_trips;     /* non-finite state or energy change above its bound */
  double max_audit_err;      /* largest audited relative error                    */
  double last_audit_err;
  long long bound_calls;     /* calls advanced by HOS because of drift_tol        */
  double drift_est;          /* estimated accumulated error after the last call  */
} swense_surrogate_stats;

typedef struct swense_surrogate swense_surrogate; /* (opaque) */

/* Tie a network to a realisation: h must be 3D with nx = ny = the network's
 * n, and both handles must use the same stream.  The surrogate owns its
 * scratch (a state backup and two network buffers); h and f must outlive it. */
int swense_surrogate_create(swense_hos* h, swense_fno* f, const swense_surrogate_desc* d, swense_surrogate** out);

/* Network input of the current state, x (device [2][n][n] FP32), and, when
 * lin is non-NULL, the scaled fields of the base prediction B of the current
 * state in the same units (device [2][n][n]); the state is left unchanged.
 * Training data come from these two and swense_surrogate_target.
 * Asynchronous. */
int swense_surrogate_features(swense_surrogate* s, float* x, float* lin);

/* Training target of a pair: t = (x_next - base) / rho, elementwise over
 * [2][n][n] (x_next: features of the state s steps later; lin: from
 * swense_surrogate_features at the earlier state).  Asynchronous. */
int swense_surrogate_target(swense_surrogate* s, const float* x_next, const float* lin, float* t);

/* Advance the realisation by ncalls x s HOS steps of time, each call by the
 * network (guards on every call: non-finite values, energy change) or by HOS
 * (cool-down after a fallback).  A network call is judged when its guard
 * trips, when it is the A-th since the last judged one, or while fewer than
 * `probation` judged calls have passed in a row (from creation and after
 * every fallback), and, with a drift bound, while no call has been judged
 * since the reset: HOS re-runs the s steps from the saved state, the relative
 * L2 error of the network's state against it is recorded, and the HOS state
 * is kept; an error above tol (tol = 0: always) or a tripped guard counts as
 * a fallback and starts the cool-down.  A judged call adds no error of its
 * own to the rollout (its HOS state is kept); an unjudged one adds, to the
 * estimate, the largest judged error since the reset.  With drift_tol > 0,
 * once the next unjudged call would take the estimate past drift_tol the
 * rollout continues with HOS alone until swense_surrogate_reset.
 * Synchronises per call. */
int swense_surrogate_advance(swense_surrogate* s, int ncalls, swense_surrogate_stats* stats);

/* Start a new rollout (e.g. after the realisation's state was set): clears
 * the cool-down, the probation record, the audit counter, the largest judged
 * error and the drift estimate. */
int swense_surrogate_reset(swense_surrogate* s);

const char* swense_surrogate_last_error(const swense_surrogate* s);
void swense_surrogate_destroy(swense_surrogate* s);

#ifdef __cplusplus
}
#endif
#endif /* SWENSE_SURROGATE_H */
