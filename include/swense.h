/*
 * swense.h - C ABI of the MI355X (gfx950) incident-wave library.
 *
 * The library implements the incident-wave side of the two-phase SWENSE
 * method (Li et al., "Spectral Wave Explicit Navier-Stokes Equations for
 * wave-structure interactions using two-phase CFD solvers", arXiv 2005.12716):
 *   - the High-Order Spectral (HOS) free-surface step (Sec. 3.1.2),
 *   - the modal evaluation of potential, velocity, pressure and their time
 *     derivatives on an intermediate grid with zero-padding refinement and
 *     extension into the air (Sec. 3.2.2, 3.2.4, 3.3),
 *   - the interpolation of those fields to CFD cell centres (Sec. 3.2.2) and
 *     the divergence diagnostic of Sec. 3.2.3.
 *
 * Conventions shared by every entry point:
 *   - Return value: 0 (SWENSE_OK) or a negative SWENSE_E* code.  No entry point
 *     throws, aborts or frees caller memory.  The text of the last error of a
 *     handle is returned by swense_last_error.
 *   - Spectral layout: half spectrum [ny][nx/2+1] of interleaved FP64
 *     (re, im) pairs, x fastest; f(x,y) = sum_k fhat(k) exp(i k.x) with
 *     k = (2 pi p/lx, 2 pi q/ly), q >= ny/2 meaning q - ny (fhat = DFT / (nx ny)).
 *     Physical layout: [ny][nx] FP64, node (i, j) at (i lx/nx, j ly/ny).
 *     Nyquist modes (p = nx/2, q = ny/2) are held at zero.
 *   - Memory: pointers documented "host" are ordinary host memory read or
 *     written synchronously; "device" pointers are HIP device memory owned by
 *     the caller.  Each handle owns the device memory it allocates internally
 *     (state, workspaces, bound point data) and releases it in its destroy call.
 *   - Streams: all GPU work of a handle is ordered on the HIP stream given at
 *     creation (NULL = the null stream) and is asynchronous unless a call is
 *     documented to synchronise.  A handle is not thread-safe.
 *   - Units: any consistent set (g and rho are parameters).  z points up,
 *     z = 0 is the still-water level.
 */
#ifndef SWENSE_H
#define SWENSE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SWENSE_OK = 0,
  SWENSE_EINVAL = -1,    /* bad argument or descriptor                        */
  SWENSE_ENOMEM = -2,    /* device allocation failed                          */
  SWENSE_EHIP = -3,      /* HIP runtime error (message kept)                  */
  SWENSE_EUNSTABLE = -4, /* non-finite state                                  */
  SWENSE_ERANGE = -5,    /* some points outside the grid or layers (non-fatal) */
  SWENSE_ENOTSUP = -6    /* unsupported combination                           */
};

/* Field bits for evaluation and interpolation masks; the output order is the
 * bit order of the fields present in the mask. */
enum {
  SWENSE_PHI = 1u << 0,   /* velocity potential                         */
  SWENSE_U = 1u << 1,     /* velocity components                        */
  SWENSE_V = 1u << 2,
  SWENSE_W = 1u << 3,
  SWENSE_P = 1u << 4,     /* pressure -rho (phi_t + |grad phi|^2/2 + g z) */
  SWENSE_PHI_T = 1u << 5, /* time derivatives of phi, u, v, w           */
  SWENSE_U_T = 1u << 6,
  SWENSE_V_T = 1u << 7,
  SWENSE_W_T = 1u << 8,
  SWENSE_ETA = 1u << 9,   /* free-surface elevation (z-independent)     */
  SWENSE_ETA_T = 1u << 10,
  SWENSE_ALL_FIELDS = (1u << 11) - 1u
};

enum { SWENSE_PHYSICAL = 0, SWENSE_SPECTRAL = 1 };

typedef struct swense_hos swense_hos;     /* one HOS realisation (opaque)       */
typedef struct swense_cells swense_cells; /* a bound, static point cloud (opaque) */

/* One HOS realisation (Sec. 3.1.2).
 *   dim: 2 (x, z; ny must be 1) or 3.  nx, ny: modes per direction, even and
 *   2/3/5-smooth (ny = 1 for dim 2).  depth <= 0 selects infinite depth.
 *   order_m >= 1: order of the vertical-velocity series.  dealias: 1 forms
 *   products on the (M+1)/2 zero-padded grid (the smallest even 2/3/5-smooth
 *   length past (M+1) n / 2), 2 on the smallest 2^k or 3 2^k length past it
 *   (more points, transforms compiled for the length; the truncated products
 *   are the same), 0 on the mode grid.
 *   precision: 0 = FP32 transforms with FP64 state, symbols and time
 *   integration; 1 = FP64 throughout.  dt: RK4 time step; t0: initial time. */
typedef struct {
  int dim;
  int nx, ny;
  double lx, ly;
  double depth;
  double g, rho;
  int order_m;
  int dealias;
  int precision;
  double dt, t0;
} swense_hos_desc;

/* Intermediate grid (Sec. 3.2.2, 3.2.4).  gx, gy nodes per period: gx > nx
 * zero-pads the spectrum (refinement n = gx/nx), gx < nx folds it; both give
 * the exact modal sum at the nodes.  Window: nodes ix0..ix0+wx-1 (mod gx),
 * iy0..iy0+wy-1 (mod gy).  nl layer heights z (ascending, host memory), any
 * z (above z = 0 the modal formula extends the fields into the air, Sec. 3.3).
 * In 2D gy = wy = 1, iy0 = 0. */
typedef struct {
  int gx, gy;
  int ix0, iy0, wx, wy;
  int nl;
  const double* z;
} swense_grid_desc;

/* Sea-state description for the initial spectra (set-up, Sec. 3.1.2 and the
 * JONSWAP example of Sec. 3.2.2).  kind 0: JONSWAP with peak wavenumber kp,
 * significant height hs, peakedness gamma, spreading 0 = cos^2, 1 = all energy
 * along +x; amplitudes scaled so that 4 sqrt(m0) = hs on the discrete modes.
 * kind 1: second-order Stokes wave on mode `mode` along x with steepness ka. */
typedef struct {
  int kind;
  double hs, kp, gamma;
  int spreading;
  int mode;
  double ka;
} swense_sea_desc;

/* ---- set-up ----------------------------------------------------------- */

/* Initial half spectra of a linear sea (kind 0) or a second-order Stokes wave
 * (kind 1).  phases: host [ny][nx/2+1] FP64 phases of the modes (kind 0 only;
 * may be NULL for kind 1).  eta_hat, phis_hat: host outputs, spectral layout.
 * Deterministic amplitudes; the random phases are an input. */
int swense_sea_spectrum(const swense_hos_desc* d, const swense_sea_desc* sea,
                        const double* phases, double* eta_hat, double* phis_hat);

/* Create a realisation and load its initial state (eta, surface potential
 * phis = phi at z = eta).  eta0, phis0: host arrays in `layout` (SWENSE_PHYSICAL
 * or SWENSE_SPECTRAL).  stream: a hipStream_t or NULL.  Allocates the state and
 * workspaces on the current device.  EINVAL on a bad descriptor. */
int swense_hos_init(const swense_hos_desc* d, const double* eta0, const double* phis0, int layout,
                    void* stream, swense_hos** out);

/* Bytes of device workspace a realisation needs when its caller owns the
 * memory (swense_hos_init_ws): the FP64 state and spectral buffers, the
 * transform-precision intermediates of the HOS step (Sec. 3.1.2), physical
 * staging, the twiddle tables of the product and mode grids, and the
 * buffers of the concurrent interpolation and of evaluation between two
 * outputs.  EINVAL on a bad descriptor. */
int swense_hos_workspace_bytes(const swense_hos_desc* d, size_t* bytes);

/* swense_hos_init on a caller-owned device workspace: ws (256-byte aligned,
 * on the current device) of ws_bytes >= swense_hos_workspace_bytes.  The
 * handle keeps pointers into it and frees none of it; the caller frees it
 * after swense_hos_destroy.  No later call on the handle allocates device
 * memory except swense_eval_grid (value grids) and, for cells bound by
 * swense_cells_bind, the interpolation scratch (use swense_cells_bind_ws).
 * ENOMEM when ws_bytes is too small, EINVAL when ws is null or misaligned. */
int swense_hos_init_ws(const swense_hos_desc* d, const double* eta0, const double* phis0, int layout,
                       void* stream, void* ws, size_t ws_bytes, swense_hos** out);

/* Replace the state (host arrays in `layout`) and set the time to t. */
int swense_hos_set_state(swense_hos* h, const double* eta, const double* phis, int layout, double t);

/* ---- HOS step (Sec. 3.1.2) -------------------------------------------- */

/* Advance nsteps classical RK4 steps of size dt.  Asynchronous. */
int swense_hos_step(swense_hos* h, int nsteps);

/* Advance by a time tau with nsub integrating-factor (Lawson) RK4 substeps:
 * classical RK4 on the state expressed in the frame of the exact linear
 * evolution (per mode rotation with omega^2 = g k tanh(kh)), so that only the
 * nonlinear part of the right-hand side of Sec. 3.1.2 is integrated
 * numerically.  A coarse step for the surrogate's base prediction; the
 * reference integrator stays swense_hos_step.  Asynchronous. */
int swense_hos_step_exp(swense_hos* h, double tau, int nsub);

/* Copy the state to host arrays in `layout` (eta, phis may be NULL) and the
 * time to *t (may be NULL).  Synchronises the handle's stream.  Returns
 * EUNSTABLE if the state holds a non-finite value. */
int swense_hos_get_state(swense_hos* h, double* eta, double* phis, double* t, int layout);

/* Right-hand side of the evolution equations at the current state, as half
 * spectra (host outputs).  Synchronises. */
int swense_hos_rhs(swense_hos* h, double* eta_t_hat, double* phis_t_hat);

/* Mean-level modal amplitudes of the potential A (Sec. 3.1, 3.2) and of its
 * time derivative A_t, plus eta_t, as half spectra (host outputs; any may be
 * NULL).  Synchronises. */
int swense_hos_modes(swense_hos* h, double* a_hat, double* a_t_hat, double* eta_t_hat);

/* Choice of the product-grid length for a realisation of descriptor d
 * (dealias 1 or 2): when the two lengths differ, one HOS step of each is
 * timed (nsteps steps after one warm-up, on a scratch realisation of zero
 * state, with hipEvents on `stream`) and *dealias receives the faster one
 * (1 when they are the same length); ms (may be NULL) receives both times per
 * step, -1 when not timed.  Allocates and frees device memory.  Synchronises. */
int swense_hos_tune_padding(const swense_hos_desc* d, int nsteps, void* stream, int* dealias, double* ms);

/* Energy 1/2 int phis eta_t dA + 1/2 g int eta^2 dA.  Synchronises. */
int swense_hos_energy(swense_hos* h, double* energy);

/* ---- regular waves: stream-function theory (Sec. 3.1.1, 3.2.1) --------- */

typedef struct swense_stream_desc {
  double depth;       /* d > 0 (use a large kd for deep water)                 */
  double height;      /* crest-to-trough height H > 0                          */
  double wavelength;  /* L = 2 pi / k                                          */
  double g, rho;      /* gravity, water density                                */
  int n;              /* Fourier components N, 2..64                           */
} swense_stream_desc;

/* Solve the 2D steady regular wave (Fourier approximation of the stream
 * function in the frame moving with the wave, no mean Eulerian current) on the
 * host.  sol (host, 2N + 4 doubles) receives eta at the N + 1 surface points
 * X_m = m L / (2N) from crest to trough (above the mean level), B_1..B_N, the
 * phase speed c, the volume flux Q and the Bernoulli constant R (moving frame).
 * Any consistent units (SI or nondimensional): Newton's method runs on the
 * system scaled to g = k = 1 and converges to residuals of ~1e-14 relative to
 * each equation's terms.  Returns SWENSE_EINVAL for bad sizes and
 * SWENSE_EUNSTABLE if Newton's method does not converge (e.g. a wave beyond
 * breaking). */
int swense_stream_solve(const swense_stream_desc* d, double* sol);

/* Fields of `mask` at n points and time t for a solved wave travelling in +x
 * (crest at x = c t): xyz device FP64 [3][n] (y ignored); out device FP64
 * [F][n], fields in bit order (v and v_t are zero); p = rho (R - c^2/2) -
 * rho (phi_t + |u|^2/2 + g z), zero on the free surface.  stream: a
 * hipStream_t (NULL: the default stream).  Asynchronous. */
int swense_stream_eval(const swense_stream_desc* d, const double* sol, double t, long long n, const double* xyz,
                       unsigned mask, double* out, void* stream);

/* ---- evaluation between two outputs of the wave model ------------------- */

/* Record A, A_t, eta and eta_t of the current state and its time as the start
 * of an interval (e.g. before advancing the wave model by one step).
 * Asynchronous. */
int swense_hos_snapshot(swense_hos* h);

/* Evaluate at time t instead of the current time: swense_eval_grid,
 * swense_interp_cells, swense_interp_divergence, swense_fv_divergence and
 * swense_eval_points_direct then read spectra interpolated to t by cubic
 * Hermite interpolation in time of (A, A_t) and (eta, eta_t) between the
 * snapshot and the current state (the CFD step is shorter than the wave
 * model's, Sec. 4.3; the paper does not say how the fields are taken in
 * between).  t must lie in [snapshot time, current time]; t equal to the
 * current time (or any change of the state, or swense_interp_step) returns
 * to the current state.  SWENSE_EINVAL without an earlier snapshot.
 * Asynchronous. */
int swense_hos_set_eval_time(swense_hos* h, double t);

/* ---- evaluation on the intermediate grid (Sec. 3.2.2, 3.2.4, 3.3) ------ */

/* Fields of `mask` at the window nodes of every layer.  out: device FP32,
 * volume fields as [F][nl][wy][wx], then surface fields (ETA, ETA_T) as
 * [wy][wx] each, in field-bit order.  Asynchronous. */
int swense_eval_grid(swense_hos* h, const swense_grid_desc* gd, unsigned mask, float* out);

/* Number of floats swense_eval_grid writes for (gd, mask). */
size_t swense_eval_grid_size(const swense_hos* h, const swense_grid_desc* gd, unsigned mask);

/* ---- direct analytical evaluation (Sec. 3.1.1, 3.2.1) ------------------- */

/* The fields of `mask` at n arbitrary points by the modal sums themselves
 * (every mode at every point, FP64 throughout; cost modes x points - an
 * exact reference for the grid and interpolation path, or for small point
 * sets).  xyz: device FP64 [3][n] (x row, y row, z row); any z, including
 * above the mean level (the continued fields).  out: device FP64 [F][n] in
 * point order, fields in bit order.  Uses the mean-level modes of the
 * current state (computed if stale).  Asynchronous on the handle's stream. */
int swense_eval_points_direct(swense_hos* h, long long n, const double* xyz, unsigned mask, double* out);

/* ---- interpolation to cell centres (Sec. 3.2.2) ------------------------ */

/* Bind a static point cloud to a grid: xyz is device FP64 [3][n] (x row, y
 * row, z row).  Each point's stencil (periodic cubic spline horizontally on
 * the grid nodes, 4-point Lagrange vertically on the layers) is located once
 * here.  Points whose stencil leaves the window or whose z lies outside
 * [z_0, z_nl-1] are flagged out of range.  The grid descriptor (and its z
 * array) is copied.  Synchronises. */
int swense_cells_bind(swense_hos* h, const swense_grid_desc* gd, long long n, const double* xyz,
                      swense_cells** out);

/* Bytes of device workspace for swense_cells_bind_ws: n points bound to the
 * grid gd and interpolated with field masks within `mask` (Sec. 3.2.2): the
 * per-point stencil records, the coefficient grid of those fields on the
 * window, the evaluation rows, the DFT basis and the grid's twiddle tables.
 * An upper bound that needs no binning (one column and one tile per point at
 * most, skeleton coefficients for every layer). */
int swense_cells_workspace_bytes(swense_hos* h, const swense_grid_desc* gd, long long n, unsigned mask,
                                 size_t* bytes);

/* swense_cells_bind on a caller-owned device workspace: ws (256-byte
 * aligned, current device) of ws_bytes >= swense_cells_workspace_bytes for
 * the same (gd, n, mask).  Every device buffer of the handle and of its
 * interpolation calls (swense_interp_cells, swense_interp_step,
 * swense_interp_divergence) is carved from it, so those calls allocate
 * nothing; a call whose mask needs more coefficient fields than `mask`
 * returns ENOMEM.  The handle frees none of it.  Synchronises.  ENOMEM when
 * ws_bytes is too small, EINVAL on a null or misaligned ws or a bad mask. */
int swense_cells_bind_ws(swense_hos* h, const swense_grid_desc* gd, long long n, const double* xyz, unsigned mask,
                         void* ws, size_t ws_bytes, swense_cells** out);

/* Interpolate the fields of `mask` at the bound points of the current state.
 * out: device FP32 [F][n] in the caller's point order (field-bit order).
 * Out-of-range points get NaN; their count goes to *n_out_of_range if that
 * pointer is non-NULL (which synchronises) and the call then returns ERANGE
 * when the count is non-zero. */
int swense_interp_cells(swense_hos* h, swense_cells* c, unsigned mask, float* out,
                        long long* n_out_of_range);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * interpolation as swense_interp_cells - same kernels, same results - with
 * every scratch buffer (the coefficient grid, the evaluation rows and the
 * DFT basis) carved from one fixed device array of 128 MiB per GPU, held by
 * the library until the process ends.  Calls no hipMalloc, hipFree or
 * allocating library routine: the cells' twiddle tables are made by
 * swense_cells_bind, the rest lives in the handle since swense_hos_init.  A
 * call needing more scratch than 128 MiB (window nodes x layers x fields,
 * e.g. about a 216 x 216 window of 48 layers and 11 fields) returns
 * SWENSE_ENOMEM before any launch.  Every call on one GPU shares that GPU's
 * array and leaves its contents behind (nothing in it needs to start at
 * zero); calls that overlap on one GPU - from several handles or streams -
 * race on it and must be serialised by the caller.  Arguments, ownership and
 * the other error codes as for swense_interp_cells. */
int swense_interp_cells_noalloc(swense_hos* h, swense_cells* c, unsigned mask, float* out,
                                long long* n_out_of_range);

/* Divergence diagnostic (Sec. 3.2.3) at the bound points: du/dx + dv/dy +
 * dw/dz of the interpolant (device FP32 [n], caller order).  Asynchronous. */
int swense_interp_divergence(swense_hos* h, swense_cells* c, float* div);

/* Finite-volume divergence of the interpolated velocity (Sec. 3.2.3) on a
 * structured box mesh with increasing cell edges xe[nx+1], ye[ny+1] (3D; in
 * 2D ny = 1 and ye may be NULL) and ze[nz+1] (host FP64): the velocity of the
 * interpolant on the grid gd (as swense_interp_cells) at every face centre,
 * then per cell div = sum over its faces of u_f . A_f / V.  div: device FP32
 * [nz][ny][nx], x fastest.  *rms and *maxabs (may be NULL) receive the RMS and
 * the largest magnitude over the cells.  The face centres are bound and
 * released inside the call (a diagnostic, not a per-step path); every face
 * centre must lie inside the window and layers (else SWENSE_EINVAL).
 * Synchronises. */
int swense_fv_divergence(swense_hos* h, const swense_grid_desc* gd, const double* xe, int nx, const double* ye,
                         int ny, const double* ze, int nz, float* div, double* rms, double* maxabs);

/* ---- cell-side use of the incident fields (Sec. 2.1.3, 3.2.2, 4.2) ------ */

/* Incident volume fraction of n cells (Sec. 3.2.2, the VOF field rebuilt
 * from eta_I): the share of each cell's height [zc - dz/2, zc + dz/2] below
 * the elevation eta at its centre, clamped to [0, 1] (a flat interface
 * across the cell).  eta, dz, alpha: device FP32 [n]; zc: device FP64 [n]
 * (e.g. the z row of the bound coordinates).  Asynchronous. */
int swense_cells_alpha(swense_hos* h, long long n, const float* eta, const double* zc, const float* dz,
                       float* alpha);

/* Modified incident pressure (Sec. 2.1.3, Eq. pIStar): pstar = rho p / rho_I
 * with the mixture density rho = alpha rho_I + (1 - alpha) rho_air and rho_I
 * the handle's water density.  p, alpha, pstar: device FP32 [n] (pstar may
 * alias p).  Asynchronous. */
int swense_cells_pstar(swense_hos* h, long long n, const float* p, const float* alpha, double rho_air, float* pstar);

/* Relaxation zones (Sec. 4.2, Eq. weightFunction, swUcRelax, swVOFRelax), in
 * place: with omega = -2 x^3 + 3 x^2 of the zone coordinate x (clamped to
 * [0, 1]; 0 at the inner boundary, 1 at the outer one), alpha <- omega
 * alpha_i + (1 - omega) alpha and each of the ncomp (<= 3) complementary
 * velocity rows uc[c][n] <- (1 - omega) uc.  Cells with omega = 0 are left
 * untouched.  alpha may be NULL (velocity only); uc may be NULL with
 * ncomp = 0.  All device FP32.  Asynchronous. */
int swense_cells_relax(swense_hos* h, long long n, int ncomp, const float* x, const float* alpha_i, float* alpha,
                       float* uc);

/* One CFD coupling step in one call (Sec. 4.3: the incident fields at the
 * current time are mapped to the cells, then the wave model advances): the
 * fields of the current state, as swense_interp_cells would produce them, go
 * to `out` while the state advances by nsteps RK4 steps; the evaluation and
 * interpolation run on an internal stream concurrently with the step, reading
 * the modes and a copy of eta taken at the start.  The whole call is ordered
 * on the handle's stream (work issued after it waits for both halves).
 * Asynchronous. */
int swense_interp_step(swense_hos* h, swense_cells* c, unsigned mask, float* out, int nsteps);

/* ---- batched realisations ---------------------------------------------- */

typedef struct swense_batch swense_batch; /* many realisations, one captured graph (opaque) */

/* Batch n independent realisations of any sizes: one swense_batch_run advances
 * every hos[i] by nsteps RK4 steps and, where cells[i] is non-NULL,
 * interpolates masks[i] (NULL: all fields) into the device buffer outs[i]
 * ([F][n_i] FP32).  The whole batch is captured once as a HIP graph whose
 * branches (realisations spread over K worker streams) run concurrently;
 * replays record nothing new.  Creation runs the work once eagerly to size
 * every workspace and then restores the states, so the realisations are
 * unchanged when it returns.  stream: the stream graph launches go to.
 * The handles must stay alive and must not be used concurrently with the
 * batch.  (Batched execution of uneven realisations; no passage of the paper
 * - the paper runs one wave model.) */
int swense_batch_create(swense_hos* const* hos, swense_cells* const* cells, const unsigned* masks,
                        float* const* outs, int n, int nsteps, void* stream, swense_batch** out);

/* One graph launch (asynchronous on the batch stream). */
int swense_batch_run(swense_batch* b);

/* Choose K (concurrent branches) by timing candidate graphs with HIP events,
 * or take it from the JSON cache file `cache_path` (may be NULL) keyed by the
 * GPU architecture and the batch's shapes; stores new choices there.  States
 * are restored after timing.  *chosen: K; *best_ms: measured ms per launch
 * (-1 when taken from the cache). */
int swense_batch_autotune(swense_batch* b, const char* cache_path, int* chosen, double* best_ms);

const char* swense_batch_last_error(const swense_batch* b);
void swense_batch_destroy(swense_batch* b);

/* ---- per-kernel timing -------------------------------------------------- */

/* Kernel classes timed by the profiler. */
enum {
  SWENSE_K_YINV = 0,      /* HOS inverse y transforms                   */
  SWENSE_K_XPASS = 1,     /* HOS fused x pass (products)                */
  SWENSE_K_YFWD = 2,      /* HOS forward y transforms + RK4 epilogue    */
  SWENSE_K_YINV_EVAL = 3, /* grid evaluation, y transforms              */
  SWENSE_K_XEVAL = 4,     /* grid evaluation, x transforms (volume)     */
  SWENSE_K_XEVAL_SURF = 5,/* grid evaluation, x transforms (surface)    */
  SWENSE_K_INTERP = 6,    /* interpolation gather                       */
  SWENSE_K_INTERP_DIV = 7,/* divergence of the interpolant              */
  SWENSE_K_BIND = 8,      /* point binding                              */
  SWENSE_K_AUX = 9,       /* copies, fills, state conversion            */
  SWENSE_K_COUNT = 10
};

/* Enable (1) or disable (0) per-kernel timing on the handle's stream: while
 * enabled, every launch is bracketed by a pair of HIP events.  Enabling
 * clears the accumulated records. */
int swense_profile_enable(swense_hos* h, int enable);

/* Synchronise and return the summed duration (ms) and the launch count of
 * kernel class `kernel` recorded since profiling was enabled. */
int swense_profile_read(swense_hos* h, int kernel, double* total_ms, long long* count);

/* Compulsory HBM bytes (every distinct input read once, every output written
 * once, by each launch's own arguments) of the launches of kernel class
 * `kernel` issued while profiling was enabled.  Counted for the HOS classes
 * (YINV, XPASS, YFWD), the evaluation classes (YINV_EVAL: spectra read, window
 * rows written; XEVAL: window rows read, grid written) and the gather
 * (INTERP: per-point stencil data and outputs, grid read once); 0 for the
 * others. */
int swense_profile_bytes(swense_hos* h, int kernel, double* bytes);

/* Algorithmic HBM bytes of the same launches under the two-pass transform
 * model: every real two-dimensional transform of the HOS step (Sec. 3.1.2:
 * the spectral derivatives, the series terms and the right-hand side, each
 * a real field on the padded product grid) streams its field once per pass,
 * read and written, i.e. 2 x (4 or 8) bytes per product-grid point in each of
 * its y and x passes.  YINV and YFWD count their jobs, XPASS its inverse
 * inputs plus forward outputs; the evaluation classes count every (field,
 * layer) job on the whole refined grid (Sec. 3.2.4); the gather counts 16 B of
 * coordinates and index plus 4 B per output field per point, and the grid
 * read once.  0 for the other classes. */
int swense_profile_transform_bytes(swense_hos* h, int kernel, double* bytes);

/* ---- host self-check ----------------------------------------------------- */

/* Host-only consistency check of launch geometry (no device work): for every
 * even mode count up to max_nx, the DFT coefficient pass of the evaluation
 * reads no row of its basis operand past the rows allocated per node tile.
 * Returns 0, or the first mode count that fails. */
int swense_selfcheck_launch_geometry(int max_nx);

/* ---- lifetime ---------------------------------------------------------- */
void swense_hos_destroy(swense_hos* h);
void swense_cells_destroy(swense_cells* c);
const char* swense_last_error(const swense_hos* h);
const char* swense_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SWENSE_H */
