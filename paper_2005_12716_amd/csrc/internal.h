// Internal state of a realisation handle and the launch helpers shared by
// the HOS and reconstruction translation units.
#pragma once

#include <hip/hip_ext.h>

#include "common.h"
#include "swense_surrogate.h"

// Symbol kinds multiplied into a half spectrum before the y transform.
enum SymKind { SYM_ONE = 0, SYM_IKX = 1, SYM_IKY = 2, SYM_DZ = 3, SYM_EVAL = 4 };

// Field-in-layer description of an evaluation symbol: vertical factor
// (0: C = cosh k(z+h)/cosh kh, 1: S = sinh k(z+h)/cosh kh, 2: none) times
// multiplier (0: 1, 1: i kx, 2: i ky, 3: |k|), optional B-spline prefilter.
struct EvalSym {
  int vf;
  int mult;
  int pre;
  int gx, gy;
};

struct YInvJob {
  const cd* src;  // [ny][nxh] FP64 half spectrum
  void* dst;      // [nrows][nxh] complex, transform precision
  int sym;
  int jpow;
  double z;
  EvalSym ev;
};

constexpr int kMaxYJobs = 16;
struct YInvArgs {
  int njobs;
  YInvJob job[kMaxYJobs];
};

// Roles of an input field of the fused x pass (see the HOS x-pass kernel).
enum XRole { XR_NONE = 0, XR_ETA = 1, XR_GRADPAIR = 2, XR_G = 3, XR_ETAT = 4, XR_PHIT = 5 };
enum XStage { XS_SERIES = 0, XS_FINAL = 1, XS_FTILDE = 2 };

struct XIn {
  const void* src;  // [Py][nxh] complex rows (x still spectral)
  int dx;           // multiply by i kx before the x transform
  int role;
  int slot;         // accumulator slot written by XR_G
  int pw;           // power of eta for XR_G
  int wi;           // index of the W order (or series sum) XR_G adds to
};

constexpr int kMaxXIn = 24;
constexpr int kMaxM = 8;
struct XArgs {
  int nin;
  XIn in[kMaxXIn];
  int stage;
  int M;
  int nslots;
  int ng;  // final stage on rows of 3Q points: leading inputs before the gradient pairs
  int s_eta, s_ge2, s_dot, s_gp2, s_etat, s_phit;
  int s_w[kMaxM];
  void* out0;
  void* out1;
};

// Epilogue of the forward y transform.
// YE_NL_*: store the nonlinear part of the right-hand side only (kout).
enum YEpi { YE_STORE = 0, YE_RHS_ETA = 1, YE_RHS_PHI = 2, YE_NL_ETA = 3, YE_NL_PHI = 4 };

struct YFwdJob {
  const void* src;  // [Py][nxh] complex rows
  cd* dst;          // [ny][nxh] FP64 (YE_STORE)
  cd* acc;          // accumulate target (YE_STORE) or null
  int acc_mode;     // 0 none, 1 add, 2 assign
  int epi;
};

// RK4 bookkeeping for the right-hand-side epilogue (classical RK4 on the
// spectral state; stage 0 only stores the right-hand side).
struct RkArgs {
  int stage;
  double dt;
  cd* xn[2];         // base state (eta, phis), updated in place at stage 4
  const cd* sin[2];  // stage input state (used by the exact linear part)
  cd* sout[2];       // next stage input
  cd* acc[2];        // k1 + 2 k2 + 2 k3
  cd* kout[2];       // right-hand side output (stage 0)
};

constexpr int kMaxYFwd = 4;
struct YFwdArgs {
  int njobs;
  YFwdJob job[kMaxYFwd];
  RkArgs rk;
};

struct EvalWork;  // reconstruction workspace (evalgrid.hip)

// Per-kernel event timing (enabled on demand).
struct ProfRec {
  int kid;
  hipEvent_t a, b;
};
struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<ProfRec> recs;
  double total_ms[SWENSE_K_COUNT] = {};
  long long count[SWENSE_K_COUNT] = {};
  double bytes[SWENSE_K_COUNT] = {};  // compulsory HBM bytes of the recorded launches
  double tbytes[SWENSE_K_COUNT] = {}; // two-pass transform model: every real transform's product-grid
                                      // field read and written once per pass (per pass 2 x precision B/point)
  hipEvent_t take() {
    if (used == pool.size()) {
      hipEvent_t e;
      SW_HIP(hipEventCreate(&e));
      pool.push_back(e);
    }
    return pool[used++];
  }
  void release() {
    for (auto e : pool) (void)hipEventDestroy(e);
    pool.clear();
    recs.clear();
    used = 0;
  }
};

struct swense_hos {
  swense_hos_desc d{};
  Geom G{};
  hipStream_t st = nullptr;
  bool fp64 = false;
  int Px = 0, Py = 0;
  TwiddleCache tw;
  FftPlan plan_px{}, plan_py{}, plan_nx{}, plan_ny{};
  double t = 0.0;
  long version = 0;        // bumped whenever the state changes
  long modes_version = -1;  // state version the mean-level modes belong to
  long kk_version = -1;     // state version whose right-hand side kk holds
  bool graph_reuse_k = false;  // under capture: first RK stage takes kk (the graph's modes refresh it)
  // concurrent interpolation + step (swense_interp_step): a copy of the
  // surface elevation the evaluation reads while the step advances the state,
  // an auxiliary stream and two events
  cd* eta_snap = nullptr;
  const cd* eta_src = nullptr;  // evaluation source of eta (null: the state)
  // evaluation at a time between a snapshot and the current state
  // (swense_hos_snapshot, swense_hos_set_eval_time): the snapshot's A, A_t,
  // eta, eta_t, the interpolated ones, and the state version they were
  // formed for (a later state change drops them)
  cd* snapm = nullptr;   // [4][nc]
  cd* herm = nullptr;    // [4][nc]
  double snap_t = 0.0;
  bool snap_ok = false;
  bool herm_on = false;
  long herm_version = -1;
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::string err;
  int device = 0;
  bool own_mem = true;  // false: pool, twiddles and snapshot buffers live in a caller's workspace
  // bumped whenever a device buffer that evaluations or interpolations write
  // is reallocated (captured graphs hold the old addresses)
  long scratch_epoch = 0;
  int* flag = nullptr;  // one device int for state checks

  // FP64 spectral buffers, each [ny][nxh]
  size_t nc = 0;
  void* pool = nullptr;  // one allocation carved below
  cd* xn[2]{};
  cd* sa[2]{};
  cd* sb[2]{};
  cd* acc[2]{};
  cd* kk[2]{};            // right-hand side at the current state
  cd* phim[kMaxM + 1]{};  // series modes phi^(m), m >= 2 (index m)
  cd* amod = nullptr;     // A   = sum_m phi^(m)
  cd* atmod = nullptr;    // A_t = sum_m B^(m)
  cd* bm[kMaxM + 1]{};    // series modes of phi_t
  // transform-precision intermediates, each [Py][nxh] complex
  size_t ni = 0;           // elements per intermediate
  void* e_ = nullptr;      // eta
  void* ey_ = nullptr;     // i ky eta
  void* ph_ = nullptr;     // phis
  void* py_ = nullptr;     // i ky phis
  void* gbuf[kMaxM + 1][kMaxM + 2]{};  // g(m, j) = F^-1(Dz^j phi^(m))
  void* q_ = nullptr;      // series product
  void* r0_ = nullptr;     // nonlinear eta_t
  void* r1_ = nullptr;     // nonlinear phis_t
  void* et_ = nullptr;     // eta_t rows
  void* pt_ = nullptr;     // phis_t rows
  // physical staging for state in/out, FP64 [ny][nx] x 2
  double* phys = nullptr;
  EvalWork* ev = nullptr;
  Profiler prof;

  size_t isz() const { return fp64 ? sizeof(cd) : sizeof(cf); }
};

// Launch with optional >64 KB dynamic LDS and per-kernel timing: while the
// handle's profiler is on, the launch carries a start and a stop event that
// the runtime stamps when the kernel itself starts and ends (kernel time, as
// a trace records it, without the launch's queueing).
template <typename... KArgs, typename... Args>
void sw_launch(swense_hos* h, int kid, void (*kernel)(KArgs...), dim3 grid, dim3 block, size_t lds, hipStream_t st,
               Args... args) {
  if (lds > 65536) {
    // once per kernel and size, so that graph capture records launches only
    static thread_local std::map<const void*, size_t> done;
    const void* key = reinterpret_cast<const void*>(kernel);
    auto it = done.find(key);
    if (it == done.end() || it->second < lds) {
      SW_HIP(hipFuncSetAttribute(key, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      done[key] = lds;
    }
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (h->prof.on) SW_HIP(hipStreamIsCapturing(st, &cs));
  if (h->prof.on && cs == hipStreamCaptureStatusNone) {  // launches being captured are not timed
    hipEvent_t a = h->prof.take(), b = h->prof.take();
    h->prof.recs.push_back(ProfRec{kid, a, b});
    hipExtLaunchKernelGGL(kernel, grid, block, (std::uint32_t)lds, st, a, b, 0u, args...);
  } else {
    hipLaunchKernelGGL(kernel, grid, block, lds, st, args...);
  }
  SW_HIP(hipGetLastError());
}

#define SW_LAUNCH(h, kid, kernel, ...) sw_launch((h), (kid), &kernel, __VA_ARGS__)

// ---- launch helpers implemented in hos.hip (templated on precision there)
void launch_yinv(swense_hos* h, const YInvArgs& a, const FftPlan& plan, int nrows, int row0, hipStream_t st);
void launch_modes(swense_hos* h);  // A, A_t, eta_t at the current state (if stale)

// Spectra the evaluation reads: A, A_t, eta, eta_t of the current state, or
// the ones interpolated to the evaluation time set for this state.
inline void eval_sources(const swense_hos* h, const cd** a, const cd** at, const cd** eta, const cd** etat) {
  const bool tset = h->herm_on && h->herm_version == h->version;
  *a = tset ? h->herm : h->amod;
  *at = tset ? h->herm + h->nc : h->atmod;
  *eta = tset ? h->herm + 2 * h->nc : (h->eta_src ? h->eta_src : h->xn[0]);
  *etat = tset ? h->herm + 3 * h->nc : h->kk[0];
}
void set_error(swense_hos* h, const SwenseError& e);
// Physical fields at h->phys ([ny][nx] FP64, eta then phis) -> half spectra
// (e, p); add = true adds them into (e, p) instead of overwriting.
void hos_phys_to_spec(swense_hos* h, cd* e, cd* p, bool add);
// Half spectra (e, p) -> physical fields at h->phys.
void hos_spec_to_phys(swense_hos* h, const cd* e, const cd* p);
void hos_step(swense_hos* h, int nsteps);
// Advance by tau with nsub integrating-factor RK4 substeps (exact linear
// propagation, RK4 on the nonlinear part).
void hos_step_exp(swense_hos* h, double tau, int nsub);
double hos_energy(swense_hos* h);  // synchronises
// Make kk the right-hand side of the current state (evaluates the mean-level
// modes when it is not); asynchronous on h->st.
void hos_prime_rhs(swense_hos* h);
// Network handle accessors (the surrogate runs the network on the HOS stream).
hipStream_t fno_stream(const swense_fno* f);
swense_fno_desc fno_desc_of(const swense_fno* f);

// Device address of the allocation-free interpolation's scratch array on
// device `dev` (interp.hip), looked up once per device; the set-up call is
// made by swense_hos_init with the device current.
void noalloc_scratch_setup(int dev);

// ---- reconstruction (evalgrid.hip)
void eval_release(swense_hos* h);
void check_grid_desc(const swense_hos* h, const swense_grid_desc* gd);
void ensure_device(void** p, size_t* cap, size_t bytes);
// Node-major coefficient grid: per window node K = fv nl + fs floats, volume
// field f of layer l at offset l fv + f (a band of layers holds every field
// contiguously), surface field s at fv nl + s; idx[bit] = field index, -1 when the field is absent (also v, v_t
// in 2D, which are zero).
struct CoefLayout {
  int fv, fs, nl, k;
  int idx[11];
};
CoefLayout coef_layout(swense_hos* h, unsigned cm, int nl);
// Skeleton heights for the vertical factors: the factors C(k, z_l) (and
// S(k, z_l)) of every layer are reproduced, for all |k| of the mode grid, by
// combinations  sum_r T[l][r] C(k, zeta_r)  of r < R skeleton heights chosen
// among the layers, so only R transforms per field are needed.
struct Skel {
  int R;              // 0: not used
  const double* zeta; // device [R]
  const float* tc;    // device [nl][R] for C-type fields (phi, u, v and their time derivatives)
  const float* ts;    // device [nl][R] for S-type fields (w, w_t)
};
// *plane: 0 node-major layout (above), 1 plane layout coef[c][wy][wx] with c
// the same coefficient index (l fv + f, then fv nl + s).
void eval_coef(swense_hos* h, const swense_grid_desc* gd, const double* zdev, unsigned cm, float* coef,
               const Skel* sk, int* plane);
size_t coef_floats(swense_hos* h, const swense_grid_desc* gd, unsigned cm);
// Scratch bytes one coefficient evaluation needs: the y-pass rows and (with
// skeleton heights) the DFT basis.
void eval_scratch_need(swense_hos* h, const swense_grid_desc* gd, unsigned cm, int skel_r, size_t* inter,
                       size_t* basis);
// Evaluations on this handle take their rows (inter bytes) and basis (basis
// bytes after them) from `base` instead of the handle's own buffers; a null
// base restores those.
void eval_set_scratch(swense_hos* h, void* base, size_t inter, size_t basis);
// Evaluations on this handle take the twiddle tables of grid lengths gx, gy
// from twx, twy (null: the handle's cache).
void eval_set_twiddles(swense_hos* h, int gx, void* twx, int gy, void* twy);

// run a body and convert exceptions to error codes
template <typename F>
int guarded(swense_hos* h, F&& f) {
  try {
    return f();
  } catch (const SwenseError& e) {
    if (h) set_error(h, e);
    return e.code;
  } catch (const std::exception& e) {
    if (h) set_error(h, SwenseError{SWENSE_EHIP, e.what()});
    return SWENSE_EHIP;
  }
}
