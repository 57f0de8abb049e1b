// Rollout of a realisation by the spectral neural operator with the HOS step
// as fallback and judge: per call the state is saved, the network's residual
// is added to the exact linear propagation of the saved state (FP64,
// spectral), cheap guards run (non-finite values, energy change), and every
// A-th call (or a guarded one) HOS re-runs the same steps from the saved
// state, the error is measured and the HOS state is kept.
#include <cmath>
#include <cstring>
#include <string>

#include "internal.h"

struct swense_surrogate {
  swense_hos* h = nullptr;
  swense_fno* f = nullptr;
  swense_surrogate_desc d{};
  std::string err;
  cd* backup[2]{};
  cd* sur[2]{};
  float* x = nullptr;
  float* y = nullptr;
  double* sums = nullptr;  // 4 reduction slots
  int* bad = nullptr;
  void* mem = nullptr;
  int in_channels = 2;     // network input: 2 (state) or 4 (state, linear propagation)
  int cool = 0;            // cool-down calls left
  int trust = 0;           // judged calls passed in a row
  long long nsur = 0;      // network calls so far (audit counter)
  double drift = 0.0;      // estimated error accumulated by unjudged calls since the reset
  double est = -1.0;       // largest judged error since the reset (< 0: none yet)
  bool spent = false;      // drift bound reached: HOS alone until the next reset
};

// network output without the pre-activations a backward pass would need
__attribute__((visibility("hidden"))) int fno_forward_infer(swense_fno* f, const float* x, float* y, int batch);

namespace {

__device__ __forceinline__ double wavenumber(const Geom& G, int p, int q) {
  const double kx = 2.0 * M_PI * (double)p / G.lx;
  const double ky = G.ny > 1 ? 2.0 * M_PI * (double)signed_q(q, G.ny) / G.ly : 0.0;
  return sqrt(kx * kx + ky * ky);
}

// Exact linear propagation of the half spectra over tau (mode by mode).
__global__ void k_linear(const cd* __restrict__ e, const cd* __restrict__ p, cd* __restrict__ oe,
                         cd* __restrict__ op, Geom G, double tau) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)G.ny * G.nxh) return;
  const int q = (int)(i / G.nxh), pp = (int)(i % G.nxh);
  const double k = wavenumber(G, pp, q);
  const cd a = e[i], b = p[i];
  if (k == 0.0) {
    oe[i] = a;
    op[i] = b - cscale(a, G.g * tau);
    return;
  }
  const double kt = G.depth > 0.0 ? k * tanh(k * G.depth) : k;
  const double w = sqrt(G.g * kt);
  const double c = cos(w * tau), s = sin(w * tau);
  oe[i] = cscale(a, c) + cscale(b, kt * s / w);
  op[i] = cscale(b, c) - cscale(a, G.g * s / w);
}

__global__ void k_features(const double* __restrict__ pe, const double* __restrict__ pp, float* __restrict__ x,
                           long long np, double ie, double ip) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  x[i] = (float)(pe[i] * ie);
  x[np + i] = (float)(pp[i] * ip);
}

__global__ void k_residual_in(const float* __restrict__ y, double* __restrict__ pe, double* __restrict__ pp,
                              long long np, double ae, double ap) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  pe[i] = ae * (double)y[i];
  pp[i] = ap * (double)y[np + i];
}

__global__ void k_target(const float* __restrict__ xn, const float* __restrict__ lin, float* __restrict__ t,
                         long long n, float inv_rho) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) t[i] = (xn[i] - lin[i]) * inv_rho;
}

__global__ void k_keep_mean(cd* e, const cd* from) { e[0] = from[0]; }

__global__ void k_zero(double* a, int n, int* flag) {
  const int i = threadIdx.x;
  if (i < n) a[i] = 0.0;
  if (i == 0 && flag) *flag = 0;
}

__global__ void k_finite2(const cd* a, const cd* b, size_t n, int* bad) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && (!isfinite(a[i].x) || !isfinite(a[i].y) || !isfinite(b[i].x) || !isfinite(b[i].y))) atomicOr(bad, 1);
}

// Weighted (Parseval on the half spectrum) sums |a - b|^2 and |b|^2 for the
// two fields: sums[0..1] for eta, sums[2..3] for phis.
__global__ void __launch_bounds__(256) k_relerr(const cd* a0, const cd* a1, const cd* b0, const cd* b1, int nxh,
                                                size_t n, double* sums) {
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double w = (i % nxh) == 0 ? 1.0 : 2.0;
    const cd d0 = a0[i] - b0[i], d1 = a1[i] - b1[i];
    s[0] += w * (d0.x * d0.x + d0.y * d0.y);
    s[1] += w * (b0[i].x * b0[i].x + b0[i].y * b0[i].y);
    s[2] += w * (d1.x * d1.x + d1.y * d1.y);
    s[3] += w * (b1[i].x * b1[i].x + b1[i].y * b1[i].y);
  }
  __shared__ double red[4][256];
  for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = s[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) atomicAdd(&sums[threadIdx.x], red[threadIdx.x][0]);
}

__global__ void k_copy2(const cd* __restrict__ a, const cd* __restrict__ b, cd* __restrict__ oa, cd* __restrict__ ob,
                        size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    oa[i] = a[i];
    ob[i] = b[i];
  }
}

unsigned nblk(long long n) { return (unsigned)((n + 255) / 256); }

void copy_state(swense_surrogate* s, const cd* a, const cd* b, cd* oa, cd* ob) {
  hipLaunchKernelGGL(k_copy2, dim3(nblk((long long)s->h->nc)), dim3(256), 0, s->h->st, a, b, oa, ob, s->h->nc);
  SW_HIP(hipGetLastError());
}

// scaled physical fields of the spectra (e, p) into x [2][n][n]
void features_of(swense_surrogate* s, const cd* e, const cd* p, float* x) {
  swense_hos* h = s->h;
  hos_spec_to_phys(h, e, p);
  const long long np = (long long)h->G.nx * h->G.ny;
  hipLaunchKernelGGL(k_features, dim3(nblk(np)), dim3(256), 0, h->st, h->phys, h->phys + np, x, np,
                     1.0 / s->d.sigma_eta, 1.0 / s->d.sigma_phi);
  SW_HIP(hipGetLastError());
}

double tau_of(const swense_surrogate* s) { return (double)s->d.stride_s * s->h->d.dt; }

void linear_into(swense_surrogate* s, const cd* e, const cd* p, cd* oe, cd* op) {
  swense_hos* h = s->h;
  hipLaunchKernelGGL(k_linear, dim3(nblk((long long)h->nc)), dim3(256), 0, h->st, e, p, oe, op, h->G, tau_of(s));
  SW_HIP(hipGetLastError());
}

// State <- B(from): linear propagation, or integrating-factor RK4 substeps
// run in place on the state (the caller restores the time).
void base_into_state(swense_surrogate* s, const cd* e, const cd* p) {
  swense_hos* h = s->h;
  if (s->d.base_substeps <= 0) {
    linear_into(s, e, p, h->xn[0], h->xn[1]);
    return;
  }
  if (e != h->xn[0]) copy_state(s, e, p, h->xn[0], h->xn[1]);
  h->version++;
  hos_step_exp(h, tau_of(s), s->d.base_substeps);
}

bool state_finite(swense_surrogate* s) {
  swense_hos* h = s->h;
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, h->st, s->sums, 0, s->bad);
  hipLaunchKernelGGL(k_finite2, dim3(nblk((long long)h->nc)), dim3(256), 0, h->st, h->xn[0], h->xn[1], h->nc,
                     s->bad);
  SW_HIP(hipGetLastError());
  int hb = 0;
  SW_HIP(hipMemcpyAsync(&hb, s->bad, sizeof(int), hipMemcpyDeviceToHost, h->st));
  SW_HIP(hipStreamSynchronize(h->st));
  return hb == 0;
}

// relative L2 error of (a0, a1) against the current HOS state, max over fields
double rel_error(swense_surrogate* s, const cd* a0, const cd* a1) {
  swense_hos* h = s->h;
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, h->st, s->sums, 4, nullptr);
  const unsigned blocks = std::min<unsigned>(nblk((long long)h->nc), 1024);
  hipLaunchKernelGGL(k_relerr, dim3(blocks), dim3(256), 0, h->st, a0, a1, h->xn[0], h->xn[1], h->G.nxh, h->nc,
                     s->sums);
  SW_HIP(hipGetLastError());
  double hs[4];
  SW_HIP(hipMemcpyAsync(hs, s->sums, sizeof(hs), hipMemcpyDeviceToHost, h->st));
  SW_HIP(hipStreamSynchronize(h->st));
  const double e0 = std::sqrt(hs[0] / std::max(hs[1], 1e-300));
  const double e1 = std::sqrt(hs[2] / std::max(hs[3], 1e-300));
  if (!(e0 == e0) || !(e1 == e1)) return NAN;
  return std::max(e0, e1);
}

// s HOS steps from the current state, time advanced step by step as in HOS
void hos_call(swense_surrogate* s) { hos_step(s->h, s->d.stride_s); }

// One call of the learned step (or, with base_only, of the base prediction
// alone); judged when forced, guarded, on probation or the A-th.
void network_call(swense_surrogate* s, swense_surrogate_stats* st, bool force_audit) {
  swense_hos* h = s->h;
  const double t0 = h->t;
  copy_state(s, h->xn[0], h->xn[1], s->backup[0], s->backup[1]);
  const bool eguard = s->d.energy_tol > 0.0;
  const double E0 = eguard ? hos_energy(h) : 0.0;
  const long long np = (long long)h->G.nx * h->G.ny;
  if (s->d.base_only) {
    base_into_state(s, s->backup[0], s->backup[1]);
  } else {
    features_of(s, s->backup[0], s->backup[1], s->x);
    base_into_state(s, s->backup[0], s->backup[1]);
    if (s->in_channels == 4) features_of(s, h->xn[0], h->xn[1], s->x + 2 * np);
    const int rc = fno_forward_infer(s->f, s->x, s->y, 1);
    if (rc != SWENSE_OK) throw SwenseError{rc, "network forward failed"};
    hipLaunchKernelGGL(k_residual_in, dim3(nblk(np)), dim3(256), 0, h->st, s->y, h->phys, h->phys + np, np,
                       s->d.rho * s->d.sigma_eta, s->d.rho * s->d.sigma_phi);
    SW_HIP(hipGetLastError());
    hos_phys_to_spec(h, h->xn[0], h->xn[1], true);
  }
  hipLaunchKernelGGL(k_keep_mean, dim3(1), dim3(1), 0, h->st, h->xn[0], s->backup[0]);
  SW_HIP(hipGetLastError());
  double t = t0;
  for (int i = 0; i < s->d.stride_s; ++i) t += h->d.dt;
  h->t = t;
  h->version++;
  bool guard = !state_finite(s);
  if (!guard && eguard) {
    const double E1 = hos_energy(h);
    guard = !(std::fabs(E1 - E0) <= s->d.energy_tol * std::fabs(E0));
  }
  st->surrogate_calls++;
  s->nsur++;
  const bool audit = force_audit || guard || s->trust < s->d.probation || (s->nsur % s->d.audit_every == 0);
  if (!audit) {
    // an unjudged call adds the largest judged error since the reset to the
    // estimate of the error accumulated against plain HOS
    if (s->est > 0.0) s->drift += s->est;
    return;
  }
  // judge: HOS from the saved state; its result is kept
  copy_state(s, h->xn[0], h->xn[1], s->sur[0], s->sur[1]);
  copy_state(s, s->backup[0], s->backup[1], h->xn[0], h->xn[1]);
  h->t = t0;
  h->version++;
  hos_call(s);
  const double err = rel_error(s, s->sur[0], s->sur[1]);
  st->audits++;
  st->last_audit_err = err;
  if (err == err && err > st->max_audit_err) st->max_audit_err = err;
  s->est = err == err ? std::max(s->est, err) : INFINITY;
  if (guard) st->guard_trips++;
  if (guard || !(err <= s->d.tol)) {
    st->fallbacks++;
    s->cool = s->d.cooldown;
    s->trust = 0;
  } else {
    s->trust++;
  }
}

template <typename F>
int guarded_s(swense_surrogate* s, F&& fn) {
  try {
    return fn();
  } catch (const SwenseError& e) {
    if (s) s->err = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    if (s) s->err = e.what();
    return SWENSE_EHIP;
  }
}

}  // namespace

extern "C" {

int swense_surrogate_create(swense_hos* h, swense_fno* f, const swense_surrogate_desc* d, swense_surrogate** out) {
  if (!out || !h || !f || !d) return SWENSE_EINVAL;
  *out = nullptr;
  swense_surrogate* s = new swense_surrogate();
  const int rc = guarded_s(s, [&] {
    const swense_fno_desc fd = fno_desc_of(f);
    SW_REQUIRE(h->d.dim == 3 && h->G.nx == fd.n && h->G.ny == fd.n, "realisation must be n x n with the network's n");
    SW_REQUIRE(fno_stream(f) == h->st, "network and realisation must share one stream");
    SW_REQUIRE(fd.in_channels == 2 || fd.in_channels == 4, "network input must have 2 or 4 channels");
    s->in_channels = fd.in_channels;
    SW_REQUIRE(d->stride_s >= 1 && d->audit_every >= 1 && d->cooldown >= 0 && d->probation >= 0 &&
                   d->base_substeps >= 0 && d->base_substeps <= 64,
               "stride, audit period, cool-down, probation or base substeps");
    SW_REQUIRE(d->sigma_eta > 0.0 && d->sigma_phi > 0.0 && d->rho > 0.0 && d->tol >= 0.0, "scales and tol");
    SW_REQUIRE(d->base_only == 0 || d->base_only == 1, "base_only must be 0 or 1");
    s->h = h;
    s->f = f;
    s->d = *d;
    const size_t nc = h->nc, np = (size_t)fd.n * fd.n;
    const size_t bytes = 4 * nc * sizeof(cd) + 6 * np * sizeof(float) + 8 * sizeof(double) + 256 * 8;
    SW_HIP(hipMalloc(&s->mem, bytes));
    char* p = reinterpret_cast<char*>(s->mem);
    auto take = [&](size_t b) {
      void* r = p;
      p += (b + 255) & ~size_t(255);
      return r;
    };
    for (int k = 0; k < 2; ++k) s->backup[k] = reinterpret_cast<cd*>(take(nc * sizeof(cd)));
    for (int k = 0; k < 2; ++k) s->sur[k] = reinterpret_cast<cd*>(take(nc * sizeof(cd)));
    s->x = reinterpret_cast<float*>(take(4 * np * sizeof(float)));
    s->y = reinterpret_cast<float*>(take(2 * np * sizeof(float)));
    s->sums = reinterpret_cast<double*>(take(4 * sizeof(double)));
    s->bad = reinterpret_cast<int*>(take(sizeof(int)));
    SW_REQUIRE(p <= reinterpret_cast<char*>(s->mem) + bytes, "internal carve overflow");
    return (int)SWENSE_OK;
  });
  if (rc != SWENSE_OK) {
    swense_surrogate_destroy(s);
    return rc;
  }
  *out = s;
  return SWENSE_OK;
}

int swense_surrogate_features(swense_surrogate* s, float* x, float* lin) {
  if (!s || !x) return SWENSE_EINVAL;
  return guarded_s(s, [&] {
    swense_hos* h = s->h;
    features_of(s, h->xn[0], h->xn[1], x);
    if (lin) {
      if (s->d.base_substeps <= 0) {
        linear_into(s, h->xn[0], h->xn[1], s->sur[0], s->sur[1]);
        features_of(s, s->sur[0], s->sur[1], lin);
      } else {
        // base step on the state, then the state back (bit for bit)
        const double t0 = h->t;
        copy_state(s, h->xn[0], h->xn[1], s->sur[0], s->sur[1]);
        base_into_state(s, h->xn[0], h->xn[1]);
        features_of(s, h->xn[0], h->xn[1], lin);
        copy_state(s, s->sur[0], s->sur[1], h->xn[0], h->xn[1]);
        h->t = t0;
        h->version++;
      }
    }
    return (int)SWENSE_OK;
  });
}

int swense_surrogate_target(swense_surrogate* s, const float* x_next, const float* lin, float* t) {
  if (!s || !x_next || !lin || !t) return SWENSE_EINVAL;
  return guarded_s(s, [&] {
    const long long n = 2LL * s->h->G.nx * s->h->G.ny;
    hipLaunchKernelGGL(k_target, dim3(nblk(n)), dim3(256), 0, s->h->st, x_next, lin, t, n,
                       (float)(1.0 / s->d.rho));
    SW_HIP(hipGetLastError());
    return (int)SWENSE_OK;
  });
}

int swense_surrogate_advance(swense_surrogate* s, int ncalls, swense_surrogate_stats* st) {
  if (!s || !st || ncalls < 0) return SWENSE_EINVAL;
  return guarded_s(s, [&] {
    const bool bound = s->d.drift_tol > 0.0;
    for (int c = 0; c < ncalls; ++c) {
      st->calls++;
      if (s->cool > 0) {
        hos_call(s);
        s->cool--;
        st->hos_calls++;
        continue;
      }
      if (bound && !s->spent && s->est >= 0.0) {
        // the next call goes unjudged unless on probation or the A-th: stop
        // the learned calls when its estimated error would pass the bound
        const bool judged = s->trust < s->d.probation || ((s->nsur + 1) % s->d.audit_every == 0);
        if (!judged && !(s->drift + s->est <= s->d.drift_tol)) s->spent = true;
      }
      if (s->spent) {
        hos_call(s);
        st->hos_calls++;
        st->bound_calls++;
        continue;
      }
      network_call(s, st, bound && s->est < 0.0);
    }
    st->drift_est = s->drift;
    return (int)SWENSE_OK;
  });
}

int swense_surrogate_reset(swense_surrogate* s) {
  if (!s) return SWENSE_EINVAL;
  s->cool = 0;
  s->trust = 0;
  s->nsur = 0;
  s->drift = 0.0;
  s->est = -1.0;
  s->spent = false;
  return SWENSE_OK;
}

const char* swense_surrogate_last_error(const swense_surrogate* s) { return s ? s->err.c_str() : "no handle"; }

void swense_surrogate_destroy(swense_surrogate* s) {
  if (!s) return;
  if (s->mem) (void)hipFree(s->mem);
  delete s;
}

}  // extern "C"
