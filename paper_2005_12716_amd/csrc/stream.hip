// Regular waves by stream-function theory (Sec. 3.1.1) and their analytical
// evaluation at points (Sec. 3.2.1).
//
// Host: the Fourier approximation of the steady wave in the frame moving with
// it (X = x - c t, Y = z + d above the bed),
//   psi = -ubar Y + sqrt(g/k^3) sum_{j=1..N} B_j sinh(j k Y)/cosh(j k d) cos(j k X),
// is fitted by Newton's method: at the N + 1 surface points X_m = m pi/(N k)
// (crest to trough) the surface is a streamline (psi = -Q) and Bernoulli holds
// (|grad psi|^2/2 + g eta = R); the trapezoidal mean of eta is zero and
// eta_0 - eta_N = H; no mean Eulerian current (c = ubar).  The height is
// raised in four steps from the linear wave.  Newton's method runs on the
// nondimensional system (lengths times k, velocities over sqrt(g/k), so
// g = k = 1), whose residuals are O(1) for any wavelength, depth and g; the
// stream-function rows are O(kd) there and their tolerance scales with it.
//
// Device: one thread per point sums the N modes (FP64): u, w, phi in the fixed
// frame, eta from its cosine series through the surface points, time
// derivatives by d/dt = -c d/dX, and p = rho (R - c^2/2) - rho (phi_t +
// |u|^2/2 + g z) (zero on the free surface).
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace {

constexpr int kMaxStreamN = 64;

struct StreamCoef {
  int n;
  double k, d, g, rho, c, R, s;  // s = sqrt(g / k^3)
  double B[kMaxStreamN];          // B_1 .. B_N
  double E[kMaxStreamN + 1];      // eta(X) = sum_{j=0..N} E_j cos(j k X)
  int slot[11];                   // output row of each field bit, -1: not requested
};

// cosh(a Y)/cosh(a d) and sinh(a Y)/cosh(a d) for a = j k, without overflow
__host__ __device__ inline void ratios(double a, double Y, double d, double& ch, double& sh) {
  const double p = exp(a * (Y - d)), m = exp(-a * (Y + d)), den = 1.0 + exp(-2.0 * a * d);
  ch = (p + m) / den;
  sh = (p - m) / den;
}

// residual of the collocation system at v = [eta_0..N, B_1..N, ubar, Q, R]
void stream_residual(const std::vector<double>& v, int N, double k, double d, double H, double g,
                     std::vector<double>& r) {
  const double s = std::sqrt(g / (k * k * k));
  r.assign(2 * N + 4, 0.0);
  const double ubar = v[2 * N + 1], Q = v[2 * N + 2], R = v[2 * N + 3];
  double mean = 0.0;
  for (int m = 0; m <= N; ++m) {
    const double eta = v[m], X = m * M_PI / (N * k), Y = eta + d;
    double psi = -ubar * Y, U = -ubar, W = 0.0;
    for (int j = 1; j <= N; ++j) {
      double ch, sh;
      ratios(j * k, Y, d, ch, sh);
      const double B = v[N + j], cx = std::cos(j * k * X), sx = std::sin(j * k * X);
      psi += s * B * sh * cx;
      U += s * B * j * k * ch * cx;
      W += s * B * j * k * sh * sx;
    }
    r[m] = psi + Q;
    r[N + 1 + m] = 0.5 * (U * U + W * W) + g * eta - R;
    mean += (m == 0 || m == N) ? 0.5 * eta : eta;
  }
  r[2 * N + 2] = mean / N;
  r[2 * N + 3] = v[0] - v[N] - H;
}

// dense solve A x = b (n x n, row-major), partial pivoting; false if singular
bool dense_solve(std::vector<double>& A, std::vector<double>& b, int n) {
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int i = c + 1; i < n; ++i)
      if (std::fabs(A[(size_t)i * n + c]) > std::fabs(A[(size_t)p * n + c])) p = i;
    if (A[(size_t)p * n + c] == 0.0) return false;
    if (p != c) {
      for (int j = 0; j < n; ++j) std::swap(A[(size_t)c * n + j], A[(size_t)p * n + j]);
      std::swap(b[c], b[p]);
    }
    for (int i = c + 1; i < n; ++i) {
      const double f = A[(size_t)i * n + c] / A[(size_t)c * n + c];
      if (f == 0.0) continue;
      for (int j = c; j < n; ++j) A[(size_t)i * n + j] -= f * A[(size_t)c * n + j];
      b[i] -= f * b[c];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    double x = b[i];
    for (int j = i + 1; j < n; ++j) x -= A[(size_t)i * n + j] * b[j];
    b[i] = x / A[(size_t)i * n + i];
  }
  return true;
}

__global__ void __launch_bounds__(256) k_stream_points(StreamCoef S, double t, const double* __restrict__ xyz,
                                                        long long n, double* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = xyz[i], z = xyz[2 * n + i];
  const double X = x - S.c * t, Y = z + S.d;
  double phi = 0.0, u = 0.0, w = 0.0, ut = 0.0, wt = 0.0;
  for (int j = 1; j <= S.n; ++j) {
    const double a = j * S.k;
    double ch, sh, sn, cs;
    ratios(a, Y, S.d, ch, sh);
    sincos(a * X, &sn, &cs);
    const double B = S.s * S.B[j - 1];
    phi += B * ch * sn;
    u += B * a * ch * cs;
    w += B * a * sh * sn;
    ut += S.c * B * a * a * ch * sn;
    wt -= S.c * B * a * a * sh * cs;
  }
  double eta = 0.0, etat = 0.0;
  for (int j = 0; j <= S.n; ++j) {
    double sn, cs;
    sincos(j * S.k * X, &sn, &cs);
    eta += S.E[j] * cs;
    etat += S.c * S.E[j] * j * S.k * sn;
  }
  const double phit = -S.c * u;
  const double p = S.rho * (S.R - 0.5 * S.c * S.c) - S.rho * (phit + 0.5 * (u * u + w * w) + S.g * z);
  const double vals[11] = {phi, u, 0.0, w, p, phit, ut, 0.0, wt, eta, etat};
#pragma unroll
  for (int f = 0; f < 11; ++f)
    if (S.slot[f] >= 0) out[(size_t)S.slot[f] * n + i] = vals[f];
}

}  // namespace

extern "C" {

int swense_stream_solve(const swense_stream_desc* d, double* sol) {
  if (!d || !sol) return SWENSE_EINVAL;
  const int N = d->n;
  if (N < 2 || N > kMaxStreamN || !(d->depth > 0.0) || !(d->height > 0.0) || !(d->wavelength > 0.0) ||
      !(d->g > 0.0))
    return SWENSE_EINVAL;
  const double k = 2.0 * M_PI / d->wavelength;
  const double vs = std::sqrt(d->g / k);  // velocity scale
  const double dep = k * d->depth;        // nondimensional depth kd
  const double th = std::tanh(dep), c0 = std::sqrt(th);
  const int nv = 2 * N + 4;
  // residual tolerance per row: the stream-function rows carry terms of size
  // ubar (Y + d) ~ kd, the others O(1)
  std::vector<double> tol(nv, 1.0);
  for (int m = 0; m <= N; ++m) tol[m] = std::fmax(1.0, dep);
  auto converged = [&](const std::vector<double>& r, double eps) {
    for (int i = 0; i < nv; ++i)
      if (!(std::fabs(r[i]) < eps * tol[i])) return false;
    return true;
  };
  std::vector<double> v(nv, 0.0), r, rp, rm, A((size_t)nv * nv);
  const int steps = 4;
  for (int st = 1; st <= steps; ++st) {
    const double H = k * d->height * st / steps;
    if (st == 1) {
      for (int m = 0; m <= N; ++m) v[m] = 0.5 * H * std::cos(m * M_PI / N);
      v[N + 1] = 0.5 * H / std::sqrt(th);
      v[2 * N + 1] = c0;
      v[2 * N + 2] = c0 * dep;
      v[2 * N + 3] = 0.5 * c0 * c0;
    } else {
      for (int i = 0; i < 2 * N + 1; ++i) v[i] *= (double)st / (st - 1);
    }
    for (int it = 0; it < 60; ++it) {
      stream_residual(v, N, 1.0, dep, H, 1.0, r);
      if (converged(r, 1e-14)) break;
      for (int c = 0; c < nv; ++c) {
        const double h = 1e-7 * std::fmax(1.0, std::fabs(v[c])), keep = v[c];
        v[c] = keep + h;
        stream_residual(v, N, 1.0, dep, H, 1.0, rp);
        v[c] = keep - h;
        stream_residual(v, N, 1.0, dep, H, 1.0, rm);
        v[c] = keep;
        for (int i = 0; i < nv; ++i) A[(size_t)i * nv + c] = (rp[i] - rm[i]) / (2.0 * h);
      }
      std::vector<double> b = r;
      if (!dense_solve(A, b, nv)) return SWENSE_EUNSTABLE;
      for (int i = 0; i < nv; ++i) v[i] -= b[i];
    }
    stream_residual(v, N, 1.0, dep, H, 1.0, r);
    if (!converged(r, 1e-12)) return SWENSE_EUNSTABLE;
  }
  // back to the caller's units: eta / k, B as is, ubar and c in vs, Q in
  // vs / k, R in vs^2
  for (int m = 0; m <= N; ++m) sol[m] = v[m] / k;
  for (int j = 1; j <= N; ++j) sol[N + j] = v[N + j];
  sol[2 * N + 1] = v[2 * N + 1] * vs;
  sol[2 * N + 2] = v[2 * N + 2] * vs / k;
  sol[2 * N + 3] = v[2 * N + 3] * vs * vs;
  return SWENSE_OK;
}

int swense_stream_eval(const swense_stream_desc* d, const double* sol, double t, long long n, const double* xyz,
                       unsigned mask, double* out, void* stream) {
  if (!d || !sol) return SWENSE_EINVAL;
  const int N = d->n;
  if (N < 2 || N > kMaxStreamN || !(d->depth > 0.0) || !(d->wavelength > 0.0)) return SWENSE_EINVAL;
  if (n < 0 || (mask & ~(unsigned)SWENSE_ALL_FIELDS) != 0 || mask == 0) return SWENSE_EINVAL;
  if (n == 0) return SWENSE_OK;
  if (!xyz || !out) return SWENSE_EINVAL;
  StreamCoef S;
  std::memset(&S, 0, sizeof(S));
  S.n = N;
  S.k = 2.0 * M_PI / d->wavelength;
  S.d = d->depth;
  S.g = d->g;
  S.rho = d->rho;
  S.c = sol[2 * N + 1];
  S.R = sol[2 * N + 3];
  S.s = std::sqrt(S.g / (S.k * S.k * S.k));
  for (int j = 1; j <= N; ++j) S.B[j - 1] = sol[N + j];
  // cosine series through the surface points (trapezoidal weights)
  for (int j = 0; j <= N; ++j) {
    double e = 0.0;
    for (int m = 0; m <= N; ++m) e += ((m == 0 || m == N) ? 0.5 : 1.0) * sol[m] * std::cos(j * m * M_PI / N);
    e *= 2.0 / N;
    if (j == 0 || j == N) e *= 0.5;
    S.E[j] = e;
  }
  int s = 0;
  for (int f = 0; f < 11; ++f) S.slot[f] = (mask & (1u << f)) ? s++ : -1;
  const long long nb = (n + 255) / 256;
  if (nb > 0x7fffffffll) return SWENSE_EINVAL;
  hipLaunchKernelGGL(k_stream_points, dim3((unsigned)nb), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), S, t,
                     xyz, n, out);
  return hipGetLastError() == hipSuccess ? SWENSE_OK : SWENSE_EHIP;
}

}  // extern "C"
