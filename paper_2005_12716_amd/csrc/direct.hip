// Direct analytical evaluation of the incident fields at arbitrary points
// (Sec. 3.1.1, 3.2.1): the modal sums themselves, every mode at every point,
// in FP64 - the evaluation the paper sets aside as too costly for a CFD
// step (its cost is modes x points), kept here as an exact reference for the
// grid-and-interpolation path and for small point sets.
//
// Value of a volume field at (x, y, z), with the mean-level half spectra A
// (potential) or A_t (its time derivative):
//   sum over kept modes (q, p < nx/2 + 1) of c_p Re( A M(k) F(k, z) e^{i(kx x + ky y)} )
// with c_0 = 1, c_p = 2 otherwise, multiplier M = 1, i kx, i ky or k (phi,
// u, v, w) and vertical factor F = C = cosh k(z+h)/cosh kh (S = sinh ... for
// w), e^{kz} in deep water; surface fields eta, eta_t use their own spectra
// and no vertical factor; p = -rho (phi_t + |u|^2/2 + g z) at the point.
//
// One thread per point; the modes pass through LDS in chunks, each thread
// accumulating its point's sums in registers.  Along a row of modes (fixed
// q, p = 0, 1, ...) the phase e^{i(kx x + ky y)} advances by e^{i dkx x}, one
// complex product; sin/cos are evaluated afresh at each row start and
// chunk start (the rounding drift over a row of at most nx/2 products stays
// near 1e-13).  The vertical factor takes one exponential per mode and
// point: bound by the FP64 vector units.
#include <cmath>
#include <cstring>

#include "internal.h"

namespace {

constexpr int kNumFields = 11;     // field bits of the masks (phi ... eta_t)
constexpr int kDirectChunk = 128;  // modes per LDS chunk
constexpr int kDirectBlock = 256;  // points per workgroup

struct DirectArgs {
  const cd* a;    // A (mean-level potential)
  const cd* at;   // A_t
  const cd* e;    // eta
  const cd* et;   // eta_t
  int need_a, need_at, need_e, need_et;
  int slot[kNumFields];  // output row of each field, -1: not requested
};

// FINITE: finite depth (the vertical factors take the seabed image term).
template <bool FINITE>
__global__ void __launch_bounds__(kDirectBlock) k_direct_points(DirectArgs D, Geom G, const double* __restrict__ xyz,
                                                                 long long n, double* __restrict__ out) {
  __shared__ double s_kx[kDirectChunk], s_ky[kDirectChunk], s_k[kDirectChunk];
  __shared__ double s_e2h[kDirectChunk], s_dinv[kDirectChunk];
  __shared__ cd s_a[kDirectChunk], s_at[kDirectChunk], s_e[kDirectChunk], s_et[kDirectChunk];
  const long long i = (long long)blockIdx.x * kDirectBlock + threadIdx.x;
  const bool live = i < n;
  const double x = live ? xyz[i] : 0.0, y = live ? xyz[n + i] : 0.0, z = live ? xyz[2 * n + i] : 0.0;
  double c1, s1;  // e^{i dkx x}
  sincos(2.0 * M_PI * x / G.lx, &s1, &c1);
  double cs = 1.0, sn = 0.0;  // e^{i theta} of the current mode
  double phi = 0.0, u = 0.0, v = 0.0, w = 0.0, phit = 0.0, ut = 0.0, vt = 0.0, wt = 0.0, eta = 0.0, etat = 0.0;
  const long long nmodes = (long long)G.ny * G.nxh;
  for (long long m0 = 0; m0 < nmodes; m0 += kDirectChunk) {
    __syncthreads();
    if (threadIdx.x < kDirectChunk) {
      const long long m = m0 + threadIdx.x;
      double kx = 0.0, ky = 0.0, k = 0.0, e2h = 0.0, dinv = 1.0, c = 0.0;
      cd a = mk(0.0, 0.0), at = a, e = a, et = a;
      if (m < nmodes) {
        const int q = (int)(m / G.nxh), p = (int)(m - (long long)q * G.nxh);
        kx = 2.0 * M_PI * (double)p / G.lx;
        ky = G.ny > 1 ? 2.0 * M_PI * (double)signed_q(q, G.ny) / G.ly : 0.0;
        k = sqrt(kx * kx + ky * ky);
        if (FINITE) {
          e2h = exp(-2.0 * k * G.depth);
          dinv = 1.0 / (1.0 + e2h);
        }
        c = p == 0 ? 1.0 : 2.0;  // the p > 0 modes stand for their conjugate images too
        if (D.need_a) a = cscale(D.a[m], c);
        if (D.need_at) at = cscale(D.at[m], c);
        if (D.need_e) e = cscale(D.e[m], c);
        if (D.need_et) et = cscale(D.et[m], c);
      }
      s_kx[threadIdx.x] = kx;
      s_ky[threadIdx.x] = ky;
      s_k[threadIdx.x] = k;
      s_e2h[threadIdx.x] = e2h;
      s_dinv[threadIdx.x] = dinv;
      s_a[threadIdx.x] = a;
      s_at[threadIdx.x] = at;
      s_e[threadIdx.x] = e;
      s_et[threadIdx.x] = et;
    }
    __syncthreads();
    const int cnt = (int)min((long long)kDirectChunk, nmodes - m0);
    for (int j = 0; j < cnt; ++j) {
      const double kx = s_kx[j], ky = s_ky[j];
      if (j == 0 || kx == 0.0) {
        // chunk start or row start (p = 0): the phase afresh
        sincos(kx * x + ky * y, &sn, &cs);
      } else {
        // mode (q, p) follows (q, p - 1) in the chunk
        const double c2 = cs * c1 - sn * s1;
        sn = sn * c1 + cs * s1;
        cs = c2;
      }
      if (D.need_e) {
        const cd e = s_e[j];
        eta += e.x * cs - e.y * sn;
      }
      if (D.need_et) {
        const cd e = s_et[j];
        etat += e.x * cs - e.y * sn;
      }
      if (D.need_a || D.need_at) {
        const double k = s_k[j];
        const double ez = exp(k * z);
        double C = ez, S = ez;
        if constexpr (FINITE) {
          const double b = s_e2h[j] / ez;  // e^{-k(z + 2h)}
          C = (ez + b) * s_dinv[j];
          S = (ez - b) * s_dinv[j];
        }
        if (D.need_a) {
          const cd a = s_a[j];
          const double re = a.x * cs - a.y * sn, im = a.x * sn + a.y * cs;  // A e^{i theta}
          phi += re * C;
          u -= kx * im * C;  // Re(i kx A e^{i theta}) = -kx Im(A e^{i theta})
          v -= ky * im * C;
          w += k * re * S;
        }
        if (D.need_at) {
          const cd a = s_at[j];
          const double re = a.x * cs - a.y * sn, im = a.x * sn + a.y * cs;
          phit += re * C;
          ut -= kx * im * C;
          vt -= ky * im * C;
          wt += k * re * S;
        }
      }
    }
  }
  if (!live) return;
  const double vals[kNumFields] = {phi, u, v, w, -G.rho * (phit + 0.5 * (u * u + v * v + w * w) + G.g * z),
                                   phit, ut, vt, wt, eta, etat};
#pragma unroll
  for (int f = 0; f < kNumFields; ++f)
    if (D.slot[f] >= 0) out[(size_t)D.slot[f] * n + i] = vals[f];
}

}  // namespace

extern "C" {

int swense_eval_points_direct(swense_hos* h, long long n, const double* xyz, unsigned mask, double* out) {
  if (!h) return SWENSE_EINVAL;
  return guarded(h, [&] {
    SW_REQUIRE(n >= 0 && n < (1ll << 40), "point count must be in [0, 2^40)");
    SW_REQUIRE((mask & ~(unsigned)SWENSE_ALL_FIELDS) == 0 && mask != 0, "bad field mask");
    SW_REQUIRE(n == 0 || (xyz != nullptr && out != nullptr), "null points or output");
    if (n == 0) return (int)SWENSE_OK;
    launch_modes(h);  // A, A_t, eta_t of the current state
    DirectArgs D;
    std::memset(&D, 0, sizeof(D));
    int s = 0;
    for (int f = 0; f < kNumFields; ++f) D.slot[f] = (mask & (1u << f)) ? s++ : -1;
    const bool p = (mask & SWENSE_P) != 0;
    D.need_a = p || (mask & (SWENSE_PHI | SWENSE_U | SWENSE_V | SWENSE_W)) ? 1 : 0;
    D.need_at = p || (mask & (SWENSE_PHI_T | SWENSE_U_T | SWENSE_V_T | SWENSE_W_T)) ? 1 : 0;
    D.need_e = (mask & SWENSE_ETA) ? 1 : 0;
    D.need_et = (mask & SWENSE_ETA_T) ? 1 : 0;
    eval_sources(h, &D.a, &D.at, &D.e, &D.et);
    const long long nblk = (n + kDirectBlock - 1) / kDirectBlock;
    SW_REQUIRE(nblk <= 0x7fffffffll, "too many points for one launch");
    if (h->G.depth > 0.0)
      SW_LAUNCH(h, SWENSE_K_AUX, k_direct_points<true>, dim3((unsigned)nblk), dim3(kDirectBlock), 0, h->st, D, h->G,
                xyz, n, out);
    else
      SW_LAUNCH(h, SWENSE_K_AUX, k_direct_points<false>, dim3((unsigned)nblk), dim3(kDirectBlock), 0, h->st, D, h->G,
                xyz, n, out);
    SW_HIP(hipGetLastError());
    return (int)SWENSE_OK;
  });
}

}  // extern "C"
