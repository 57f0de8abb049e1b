// Initial sea states as FP64 half spectra (set-up; host code).
//
// JONSWAP (the irregular seas of Sec. 3.1.2 and the reconstruction example of
// Sec. 3.2.2, which give only Tp/Hs/gamma): frequency spectrum
//   S(w) = g^2 w^-5 exp(-5/4 (wp/w)^4) gamma^exp(-(w-wp)^2 / (2 s^2 wp^2)),
//   s = 0.07 for w <= wp, 0.09 above,
// carried to wavenumber with deep-water dispersion w^2 = g k (S_k = S_w g/(2w)),
// spread over direction with D(theta) = (2/pi) cos^2 theta (|theta| < pi/2) or
// put entirely on ky = 0, and discretised as mode amplitudes
// a = sqrt(2 S(kx,ky) dkx dky), rescaled so that 4 sqrt(sum a^2/2) = Hs.  The
// mode with kx > 0 carries a cos(k.x + phase) and the linear potential of a
// wave travelling along +k: phis_hat = -i (g/w) eta_hat.
//
// Stokes (regular waves, Sec. 3.1.1): second-order Stokes wave on one mode.
#include <cmath>
#include <cstring>
#include <vector>

#include "swense.h"

namespace {

struct C2 {
  double re, im;
};

double jonswap_w(double w, double wp, double gamma, double g) {
  if (!(w > 0.0)) return 0.0;
  const double sig = w <= wp ? 0.07 : 0.09;
  const double r = (w - wp) / (sig * wp);
  return g * g * std::pow(w, -5.0) * std::exp(-1.25 * std::pow(wp / w, 4.0)) * std::pow(gamma, std::exp(-0.5 * r * r));
}

}  // namespace

extern "C" int swense_sea_spectrum(const swense_hos_desc* d, const swense_sea_desc* sea, const double* phases,
                                   double* eta_hat, double* phis_hat) {
  if (!d || !sea || !eta_hat || !phis_hat) return SWENSE_EINVAL;
  const int nx = d->nx, ny = d->dim == 2 ? 1 : d->ny, nxh = nx / 2 + 1;
  if (nx < 4 || nx % 2 || ny < 1 || !(d->lx > 0) || !(d->g > 0)) return SWENSE_EINVAL;
  const size_t nc = (size_t)ny * nxh;
  C2* E = reinterpret_cast<C2*>(eta_hat);
  C2* P = reinterpret_cast<C2*>(phis_hat);
  std::memset(E, 0, nc * sizeof(C2));
  std::memset(P, 0, nc * sizeof(C2));
  const double g = d->g;
  const double lx = d->lx, ly = d->dim == 2 ? 1.0 : d->ly;
  if (sea->kind == 1) {
    const int mode = sea->mode;
    if (mode < 1 || 2 * mode >= nx / 2) return SWENSE_EINVAL;
    const double k = 2.0 * M_PI * mode / lx;
    const double a = sea->ka / k;
    double w, a2, b2;
    if (d->depth > 0) {
      const double h = d->depth, th = std::tanh(k * h), sh = std::sinh(k * h);
      w = std::sqrt(g * k * th);
      a2 = 0.25 * k * a * a * std::cosh(k * h) * (2.0 + std::cosh(2.0 * k * h)) / (sh * sh * sh);
      b2 = 0.375 * w * a * a * std::cosh(2.0 * k * h) / (sh * sh * sh * sh);
    } else {
      w = std::sqrt(g * k);
      a2 = 0.5 * k * a * a;
      b2 = 0.0;
    }
    // eta = a cos t + a2 cos 2t; phis(x) = (g a/w) sin t + (b2 + w a^2/2) sin 2t
    // (the last term is eta1 * dphi1/dz at z = 0).  cos -> 1/2, sin -> -i/2.
    E[mode].re = 0.5 * a;
    E[2 * mode].re = 0.5 * a2;
    P[mode].im = -0.5 * g * a / w;
    P[2 * mode].im = -0.5 * (b2 + 0.5 * w * a * a);
    return SWENSE_OK;
  }
  if (sea->kind != 0 || !phases || !(sea->hs > 0) || !(sea->kp > 0) || !(sea->gamma >= 1.0)) return SWENSE_EINVAL;
  const double dkx = 2.0 * M_PI / lx, dky = ny > 1 ? 2.0 * M_PI / ly : 1.0;
  const double wp = std::sqrt(g * sea->kp);
  std::vector<double> amp(nc, 0.0);
  double m0 = 0.0;
  for (int q = 0; q < ny; ++q) {
    const int qs = (ny > 1 && q >= ny / 2) ? q - ny : q;
    if (ny > 1 && 2 * q == ny) continue;
    for (int p = 1; p < nx / 2; ++p) {
      const double kx = p * dkx, ky = ny > 1 ? qs * dky : 0.0;
      const double k = std::sqrt(kx * kx + ky * ky);
      const double w = std::sqrt(g * k);
      const double sk = jonswap_w(w, wp, sea->gamma, g) * g / (2.0 * w);
      double dens;
      if (ny == 1 || sea->spreading == 1) {
        dens = (qs == 0) ? sk / dky : 0.0;
      } else {
        const double th = std::atan2(ky, kx);
        const double D = std::fabs(th) < 0.5 * M_PI ? (2.0 / M_PI) * std::cos(th) * std::cos(th) : 0.0;
        dens = sk * D / k;
      }
      const double a = std::sqrt(2.0 * dens * dkx * dky);
      amp[(size_t)q * nxh + p] = a;
      m0 += 0.5 * a * a;
    }
  }
  if (!(m0 > 0)) return SWENSE_EINVAL;
  const double scale = sea->hs / (4.0 * std::sqrt(m0));
  for (int q = 0; q < ny; ++q)
    for (int p = 1; p < nx / 2; ++p) {
      const size_t i = (size_t)q * nxh + p;
      if (amp[i] == 0.0) continue;
      const int qs = (ny > 1 && q >= ny / 2) ? q - ny : q;
      const double kx = p * dkx, ky = ny > 1 ? qs * dky : 0.0;
      const double w = std::sqrt(g * std::sqrt(kx * kx + ky * ky));
      const double half = 0.5 * amp[i] * scale;
      E[i].re = half * std::cos(phases[i]);
      E[i].im = half * std::sin(phases[i]);
      // -i (g/w) eta
      P[i].re = (g / w) * E[i].im;
      P[i].im = -(g / w) * E[i].re;
    }
  return SWENSE_OK;
}
