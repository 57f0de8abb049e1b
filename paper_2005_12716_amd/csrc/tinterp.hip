// Evaluation between two outputs of the wave model.  The CFD step is several
// times shorter than the HOS step (Sec. 4.3 and the validation cases); the
// paper does not say how the incident fields are taken in between.  Here:
// cubic Hermite interpolation in time of the mean-level spectra from their
// values and time derivatives at the ends of the interval - (A, A_t) and
// (eta_hat, eta_t_hat) - with the derivative of that cubic as the time
// derivative at t.  A snapshot records the start of the interval; the
// current state is its end.
#include "internal.h"

namespace {

// y(s) = h00 y0 + h10 D y0' + h01 y1 + h11 D y1',  y'(s) = d/dt of that,
// s = (t - t0) / D, for the pairs (A, A_t) and (eta, eta_t).
__global__ void __launch_bounds__(256) k_hermite(const cd* __restrict__ snap, const cd* __restrict__ a1,
                                                  const cd* __restrict__ at1, const cd* __restrict__ e1,
                                                  const cd* __restrict__ et1, cd* __restrict__ out, size_t nc,
                                                  double s, double D) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  const double s2 = s * s, s3 = s2 * s;
  const double h00 = 2.0 * s3 - 3.0 * s2 + 1.0, h10 = s3 - 2.0 * s2 + s, h01 = -2.0 * s3 + 3.0 * s2, h11 = s3 - s2;
  const double d00 = 6.0 * s2 - 6.0 * s, d10 = 3.0 * s2 - 4.0 * s + 1.0, d01 = -6.0 * s2 + 6.0 * s,
               d11 = 3.0 * s2 - 2.0 * s;
  const cd* y1s[2] = {a1, e1};
  const cd* dy1s[2] = {at1, et1};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const cd y0 = snap[(2 * k) * nc + i], dy0 = snap[(2 * k + 1) * nc + i];
    const cd y1 = y1s[k][i], dy1 = dy1s[k][i];
    cd y, dy;
    y.x = h00 * y0.x + h10 * D * dy0.x + h01 * y1.x + h11 * D * dy1.x;
    y.y = h00 * y0.y + h10 * D * dy0.y + h01 * y1.y + h11 * D * dy1.y;
    dy.x = (d00 * y0.x + d10 * D * dy0.x + d01 * y1.x + d11 * D * dy1.x) / D;
    dy.y = (d00 * y0.y + d10 * D * dy0.y + d01 * y1.y + d11 * D * dy1.y) / D;
    out[(2 * k) * nc + i] = y;
    out[(2 * k + 1) * nc + i] = dy;
  }
}

bool same_time(double a, double b) { return std::fabs(a - b) <= 1e-12 * std::fmax(1.0, std::fabs(b)); }

}  // namespace

extern "C" {

int swense_hos_snapshot(swense_hos* h) {
  if (!h) return SWENSE_EINVAL;
  return guarded(h, [&] {
    launch_modes(h);
    if (!h->snapm) SW_HIP(hipMalloc(&h->snapm, 4 * h->nc * sizeof(cd)));
    const cd* src[4] = {h->amod, h->atmod, h->xn[0], h->kk[0]};
    for (int k = 0; k < 4; ++k)
      SW_HIP(hipMemcpyAsync(h->snapm + k * h->nc, src[k], h->nc * sizeof(cd), hipMemcpyDeviceToDevice, h->st));
    h->snap_t = h->t;
    h->snap_ok = true;
    return (int)SWENSE_OK;
  });
}

int swense_hos_set_eval_time(swense_hos* h, double t) {
  if (!h) return SWENSE_EINVAL;
  return guarded(h, [&] {
    h->herm_on = false;
    if (same_time(t, h->t)) return (int)SWENSE_OK;
    SW_REQUIRE(h->snap_ok && h->snap_t < h->t && !same_time(h->snap_t, h->t),
               "no snapshot earlier than the current state");
    SW_REQUIRE(t >= h->snap_t - 1e-12 * std::fmax(1.0, std::fabs(h->snap_t)) && t <= h->t,
               "evaluation time outside [snapshot time, current time]");
    launch_modes(h);
    if (!h->herm) SW_HIP(hipMalloc(&h->herm, 4 * h->nc * sizeof(cd)));
    const double D = h->t - h->snap_t;
    const double s = std::fmin(1.0, std::fmax(0.0, (t - h->snap_t) / D));
    hipLaunchKernelGGL(k_hermite, dim3((unsigned)((h->nc + 255) / 256)), dim3(256), 0, h->st, h->snapm, h->amod,
                       h->atmod, h->xn[0], h->kk[0], h->herm, h->nc, s, D);
    SW_HIP(hipGetLastError());
    h->herm_on = true;
    h->herm_version = h->version;
    return (int)SWENSE_OK;
  });
}

}  // extern "C"
