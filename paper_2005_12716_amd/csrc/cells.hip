// Cell-side use of the incident fields in the CFD solver: the incident
// volume fraction from the free-surface elevation (Sec. 3.2.2), the modified
// incident pressure p_I* = rho p_I / rho_I (Sec. 2.1.3, Eq. pIStar) and the
// relaxation-zone blending (Sec. 4.2, Eq. weightFunction, swUcRelax,
// swVOFRelax).  Element-wise over the cells, FP64 arithmetic on FP32 (and
// FP64 coordinate) inputs, FP32 results; bound by HBM.
#include "internal.h"

namespace {

constexpr int kCellBlock = 256;

unsigned cell_blocks(long long n) {
  const long long b = (n + kCellBlock - 1) / kCellBlock;
  return (unsigned)(b < 65536 ? b : 65536);  // grid-stride beyond
}

// Cell height [zc - dz/2, zc + dz/2]: the share below eta (a flat
// interface across the cell), clamped to [0, 1].
__global__ void __launch_bounds__(kCellBlock) k_cell_alpha(long long n, const float* __restrict__ eta,
                                                             const double* __restrict__ zc,
                                                             const float* __restrict__ dz, float* __restrict__ alpha) {
  for (long long i = (long long)blockIdx.x * kCellBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kCellBlock) {
    const double h = (double)dz[i];
    const double zlo = zc[i] - 0.5 * h;
    double a = ((double)eta[i] - zlo) / h;
    a = a < 0.0 ? 0.0 : (a > 1.0 ? 1.0 : a);
    alpha[i] = (float)a;
  }
}

// p* = rho p / rho_water with the mixture density rho = alpha rho_water +
// (1 - alpha) rho_air.
// (ps may alias p: each cell reads its value before writing it)
__global__ void __launch_bounds__(kCellBlock) k_cell_pstar(long long n, const float* p, const float* __restrict__ alpha,
                                                             double rho_w, double rho_a, float* ps) {
  for (long long i = (long long)blockIdx.x * kCellBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kCellBlock) {
    const double a = (double)alpha[i];
    const double rho = a * rho_w + (1.0 - a) * rho_a;
    ps[i] = (float)(rho * (double)p[i] / rho_w);
  }
}

// omega(x) = -2 x^3 + 3 x^2 on x clamped to [0, 1]; alpha <- omega alpha_I +
// (1 - omega) alpha, u_C <- (1 - omega) u_C (ncomp rows of n).
__global__ void __launch_bounds__(kCellBlock) k_cell_relax(long long n, int ncomp, const float* __restrict__ x,
                                                             const float* __restrict__ alpha_i,
                                                             float* __restrict__ alpha, float* __restrict__ uc) {
  for (long long i = (long long)blockIdx.x * kCellBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kCellBlock) {
    double t = (double)x[i];
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    const double w = -2.0 * t * t * t + 3.0 * t * t;
    if (w == 0.0) continue;  // outside the zone: unchanged
    if (alpha) alpha[i] = (float)(w * (double)alpha_i[i] + (1.0 - w) * (double)alpha[i]);
    for (int c = 0; c < ncomp; ++c) uc[(size_t)c * n + i] = (float)((1.0 - w) * (double)uc[(size_t)c * n + i]);
  }
}

}  // namespace

extern "C" {

int swense_cells_alpha(swense_hos* h, long long n, const float* eta, const double* zc, const float* dz,
                       float* alpha) {
  if (!h) return SWENSE_EINVAL;
  return guarded(h, [&] {
    SW_REQUIRE(n >= 0, "negative cell count");
    SW_REQUIRE(n == 0 || (eta && zc && dz && alpha), "null argument");
    if (n == 0) return (int)SWENSE_OK;
    SW_LAUNCH(h, SWENSE_K_AUX, k_cell_alpha, dim3(cell_blocks(n)), dim3(kCellBlock), 0, h->st, n, eta, zc, dz, alpha);
    SW_HIP(hipGetLastError());
    return (int)SWENSE_OK;
  });
}

int swense_cells_pstar(swense_hos* h, long long n, const float* p, const float* alpha, double rho_air, float* pstar) {
  if (!h) return SWENSE_EINVAL;
  return guarded(h, [&] {
    SW_REQUIRE(n >= 0, "negative cell count");
    SW_REQUIRE(n == 0 || (p && alpha && pstar), "null argument");
    SW_REQUIRE(rho_air >= 0.0, "negative air density");
    if (n == 0) return (int)SWENSE_OK;
    SW_LAUNCH(h, SWENSE_K_AUX, k_cell_pstar, dim3(cell_blocks(n)), dim3(kCellBlock), 0, h->st, n, p, alpha,
              h->G.rho, rho_air, pstar);
    SW_HIP(hipGetLastError());
    return (int)SWENSE_OK;
  });
}

int swense_cells_relax(swense_hos* h, long long n, int ncomp, const float* x, const float* alpha_i, float* alpha,
                       float* uc) {
  if (!h) return SWENSE_EINVAL;
  return guarded(h, [&] {
    SW_REQUIRE(n >= 0 && ncomp >= 0 && ncomp <= 3, "negative cell count or more than 3 velocity components");
    SW_REQUIRE(n == 0 || x, "null zone coordinate");
    SW_REQUIRE(n == 0 || !alpha || alpha_i, "alpha needs alpha_i");
    SW_REQUIRE(n == 0 || ncomp == 0 || uc, "null velocity");
    if (n == 0) return (int)SWENSE_OK;
    SW_LAUNCH(h, SWENSE_K_AUX, k_cell_relax, dim3(cell_blocks(n)), dim3(kCellBlock), 0, h->st, n, ncomp, x, alpha_i,
              alpha, uc);
    SW_HIP(hipGetLastError());
    return (int)SWENSE_OK;
  });
}

}  // extern "C"
