// Reconstruction of the incident fields on gfx950 (Sec. 3.2, 3.3).
//
// Grid evaluation: for every field and layer z_l, the FP64 mean-level modes
// (A for phi, u, v, w; A_t for the time derivatives; eta_hat, eta_t_hat for
// the surface) are multiplied by the FP64 vertical factor C or S and by
// 1 | i kx | i ky | k, rounded to the transform precision, zero-padded (or
// alias-folded) to gx x gy and inverse transformed: y first (only the window
// rows are kept), then x (only the window columns are written).  Pressure is
// formed from phi_t, u, v, w in the x pass.  With the B-spline prefilter the
// same pipeline yields the interpolation coefficient grids.
//
// Interpolation: points are located once (bind, FP64) as a horizontal node
// index + fractional position and a vertical 4-point Lagrange stencil; each
// call gathers 4 x 4 (x 4 layers) coefficients per field.
#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.h"
#include "yinv.h"

namespace {

constexpr int kNumFields = 11;
constexpr int F_PHI = 0, F_U = 1, F_V = 2, F_W = 3, F_P = 4, F_PHIT = 5, F_UT = 6, F_VT = 7, F_WT = 8, F_ETA = 9,
              F_ETAT = 10;

// one spectral source field of the evaluation
struct EvField {
  const cd* src;
  int vf;        // 0 C, 1 S, 2 none (surface)
  int mult;      // 0 1, 1 i kx, 2 i ky, 3 k
  int out_slot;  // output slot (volume or surface index in the output), -1: helper only
  int p_role;    // 0 none, 1 phi_t, 2 u, 3 v, 4 w (inputs of the pressure)
};

constexpr int kMaxEvFields = 12;
struct EvArgs {
  int nvol, nsurf;  // spectral volume fields, surface fields (after the volume ones)
  EvField f[kMaxEvFields];
  const double* z;  // device layer heights
  int nl;
  int gx, gy, ix0, iy0, wx, wy;
  int pre;
  void* inter;  // [job][wy][nxh] complex rows
  float* out;
  int nvol_out;   // volume output slots (incl. pressure)
  int p_slot;     // output slot of the pressure, -1 if not requested
  const cd* srcs[4];       // distinct spectral sources of the fields
  int sid[kMaxEvFields];   // source of each field (index into srcs)
  // field whose y transform this field reuses times i kx (the x derivative
  // of a field of the same source and vertical factor: its symbol differs
  // by i kx only, a constant along each kx column); -1: transformed itself
  int alias[kMaxEvFields];
};

// y-inverse for evaluation: job = (field, layer) for volume fields, then
// one job per surface field.
__device__ __forceinline__ YInvJob eval_job(const EvArgs& A, const Geom& G, int job, size_t csz) {
  YInvJob jb = {};
  int fi;
  if (job < A.nvol * A.nl) {
    fi = job / A.nl;
    jb.z = A.z[job - fi * A.nl];
  } else {
    fi = A.nvol + (job - A.nvol * A.nl);
    jb.z = 0.0;
  }
  jb.src = A.f[fi].src;
  jb.dst = reinterpret_cast<char*>(A.inter) + (size_t)job * A.wy * G.nxh * csz;
  jb.sym = SYM_EVAL;
  jb.ev.vf = A.f[fi].vf;
  jb.ev.mult = A.f[fi].mult;
  jb.ev.pre = A.pre;
  jb.ev.gx = A.gx;
  jb.ev.gy = A.gy;
  return jb;
}

template <typename R>
__global__ void __launch_bounds__(256) k_yinv_eval(EvArgs A, Geom G, FftPlan plan, int TW) {
  extern __shared__ unsigned char smem[];
  const YInvJob jb = eval_job(A, G, blockIdx.y, sizeof(cpx<R>));
  yinv_body<R>(jb, G, plan, TW, A.wy, A.iy0, smem);
}

// wavefront version: one wavefront per kx column, four per block
template <typename R, int MAXE, int NS0>
__global__ void __launch_bounds__(256) k_yinv_eval_w(EvArgs A, Geom G, WPlan plan) {
  extern __shared__ unsigned char smem[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int p = xcd_tile(blockIdx.x, gridDim.x) * 4 + wave;
  if (p >= G.nxh) return;
  const YInvJob jb = eval_job(A, G, blockIdx.y, sizeof(cpx<R>));
  cpx<R>* buf = reinterpret_cast<cpx<R>*>(smem) + (size_t)wave * wbuf_len(plan.n);
  yinv_wave<R, MAXE, NS0>(jb, G, plan, A.wy, A.iy0, p, buf, lane);
}

// Workgroup version for the lengths of the workgroup transforms, zero-padding
// in y (single-precision transforms): block = (kx column p, layer l; l = nl:
// the surface fields), all of the layer's fields in turn, each transformed by
// the whole workgroup.  The column's values of the (at most two) sources and,
// per mode, the vertical factors C and S at z_l times the prefilter -
// computed in FP64 and rounded once - are formed once and shared by the
// fields; each field's value is their single-precision product with its
// multiplier.  TQ >= ny / 256 modes per thread.
template <typename R, int N, int TQ>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(N >= 3072 || (N >= 1536 && TQ >= 2) || (N == 768 && TQ >= 4) || (N == 2048 && TQ >= 2) ? 2 : 4))) k_yinv_eval_g(EvArgs A, Geom G, const cpx<R>* __restrict__ tw) {
  extern __shared__ unsigned char smem[];
  using C = cpx<R>;
  constexpr int T = N / 256;  // slots per thread
  C* buf = reinterpret_cast<C*>(smem);
  const int p = xcd_tile(blockIdx.x, gridDim.x);
  const int l = A.nvol > 0 ? (int)blockIdx.y : A.nl;
  const bool surf = l == A.nl;
  const int f0 = surf ? A.nvol : 0, f1 = surf ? A.nvol + A.nsurf : A.nvol;
  const int tid = threadIdx.x, half = G.ny / 2;
  const bool col = p < G.nxh && 2 * p != G.nx;
  const int s0 = A.sid[f0];
  int s1 = s0;
  for (int f = f0; f < f1; ++f)
    if (A.sid[f] != s0) s1 = A.sid[f];
  // per mode of this thread: the source values and the FP64 products of
  // vertical factor and prefilter, each rounded once to single precision
  cpx<float> v0[TQ], v1[TQ];
  float fc[TQ], fsn[TQ];
  const double kx = 2.0 * M_PI * (double)p / G.lx;
  const double bx = A.pre ? (4.0 + 2.0 * cos(2.0 * M_PI * (double)p / (double)A.gx)) / 6.0 : 1.0;
  const double z = surf ? 0.0 : A.z[l];
  const double kys = 2.0 * M_PI / G.ly;
#pragma unroll
  for (int t = 0; t < TQ; ++t) {
    const int q = tid + 256 * t;
    const int qs = q >= half ? q - G.ny : q;
    const bool ok = col && q < G.ny && qs > -half;
    const cd a = ok ? A.srcs[s0][(size_t)q * G.nxh + p] : mk(0.0, 0.0);
    const cd b = ok ? A.srcs[s1][(size_t)q * G.nxh + p] : mk(0.0, 0.0);
    v0[t] = mk((float)a.x, (float)a.y);
    v1[t] = mk((float)b.x, (float)b.y);
  }
#pragma unroll
  for (int t = 0; t < TQ; ++t) {
    const int q = tid + 256 * t;
    const int qs = q >= half ? q - G.ny : q;
    const double ky = kys * (double)qs;
    double c = 1.0, sn = 1.0;
    if (!surf) vfactors(sqrt(kx * kx + ky * ky), z, G.depth, c, sn);
    const double by = A.pre ? (4.0 + 2.0 * cos(2.0 * M_PI * (double)qs / (double)A.gy)) / 6.0 : 1.0;
    const double pre = 1.0 / (bx * by);
    fc[t] = (float)(c * pre);
    fsn[t] = (float)(sn * pre);
  }
  const float kxf = (float)kx, kysf = (float)kys;
  for (int f = f0; f < f1; ++f) {
    if (A.alias[f] >= 0) continue;  // formed by the x pass from its alias
    const EvField F = A.f[f];
    const bool first = A.sid[f] == s0;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int s = tid + 256 * t;
      if (!col || (s >= half && s <= N - half)) buf[grp_in<N>(s)] = mk((R)0, (R)0);
    }
#pragma unroll
    for (int t = 0; t < TQ; ++t) {
      const int q = tid + 256 * t;
      const int qs = q >= half ? q - G.ny : q;
      if (col && q < G.ny && qs > -half) {
        // surface fields: no vertical factor (fc = fsn = prefilter there)
        const float fac = F.vf == 1 ? fsn[t] : fc[t];
        const float ky = kysf * (float)qs;
        cpx<float> m;
        switch (F.mult) {
          case 0: m = mk(fac, 0.f); break;
          case 1: m = mk(0.f, kxf * fac); break;
          case 2: m = mk(0.f, ky * fac); break;
          default: m = mk(sqrtf(kxf * kxf + ky * ky) * fac, 0.f); break;
        }
        const cpx<float> w = cmul(first ? v0[t] : v1[t], m);
        buf[grp_in<N>(qs >= 0 ? qs : qs + N)] = mk((R)w.x, (R)w.y);
      }
    }
    grp_fft<R, N>(buf, tw, +1);
    const int job = surf ? A.nvol * A.nl + (f - A.nvol) : f * A.nl + l;
    C* dst = reinterpret_cast<C*>(A.inter) + (size_t)job * A.wy * G.nxh;
    for (int r = tid; r < A.wy; r += 256) {
      int y = A.iy0 + r;
      if (y >= N) y -= N * (y / N);
      dst[(size_t)r * G.nxh + p] = buf[grp_out<N>(y)];
    }
    __syncthreads();
  }
}

// Residue form of the zero-padded y pass, for grid lengths N = RS ny (RS in
// {2, 3, 4}, ny a power of two): with y = RS s + r the inverse transform
// splits into RS independent ny-point transforms,
//   X[RS s + r] = sum_q (x_q e^{2 pi i q r / N}) e^{2 pi i q s / ny},
// one per residue r, so wavefront r transforms the modulated modes in its own
// buffer (no zero entries, no combine, no block barrier inside the
// transform) and stores the window rows y = r (mod RS).  Same per-mode
// values, factors and fields as k_yinv_eval_g.  The passes read their
// twiddles after the LDS loads here: the registers go to occupancy (three
// waves per SIMD at 1024 modes; measured 2.3 against 2.6 ms with them read
// ahead at two).
template <int RS, int NY, int TQ>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NY >= 1024 ? 3 : 4))) k_yinv_eval_r(
    EvArgs A, Geom G, const cpx<float>* __restrict__ tw) {
  static_assert(RS >= 2 && RS <= 4 && TQ * 256 >= NY, "residues and modes per thread");
  constexpr int N = RS * NY;
  constexpr int WL = NY + NY / 16 + 1;
  using C = cpx<float>;
  extern __shared__ unsigned char smem[];
  C* buf = reinterpret_cast<C*>(smem);
  // one-dimensional grid over (column, layer slot), grouped by columns
  int p, ly;
  grouped_tile<16>(blockIdx.x, G.nxh, A.nvol > 0 ? A.nl + (A.nsurf > 0 ? 1 : 0) : 1, p, ly);
  const int l = A.nvol > 0 ? ly : A.nl;
  const bool surf = l == A.nl;
  const int f0 = surf ? A.nvol : 0, f1 = surf ? A.nvol + A.nsurf : A.nvol;
  const int tid = threadIdx.x, half = G.ny / 2;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const bool col = p < G.nxh && 2 * p != G.nx;
  const int s0 = A.sid[f0];
  int s1 = s0;
  for (int f = f0; f < f1; ++f)
    if (A.sid[f] != s0) s1 = A.sid[f];
  cpx<float> v0[TQ], v1[TQ], md[TQ];  // md: e^{2 pi i qs / N}; residue r takes its r-th power
  float fc[TQ], fsn[TQ];
  const double kx = 2.0 * M_PI * (double)p / G.lx;
  const double bx = A.pre ? (4.0 + 2.0 * cos(2.0 * M_PI * (double)p / (double)A.gx)) / 6.0 : 1.0;
  const double z = surf ? 0.0 : A.z[l];
  const double kys = 2.0 * M_PI / G.ly;
#pragma unroll
  for (int t = 0; t < TQ; ++t) {
    const int q = tid + 256 * t;
    const int qs = q >= half ? q - G.ny : q;
    const bool ok = col && q < G.ny && qs > -half;
    const cd a = ok ? A.srcs[s0][(size_t)q * G.nxh + p] : mk(0.0, 0.0);
    const cd b = ok ? A.srcs[s1][(size_t)q * G.nxh + p] : mk(0.0, 0.0);
    v0[t] = mk((float)a.x, (float)a.y);
    v1[t] = mk((float)b.x, (float)b.y);
    // modulation e^{+2 pi i qs / N} (the table holds e^{-2 pi i m / N})
    const C w = tw[(qs + N) % N];
    md[t] = mk(w.x, -w.y);
  }
#pragma unroll
  for (int t = 0; t < TQ; ++t) {
    const int q = tid + 256 * t;
    const int qs = q >= half ? q - G.ny : q;
    const double ky = kys * (double)qs;
    double c = 1.0, sn = 1.0;
    if (!surf) vfactors(sqrt(kx * kx + ky * ky), z, G.depth, c, sn);
    const double by = A.pre ? (4.0 + 2.0 * cos(2.0 * M_PI * (double)qs / (double)A.gy)) / 6.0 : 1.0;
    const double pre = 1.0 / (bx * by);
    fc[t] = (float)(c * pre);
    fsn[t] = (float)(sn * pre);
  }
  const float kxf = (float)kx, kysf = (float)kys;
  for (int f = f0; f < f1; ++f) {
    if (A.alias[f] >= 0) continue;  // formed by the x pass from its alias
    const EvField F = A.f[f];
    const bool first = A.sid[f] == s0;
#pragma unroll
    for (int t = 0; t < TQ; ++t) {
      const int q = tid + 256 * t;
      if (q >= NY) continue;
      const int qs = q >= half ? q - G.ny : q;
      cpx<float> w = mk(0.f, 0.f);
      if (col && q < G.ny && qs > -half) {
        const float fac = F.vf == 1 ? fsn[t] : fc[t];
        const float ky = kysf * (float)qs;
        cpx<float> m;
        switch (F.mult) {
          case 0: m = mk(fac, 0.f); break;
          case 1: m = mk(0.f, kxf * fac); break;
          case 2: m = mk(0.f, ky * fac); break;
          default: m = mk(sqrtf(kxf * kxf + ky * ky) * fac, 0.f); break;
        }
        w = cmul(first ? v0[t] : v1[t], m);
      }
      const int slot = q;  // qs mod ny (q itself: the mode grid's own index)
#pragma unroll
      for (int r = 0; r < RS; ++r) {
        buf[r * WL + sk(slot)] = w;
        w = cmul(w, md[t]);
      }
    }
    __syncthreads();
    const int job = surf ? A.nvol * A.nl + (f - A.nvol) : f * A.nl + l;
    C* dst = reinterpret_cast<C*>(A.inter) + (size_t)job * A.wy * G.nxh;
    if (wave < RS) {
      C* b = buf + wave * WL;
      wave_fft_static<float, NY, RS, false>(b, tw, +1, lane);
      // window rows y = iy0 + rr (mod N) with y = wave (mod RS)
      const int r0 = ((wave - A.iy0) % RS + RS) % RS;
      for (int rr = r0 + RS * lane; rr < A.wy; rr += RS * 64) {
        int y = A.iy0 + rr;
        if (y >= N) y -= N * (y / N);
        dst[(size_t)rr * G.nxh + p] = b[sk((y - wave) / RS)];
      }
    }
    __syncthreads();
  }
}

// The same residue form for mode counts whose transform has a runtime plan
// (ny up to 64 MAXE points, any 2/3/5-smooth length): wavefront r runs the
// ny-point transform of its modulated modes with the plan `pny`, whose
// twiddles are every RS-th entry of the N = RS ny table `tw` that also gives
// the modulations.
template <int RS, int TQ, int MAXE>
__global__ void __launch_bounds__(256) k_yinv_eval_rr(EvArgs A, Geom G, const cpx<float>* __restrict__ tw, WPlan pny) {
  static_assert(RS >= 2 && RS <= 4, "residues");
  using C = cpx<float>;
  extern __shared__ unsigned char smem[];
  C* buf = reinterpret_cast<C*>(smem);
  const int ny = G.ny, N = RS * ny, WL = wbuf_len(ny);
  int p, ly;
  grouped_tile<16>(blockIdx.x, G.nxh, A.nvol > 0 ? A.nl + (A.nsurf > 0 ? 1 : 0) : 1, p, ly);
  const int l = A.nvol > 0 ? ly : A.nl;
  const bool surf = l == A.nl;
  const int f0 = surf ? A.nvol : 0, f1 = surf ? A.nvol + A.nsurf : A.nvol;
  const int tid = threadIdx.x, half = ny / 2;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const bool col = p < G.nxh && 2 * p != G.nx;
  const int s0 = A.sid[f0];
  int s1 = s0;
  for (int f = f0; f < f1; ++f)
    if (A.sid[f] != s0) s1 = A.sid[f];
  C v0[TQ], v1[TQ], md[TQ];
  float fc[TQ], fsn[TQ];
  const double kx = 2.0 * M_PI * (double)p / G.lx;
  const double bx = A.pre ? (4.0 + 2.0 * cos(2.0 * M_PI * (double)p / (double)A.gx)) / 6.0 : 1.0;
  const double z = surf ? 0.0 : A.z[l];
  const double kys = 2.0 * M_PI / G.ly;
#pragma unroll
  for (int t = 0; t < TQ; ++t) {
    const int q = tid + 256 * t;
    const int qs = q >= half ? q - ny : q;
    const bool ok = col && q < ny && qs > -half;
    const cd a = ok ? A.srcs[s0][(size_t)q * G.nxh + p] : mk(0.0, 0.0);
    const cd b = ok ? A.srcs[s1][(size_t)q * G.nxh + p] : mk(0.0, 0.0);
    v0[t] = mk((float)a.x, (float)a.y);
    v1[t] = mk((float)b.x, (float)b.y);
    const C w = q < ny ? tw[(qs + N) % N] : mk(1.f, 0.f);
    md[t] = mk(w.x, -w.y);
  }
#pragma unroll
  for (int t = 0; t < TQ; ++t) {
    const int q = tid + 256 * t;
    const int qs = q >= half ? q - ny : q;
    const double ky = kys * (double)qs;
    double c = 1.0, sn = 1.0;
    if (!surf) vfactors(sqrt(kx * kx + ky * ky), z, G.depth, c, sn);
    const double by = A.pre ? (4.0 + 2.0 * cos(2.0 * M_PI * (double)qs / (double)A.gy)) / 6.0 : 1.0;
    const double pre = 1.0 / (bx * by);
    fc[t] = (float)(c * pre);
    fsn[t] = (float)(sn * pre);
  }
  const float kxf = (float)kx, kysf = (float)kys;
  for (int f = f0; f < f1; ++f) {
    if (A.alias[f] >= 0) continue;  // formed by the x pass from its alias
    const EvField F = A.f[f];
    const bool first = A.sid[f] == s0;
#pragma unroll
    for (int t = 0; t < TQ; ++t) {
      const int q = tid + 256 * t;
      if (q >= ny) continue;
      const int qs = q >= half ? q - ny : q;
      C w = mk(0.f, 0.f);
      if (col && qs > -half) {
        const float fac = F.vf == 1 ? fsn[t] : fc[t];
        const float ky = kysf * (float)qs;
        C m;
        switch (F.mult) {
          case 0: m = mk(fac, 0.f); break;
          case 1: m = mk(0.f, kxf * fac); break;
          case 2: m = mk(0.f, ky * fac); break;
          default: m = mk(sqrtf(kxf * kxf + ky * ky) * fac, 0.f); break;
        }
        w = cmul(first ? v0[t] : v1[t], m);
      }
#pragma unroll
      for (int r = 0; r < RS; ++r) {
        buf[r * WL + sk(q)] = w;
        w = cmul(w, md[t]);
      }
    }
    __syncthreads();
    const int job = surf ? A.nvol * A.nl + (f - A.nvol) : f * A.nl + l;
    C* dst = reinterpret_cast<C*>(A.inter) + (size_t)job * A.wy * G.nxh;
    if (wave < RS) {
      C* b = buf + wave * WL;
      wave_fft<float, MAXE>(b, pny, +1, lane, RS);
      const int r0 = ((wave - A.iy0) % RS + RS) % RS;
      for (int rr = r0 + RS * lane; rr < A.wy; rr += RS * 64) {
        int y = A.iy0 + rr;
        if (y >= N) y -= N * (y / N);
        dst[(size_t)rr * G.nxh + p] = b[sk((y - wave) / RS)];
      }
    }
    __syncthreads();
  }
}

// Complex length-gx sequence whose inverse transform is a + i b at the nodes,
// from two rows of half spectra (x modes p < nx/2), padding or folding.
template <typename R>
__device__ __forceinline__ cpx<R> gather_x(const cpx<R>* ra, const cpx<R>* rb, int s, int gx, int hx) {
  R zx = 0, zy = 0;
  for (int p = s; p < hx; p += gx) {
    cpx<R> va = ra[p], vb = rb ? rb[p] : mk((R)0, (R)0);
    zx += va.x - vb.y;
    zy += va.y + vb.x;
  }
  int p0 = (gx - s) % gx;
  if (p0 == 0) p0 = gx;
  for (int p = p0; p < hx; p += gx) {
    cpx<R> va = conjg(ra[p]), vb = rb ? conjg(rb[p]) : mk((R)0, (R)0);
    zx += va.x - vb.y;
    zy += va.y + vb.x;
  }
  return mk(zx, zy);
}

// x pass for volume fields: block (window row r, layer l).
template <typename R>
__global__ void __launch_bounds__(256) k_xeval_vol(EvArgs A, Geom G, FftPlan plan) {
  extern __shared__ unsigned char smem[];
  using C = cpx<R>;
  const int gx = plan.n, r = blockIdx.x, l = blockIdx.y, hx = G.nx / 2;
  C* za = reinterpret_cast<C*>(smem);
  C* zb = za + gx;
  R* pin = reinterpret_cast<R*>(zb + gx);  // [4][wx] pressure inputs
  const C* inter = reinterpret_cast<const C*>(A.inter);
  if (A.p_slot >= 0)
    for (int e = threadIdx.x; e < 4 * A.wx; e += blockDim.x) pin[e] = (R)0;
  for (int i = 0; i < A.nvol; i += 2) {
    const bool hasb = i + 1 < A.nvol;
    const C* ra = inter + ((size_t)(i * A.nl + l) * A.wy + r) * G.nxh;
    const C* rb = hasb ? inter + ((size_t)((i + 1) * A.nl + l) * A.wy + r) * G.nxh : nullptr;
    for (int s = threadIdx.x; s < gx; s += blockDim.x) za[s] = gather_x<R>(ra, rb, s, gx, hx);
    __syncthreads();
    C* res = block_fft<R>(za, zb, plan, 1, +1);
    for (int xw = threadIdx.x; xw < A.wx; xw += blockDim.x) {
      const int x = (A.ix0 + xw) % gx;
      const R v[2] = {res[x].x, res[x].y};
      for (int k = 0; k < 2; ++k) {
        if (k == 1 && !hasb) break;
        const EvField& f = A.f[i + k];
        if (f.out_slot >= 0) A.out[((size_t)(f.out_slot * A.nl + l) * A.wy + r) * A.wx + xw] = (float)v[k];
        if (f.p_role > 0) pin[(f.p_role - 1) * A.wx + xw] = v[k];
      }
    }
    __syncthreads();
  }
  if (A.p_slot >= 0) {
    const double zl = A.z[l];
    for (int xw = threadIdx.x; xw < A.wx; xw += blockDim.x) {
      const R pt = pin[xw], u = pin[A.wx + xw], v = pin[2 * A.wx + xw], w = pin[3 * A.wx + xw];
      const double pr = -G.rho * ((double)pt + 0.5 * (double)(u * u + v * v + w * w) + G.g * zl);
      A.out[((size_t)(A.p_slot * A.nl + l) * A.wy + r) * A.wx + xw] = (float)pr;
    }
  }
}

// x pass for surface fields: block = window row r; surface outputs follow
// the volume outputs as [nsurf][wy][wx].
template <typename R>
__global__ void __launch_bounds__(256) k_xeval_surf(EvArgs A, Geom G, FftPlan plan) {
  extern __shared__ unsigned char smem[];
  using C = cpx<R>;
  const int gx = plan.n, r = blockIdx.x, hx = G.nx / 2;
  C* za = reinterpret_cast<C*>(smem);
  C* zb = za + gx;
  const C* inter = reinterpret_cast<const C*>(A.inter) + (size_t)A.nvol * A.nl * A.wy * G.nxh;
  float* outs = A.out + (size_t)A.nvol_out * A.nl * A.wy * A.wx;
  for (int i = 0; i < A.nsurf; i += 2) {
    const bool hasb = i + 1 < A.nsurf;
    const C* ra = inter + ((size_t)i * A.wy + r) * G.nxh;
    const C* rb = hasb ? inter + ((size_t)(i + 1) * A.wy + r) * G.nxh : nullptr;
    for (int s = threadIdx.x; s < gx; s += blockDim.x) za[s] = gather_x<R>(ra, rb, s, gx, hx);
    __syncthreads();
    C* res = block_fft<R>(za, zb, plan, 1, +1);
    for (int xw = threadIdx.x; xw < A.wx; xw += blockDim.x) {
      const int x = (A.ix0 + xw) % gx;
      const EvField& fa = A.f[A.nvol + i];
      outs[((size_t)fa.out_slot * A.wy + r) * A.wx + xw] = (float)res[x].x;
      if (hasb) {
        const EvField& fb = A.f[A.nvol + i + 1];
        outs[((size_t)fb.out_slot * A.wy + r) * A.wx + xw] = (float)res[x].y;
      }
    }
    __syncthreads();
  }
}

// x pass for interpolation coefficient grids, node-major layout: every
// node's (layer, field) values are contiguous, coef[(r wx + xw) K + l Fv + f],
// surface fields at offset L Fv + s.  Block (window row r, layer
// group g); the last group index holds the surface fields.
template <typename R>
__global__ void __launch_bounds__(256) k_xcoef(EvArgs A, Geom G, FftPlan plan, int LG, int K, float* coef) {
  extern __shared__ unsigned char smem[];
  using C = cpx<R>;
  const int gx = plan.n, r = blockIdx.x, g = blockIdx.y, hx = G.nx / 2;
  C* za = reinterpret_cast<C*>(smem);
  C* zb = za + gx;
  float* stage = reinterpret_cast<float*>(zb + gx);
  const int Fv = A.nvol;
  const int ngroups = Fv > 0 ? (A.nl + LG - 1) / LG : 0;
  const bool surf = g == ngroups;
  int nitems, base_off, l0 = 0;
  if (surf) {
    nitems = A.nsurf;
    base_off = A.nl * Fv;
  } else {
    l0 = g * LG;
    nitems = min(LG, A.nl - l0) * Fv;
    base_off = l0 * Fv;
  }
  const C* inter = reinterpret_cast<const C*>(A.inter);
  auto row = [&](int j) -> const C* {
    const int job = surf ? A.nvol * A.nl + j : (j % Fv) * A.nl + l0 + j / Fv;
    return inter + ((size_t)job * A.wy + r) * G.nxh;
  };
  for (int i = 0; i < nitems; i += 2) {
    const bool hasb = i + 1 < nitems;
    const C* ra = row(i);
    const C* rb = hasb ? row(i + 1) : nullptr;
    for (int s = threadIdx.x; s < gx; s += blockDim.x) za[s] = gather_x<R>(ra, rb, s, gx, hx);
    __syncthreads();
    C* res = block_fft<R>(za, zb, plan, 1, +1);
    for (int xw = threadIdx.x; xw < A.wx; xw += blockDim.x) {
      const int x = (A.ix0 + xw) % gx;
      stage[xw * nitems + i] = (float)res[x].x;
      if (hasb) stage[xw * nitems + i + 1] = (float)res[x].y;
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < A.wx * nitems; e += blockDim.x) {
    const int xw = e / nitems, j = e - xw * nitems;
    coef[((size_t)r * A.wx + xw) * K + base_off + j] = stage[e];
  }
}

// Wavefront version of the coefficient x pass: the (layer, field) pairs of
// the block are spread over its four wavefronts, each with its own FFT
// buffer; window values are staged in LDS and stored node-major after one
// block barrier.
template <typename R, int MAXE, int NS0>
__global__ void __launch_bounds__(256) k_xcoef_w(EvArgs A, Geom G, WPlan plan, int LG, int K, float* coef) {
  extern __shared__ unsigned char smem[];
  using C = cpx<R>;
  const int gx = plan.n, r = blockIdx.x, g = blockIdx.y, hx = G.nx / 2;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  C* zbuf = reinterpret_cast<C*>(smem) + (size_t)wave * wbuf_len(gx);
  float* stage = reinterpret_cast<float*>(reinterpret_cast<C*>(smem) + 4 * (size_t)wbuf_len(gx));
  const int Fv = A.nvol;
  const int ngroups = Fv > 0 ? (A.nl + LG - 1) / LG : 0;
  const bool surf = g == ngroups;
  int nitems, base_off, l0 = 0;
  if (surf) {
    nitems = A.nsurf;
    base_off = A.nl * Fv;
  } else {
    l0 = g * LG;
    nitems = min(LG, A.nl - l0) * Fv;
    base_off = l0 * Fv;
  }
  const C* inter = reinterpret_cast<const C*>(A.inter);
  auto row = [&](int j) -> const C* {
    const int job = surf ? A.nvol * A.nl + j : (j % Fv) * A.nl + l0 + j / Fv;
    return inter + ((size_t)job * A.wy + r) * G.nxh;
  };
  const int npairs = (nitems + 1) / 2;
  for (int pi = wave; pi < npairs; pi += 4) {
    const int i = 2 * pi;
    const bool hasb = i + 1 < nitems;
    const C* ra = row(i);
    const C* rb = hasb ? row(i + 1) : nullptr;
    for (int s = lane; s < gx; s += 64) zbuf[sk(s)] = gather_x<R>(ra, rb, s, gx, hx);
    wave_sync();
    wave_fft_any<R, MAXE, NS0>(zbuf, plan, +1, lane);
    for (int xw = lane; xw < A.wx; xw += 64) {
      int x = A.ix0 + xw;
      if (x >= gx) x -= gx;
      const C zx = zbuf[sk(x)];
      stage[xw * nitems + i] = (float)zx.x;
      if (hasb) stage[xw * nitems + i + 1] = (float)zx.y;
    }
    wave_sync();
  }
  __syncthreads();
  for (int e = threadIdx.x; e < A.wx * nitems; e += blockDim.x) {
    const int xw = e / nitems, j = e - xw * nitems;
    coef[((size_t)r * A.wx + xw) * K + base_off + j] = stage[e];
  }
}

// gather_x for the plane x pass, each row optionally multiplied by i kx
// first (ka, kb: 2 pi / lx for a row formed from its alias, else 0).
template <typename R>
__device__ __forceinline__ cpx<R> gather_x_dx(const cpx<R>* ra, const cpx<R>* rb, int s, int gx, int hx, R ka, R kb) {
  R zx = 0, zy = 0;
  auto row = [&](const cpx<R>* r, int p, R k) {
    cpx<R> v = r ? r[p] : mk((R)0, (R)0);
    if (k != (R)0) {
      const R kp = k * (R)p;
      v = mk(-kp * v.y, kp * v.x);
    }
    return v;
  };
  for (int p = s; p < hx; p += gx) {
    const cpx<R> va = row(ra, p, ka), vb = row(rb, p, kb);
    zx += va.x - vb.y;
    zy += va.y + vb.x;
  }
  int p0 = (gx - s) % gx;
  if (p0 == 0) p0 = gx;
  for (int p = p0; p < hx; p += gx) {
    const cpx<R> va = conjg(row(ra, p, ka)), vb = conjg(row(rb, p, kb));
    zx += va.x - vb.y;
    zy += va.y + vb.x;
  }
  return mk(zx, zy);
}

// Coefficient x pass in plane layout for the lengths of the workgroup
// transforms: coef[c][wy][wx] with c = l Fv + f for volume field f of layer l
// and c = L Fv + s for surface field s (the coefficient index of the
// node-major layout).  Block = (window row r, group of ppb job pairs); each
// pair of rows is transformed by the whole workgroup as one complex sequence
// and its window columns are written as two contiguous rows.
template <typename R, int N>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(N >= 3072 ? 3 : 4))) k_xplane_g(EvArgs A, Geom G, const cpx<R>* __restrict__ tw, int njobs, int ppb,
                                                  float* __restrict__ coef) {
  extern __shared__ unsigned char smem[];
  using C = cpx<R>;
  constexpr int T = N / 256;
  C* buf = reinterpret_cast<C*>(smem);
  const int r = blockIdx.x, hx = G.nx / 2, tid = threadIdx.x;
  const size_t plane = (size_t)A.wx * A.wy;
  const C* inter = reinterpret_cast<const C*>(A.inter);
  const int npair = (njobs + 1) / 2;
  const int pe = min(npair, (int)(blockIdx.y + 1) * ppb);
  auto cidx = [&](int job) {
    if (job >= A.nvol * A.nl) return job;  // surface: L Fv + s
    const int f = job / A.nl, l = job - f * A.nl;
    return l * A.nvol + f;
  };
  const R kunit = (R)(2.0 * M_PI / G.lx);
  // the row a job's transform reads (its alias's for an x derivative) and
  // the i kx factor applied to it
  auto src_row = [&](int job, R& k) -> const C* {
    int j = job;
    k = (R)0;
    if (job < A.nvol * A.nl) {
      const int f = job / A.nl;
      if (A.alias[f] >= 0) {
        j = A.alias[f] * A.nl + (job - f * A.nl);
        k = kunit;
      }
    }
    return inter + ((size_t)j * A.wy + r) * G.nxh;
  };
  for (int pi = blockIdx.y * ppb; pi < pe; ++pi) {
    const int ja = 2 * pi;
    const bool hasb = ja + 1 < njobs;
    R ka, kb = (R)0;
    const C* ra = src_row(ja, ka);
    const C* rb = hasb ? src_row(ja + 1, kb) : nullptr;
#pragma unroll 4
    for (int t = 0; t < T; ++t) {
      const int s = tid + 256 * t;
      buf[grp_in<N>(s)] = gather_x_dx<R>(ra, rb, s, N, hx, ka, kb);
    }
    grp_fft<R, N>(buf, tw, +1);
    float* oa = coef + (size_t)cidx(ja) * plane + (size_t)r * A.wx;
    float* ob = hasb ? coef + (size_t)cidx(ja + 1) * plane + (size_t)r * A.wx : nullptr;
    for (int xw = tid; xw < A.wx; xw += 256) {
      int x = A.ix0 + xw;
      if (x >= N) x -= N;
      const C zx = buf[grp_out<N>(x)];
      oa[xw] = (float)zx.x;
      if (hasb) ob[xw] = (float)zx.y;
    }
    __syncthreads();
  }
}

// Residue form of the plane x pass for grid lengths N = RS nx (RS in
// {2, 3, 4}, nx a power of two): each pair of rows, Hermitian-completed as
// one complex sequence of nx modes, gives X[RS s + r] as the nx-point
// transform of its modes times e^{2 pi i p r / N}; wavefront r transforms
// residue r and stores the window columns x = r (mod RS).  Same jobs,
// aliases and plane layout as k_xplane_g.
template <int RS, int NX>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NX >= 1024 ? 3 : 4))) k_xplane_r(
    EvArgs A, Geom G, const cpx<float>* __restrict__ tw, int njobs, int ppb, float* __restrict__ coef) {
  static_assert(RS >= 2 && RS <= 4, "residues");
  constexpr int N = RS * NX;
  constexpr int WL = NX + NX / 16 + 1;
  constexpr int PT = (NX / 2 + 255) / 256;  // kept modes p < nx/2 per thread
  using C = cpx<float>;
  extern __shared__ unsigned char smem[];
  C* buf = reinterpret_cast<C*>(smem);
  const int r = blockIdx.x, hx = G.nx / 2, tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const size_t plane = (size_t)A.wx * A.wy;
  const C* inter = reinterpret_cast<const C*>(A.inter);
  const int npair = (njobs + 1) / 2;
  const int pe = min(npair, (int)(blockIdx.y + 1) * ppb);
  auto cidx = [&](int job) {
    if (job >= A.nvol * A.nl) return job;  // surface: L Fv + s
    const int f = job / A.nl, l = job - f * A.nl;
    return l * A.nvol + f;
  };
  const float kunit = (float)(2.0 * M_PI / G.lx);
  auto src_row = [&](int job, float& k) -> const C* {
    int j = job;
    k = 0.f;
    if (job < A.nvol * A.nl) {
      const int f = job / A.nl;
      if (A.alias[f] >= 0) {
        j = A.alias[f] * A.nl + (job - f * A.nl);
        k = kunit;
      }
    }
    return inter + ((size_t)j * A.wy + r) * G.nxh;
  };
  // modulation e^{2 pi i p / N} of this thread's modes p (the table holds e^{-2 pi i m / N})
  C md[PT];
#pragma unroll
  for (int t = 0; t < PT; ++t) {
    const int pp = tid + 256 * t;
    const C w = tw[pp % N];
    md[t] = mk(w.x, -w.y);
  }
  // the pair's two rows, read one pair ahead: the next pair's loads are in
  // flight while the current pair is transformed and stored
  C la[PT], lb[PT];
  auto load_pair = [&](int pi) {
    const int ja = 2 * pi;
    float kk;
    const C* ra = src_row(ja, kk);
    const C* rb = ja + 1 < njobs ? src_row(ja + 1, kk) : nullptr;
#pragma unroll
    for (int t = 0; t < PT; ++t) {
      const int pp = tid + 256 * t;
      la[t] = pp < hx && pp < NX / 2 ? ra[pp] : mk(0.f, 0.f);
      lb[t] = rb && pp < hx && pp < NX / 2 ? rb[pp] : mk(0.f, 0.f);
    }
  };
  if (blockIdx.y * ppb < pe) load_pair(blockIdx.y * ppb);
  for (int pi = blockIdx.y * ppb; pi < pe; ++pi) {
    const int ja = 2 * pi;
    const bool hasb = ja + 1 < njobs;
    float ka, kb = 0.f;
    (void)src_row(ja, ka);
    if (hasb) (void)src_row(ja + 1, kb);
    // slot p (0 <= p < hx): a + i b; slot nx - p: conj(a) + i conj(b); the
    // Nyquist slot nx/2 stays zero
#pragma unroll
    for (int t = 0; t < PT; ++t) {
      const int pp = tid + 256 * t;
      if (pp < NX / 2) {
        C va = mk(0.f, 0.f), vb = mk(0.f, 0.f);
        if (pp < hx) {
          va = la[t];
          vb = lb[t];
          if (ka != 0.f) va = mk(-ka * (float)pp * va.y, ka * (float)pp * va.x);
          if (kb != 0.f) vb = mk(-kb * (float)pp * vb.y, kb * (float)pp * vb.x);
        }
        C zp = mk(va.x - vb.y, va.y + vb.x);                       // a + i b at +p
        C zm = pp > 0 ? mk(va.x + vb.y, vb.x - va.y) : mk(0.f, 0.f);  // conj(a) + i conj(b) at -p
        const C mc = conjg(md[t]);
#pragma unroll
        for (int q = 0; q < RS; ++q) {
          buf[q * WL + sk(pp)] = zp;
          if (pp > 0) buf[q * WL + sk(NX - pp)] = zm;
          zp = cmul(zp, md[t]);
          zm = cmul(zm, mc);
        }
        if (pp == 0)
#pragma unroll
          for (int q = 0; q < RS; ++q) buf[q * WL + sk(NX / 2)] = mk(0.f, 0.f);
      }
    }
    __syncthreads();
    if (pi + 1 < pe) load_pair(pi + 1);
    if (wave < RS) {
      C* b = buf + wave * WL;
      wave_fft_static<float, NX, RS, false>(b, tw, +1, lane);
      float* oa = coef + (size_t)cidx(ja) * plane + (size_t)r * A.wx;
      float* ob = hasb ? coef + (size_t)cidx(ja + 1) * plane + (size_t)r * A.wx : nullptr;
      const int x0 = ((wave - A.ix0) % RS + RS) % RS;
      for (int xw = x0 + RS * lane; xw < A.wx; xw += RS * 64) {
        int x = A.ix0 + xw;
        if (x >= N) x -= N;
        const C zx = b[sk((x - wave) / RS)];
        oa[xw] = zx.x;
        if (hasb) ob[xw] = zx.y;
      }
    }
    __syncthreads();
  }
}

// Coefficient x pass on skeleton heights: block (window row, field f); the
// R skeleton transforms of f are spread over the block's wavefronts, staged
// in LDS, and every layer is formed as sum_r T[l][r] s_r at each window node
// before the node-major store.  Blocks with f = Fv handle the surface fields.
template <typename R, int MAXE, int NS0>
__global__ void __launch_bounds__(256) k_xcoef_skel(EvArgs A, Geom G, WPlan plan, Skel skl, int L, int K, float* coef) {
  extern __shared__ unsigned char smem[];
  using C = cpx<R>;
  constexpr int WPB = 4;
  const int gx = plan.n, r = blockIdx.x, f = blockIdx.y, hx = G.nx / 2;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  C* zbuf = reinterpret_cast<C*>(smem) + (size_t)wave * wbuf_len(gx);
  float* stage = reinterpret_cast<float*>(reinterpret_cast<C*>(smem) + WPB * (size_t)wbuf_len(gx));
  const int Fv = A.nvol;
  const bool surf = f == Fv;
  const int nitems = surf ? A.nsurf : skl.R;
  const C* inter = reinterpret_cast<const C*>(A.inter);
  auto row = [&](int j) -> const C* {
    const int job = surf ? Fv * skl.R + j : f * skl.R + j;
    return inter + ((size_t)job * A.wy + r) * G.nxh;
  };
  const int npairs = (nitems + 1) / 2;
  for (int pi = wave; pi < npairs; pi += WPB) {
    const int i = 2 * pi;
    const bool hasb = i + 1 < nitems;
    const C* ra = row(i);
    const C* rb = hasb ? row(i + 1) : nullptr;
    for (int s = lane; s < gx; s += 64) zbuf[sk(s)] = gather_x<R>(ra, rb, s, gx, hx);
    wave_sync();
    wave_fft_any<R, MAXE, NS0>(zbuf, plan, +1, lane);
    for (int xw = lane; xw < A.wx; xw += 64) {
      int x = A.ix0 + xw;
      if (x >= gx) x -= gx;
      const C zx = zbuf[sk(x)];
      stage[i * A.wx + xw] = (float)zx.x;
      if (hasb) stage[(i + 1) * A.wx + xw] = (float)zx.y;
    }
    wave_sync();
  }
  __syncthreads();
  if (surf) {
    for (int e = threadIdx.x; e < A.wx * nitems; e += blockDim.x) {
      const int xw = e / nitems, j = e - xw * nitems;
      coef[((size_t)r * A.wx + xw) * K + (size_t)L * Fv + j] = stage[j * A.wx + xw];
    }
    return;
  }
  const float* T = A.f[f].vf == 1 ? skl.ts : skl.tc;
  for (int e = threadIdx.x; e < A.wx * L; e += blockDim.x) {
    const int xw = e / L, l = e - xw * L;
    float acc = 0.f;
    for (int j = 0; j < skl.R; ++j) acc += T[l * skl.R + j] * stage[j * A.wx + xw];
    coef[((size_t)r * A.wx + xw) * K + (size_t)l * Fv + f] = acc;
  }
}

// Coefficient x pass on skeleton heights as a dense contraction on the
// matrix cores.  For window row r and a tile of DX_T window nodes, every item
// (a skeleton height of a volume field, or a surface field) is evaluated at
// the nodes X as  out[item][x] = sum_{p < nx/2} c_p Re(a_p e^{2 pi i p X / gx}),
// c_0 = 1, c_p = 2: a real GEMM of the interleaved (Re, Im) mode rows against
// the matrix [c_p cos; -c_p sin], formed from the FP32 twiddle table in LDS
// (index p X mod gx, which also folds modes above gx/2 when gx < nx), on FP32
// MFMA with FP32 accumulation.  Each layer is then sum_j T[l][j] out[f R + j]
// and every node's run of K coefficients is stored contiguously.
constexpr int DX_T = 64, DX_KC = 32, DX_MAXMT = 8;
// LDS row strides chosen so that the MFMA operand reads (16 rows x 4
// consecutive k, or 4 k-rows x 16 columns) and the accumulator stores hit 64
// distinct banks; the results overlay the operand tiles.
constexpr int DX_SA = DX_KC + 4, DX_SB = DX_T + 16, DX_SS = DX_T + 4;

// The B operand of the contraction for every node tile: row kk = 2p + c of
// tile t holds c_p cos(theta) (c = 0) or -c_p sin(theta) (c = 1) at the 64
// nodes X of the tile, theta = 2 pi p X / gx, from the FP32 table entry
// p X mod gx; rows with p >= nx/2 (up to the chunk-padded row count) are
// zero.  It does not depend on the window row, so it is formed once per
// evaluation instead of once per workgroup.  basis: [ntx][dft_rows(hx)][DX_T].
__host__ __device__ constexpr int dft_rows(int hx) { return (2 * hx + DX_KC - 1) / DX_KC * DX_KC; }

// Host mirror of the basis rows k_xcoef_dft reads for hx kept x modes: chunk
// k0 (a multiple of DX_KC below 2 hx) reads rows 2 p0 + brow, p0 = k0 / 2,
// brow < DX_KC, and prefetches the next chunk the same way.  Returns the
// largest row read; it must stay below dft_rows(hx), the rows per node tile
// of the basis (a basis sized by the unpadded 2 hx rows once let the last
// chunk read past the allocation).
int dft_last_row_read(int hx) {
  const int Kr = 2 * hx;
  int last = -1;
  for (int k0 = 0; k0 < Kr; k0 += DX_KC) {
    const int p0 = k0 >> 1;
    last = std::max(last, 2 * p0 + DX_KC - 1);
    if (k0 + DX_KC < Kr) last = std::max(last, 2 * (p0 + DX_KC / 2) + DX_KC - 1);
  }
  return last;
}

__global__ void __launch_bounds__(256) k_dft_basis(const cf* __restrict__ tw, int gx, int ix0, int hx, int ntx,
                                                   float* __restrict__ basis) {
  const int Kp = dft_rows(hx);
  const int total = ntx * Kp * DX_T;  // < 2^31: checked by the caller
  const bool small = (long long)hx * gx < (1ll << 31);  // p X fits in 32 bits
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int n = e % DX_T;
    const int kk = (e / DX_T) % Kp;
    const int t = e / (DX_T * Kp);
    const int X = (ix0 + t * DX_T + n) % gx;
    const int p = kk >> 1;
    float v = 0.f;
    if (p < hx) {
      const cf w = tw[small ? (p * X) % gx : (int)(((long long)p * X) % gx)];
      const float cp = p == 0 ? 1.f : 2.f;
      v = (kk & 1) ? cp * w.y : cp * w.x;
    }
    basis[e] = v;
  }
}

__global__ void __launch_bounds__(256) k_xcoef_dft(EvArgs A, Geom G, const float* __restrict__ basis, Skel skl,
                                                   int L, int K, int nitems, float* __restrict__ coef) {
  extern __shared__ __align__(16) unsigned char smem[];
  typedef float v4f __attribute__((ext_vector_type(4)));
  // the tiles of one window row read the same mode rows: consecutive tiles
  // go to the workgroups of one XCD, so its L2 serves the shared rows
  const int tile = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int r = tile / gridDim.x, xt = tile - r * gridDim.x, x0 = xt * DX_T;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int hx = G.nx / 2, Kr = 2 * hx;
  const int mt_n = (nitems + 15) / 16, rows = mt_n * 16;
  const int Fv = A.nvol, R = skl.R;
  float* Ts = reinterpret_cast<float*>(smem);      // [2][R][L]: C-type then S-type factors
  float* As = Ts + ((2 * L * R + 3) & ~3);         // [rows][DX_SA]
  float* Bs = As + rows * DX_SA;                   // [DX_KC][DX_SB]
  float* S = As;                                   // after the contraction: [rows][DX_SS]
  // factor j of layer l at j L + l, so that the threads of a wavefront (one
  // layer each) read consecutive banks in the layer combine
  for (int i = tid; i < L * R; i += 256) {
    const int l = i / R, j = i - l * R;
    Ts[j * L + l] = skl.tc[i];
    Ts[L * R + j * L + l] = skl.ts[i];
  }
  const cf* inter = reinterpret_cast<const cf*>(A.inter);
  static_assert(DX_T == 64 && DX_KC == 32, "fills assume 64 nodes and 16 modes per chunk");
  // A fill: thread -> mode pp = tid & 15 of items it = tid >> 4, it + 16, ...
  const int pp = tid & 15, it0 = tid >> 4;
  const int nA = (rows + 15) / 16;  // items per thread (<= 8)
  // B fill: thread -> 8 consecutive floats (two float4) of the 32 x 64 chunk
  const int brow = tid >> 3, bcol = (tid & 7) * 8;
  const float* btile = basis + (size_t)xt * dft_rows(hx) * DX_T;  // rows >= Kr are zero
  cf pre[DX_MAXMT];
  v4f preb0, preb1;
  auto fetchA = [&](int p0) {
#pragma unroll
    for (int q = 0; q < DX_MAXMT; ++q) {
      const int item = it0 + 16 * q, p = p0 + pp;
      cf v = mk(0.f, 0.f);
      if (q < nA && item < nitems && p < hx) v = inter[((size_t)item * A.wy + r) * G.nxh + p];
      pre[q] = v;
    }
    const v4f* bsrc = reinterpret_cast<const v4f*>(btile + (size_t)(2 * p0 + brow) * DX_T + bcol);
    preb0 = bsrc[0];
    preb1 = bsrc[1];
  };
  constexpr int MTW = DX_MAXMT / 4;  // M tiles per wavefront
  v4f acc[MTW][4];
#pragma unroll
  for (int i = 0; i < MTW; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  fetchA(0);
  for (int k0 = 0; k0 < Kr; k0 += DX_KC) {
    __syncthreads();
    const int p0 = k0 >> 1;
#pragma unroll
    for (int q = 0; q < DX_MAXMT; ++q) {
      const int item = it0 + 16 * q;
      if (q < nA && item < rows) *reinterpret_cast<float2*>(&As[item * DX_SA + 2 * pp]) = make_float2(pre[q].x, pre[q].y);
    }
    *reinterpret_cast<v4f*>(&Bs[brow * DX_SB + bcol]) = preb0;
    *reinterpret_cast<v4f*>(&Bs[brow * DX_SB + bcol + 4]) = preb1;
    __syncthreads();
    if (k0 + DX_KC < Kr) fetchA(p0 + DX_KC / 2);  // next chunk in flight during the products
#pragma unroll
    for (int kk = 0; kk < DX_KC; kk += 4) {
      const int krow = kk + (lane >> 4);
      float b[4];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) b[nt] = Bs[krow * DX_SB + nt * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < MTW; ++i) {
        const int mt = wave + 4 * i;
        if (mt < mt_n) {
          const float a = As[(mt * 16 + (lane & 15)) * DX_SA + krow];
#pragma unroll
          for (int nt = 0; nt < 4; ++nt) acc[i][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[nt], acc[i][nt], 0, 0, 0);
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MTW; ++i) {
    const int mt = wave + 4 * i;
    if (mt < mt_n) {
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          S[(mt * 16 + 4 * (lane >> 4) + q) * DX_SS + nt * 16 + (lane & 15)] = acc[i][nt][q];
    }
  }
  __syncthreads();
  // layers: thread -> one coefficient index kidx of every node of the tile
  const int nvk = L * Fv;
  const int nodes = min(DX_T, A.wx - x0);
  for (int kb = 0; kb < K; kb += 256) {
    const int kidx = kb + tid;
    if (kidx >= K) break;
    float* dst = coef + ((size_t)r * A.wx + x0) * K + kidx;
    if (kidx < nvk) {
      const int l = kidx / Fv, f = kidx - l * Fv;
      const float* T = Ts + (A.f[f].vf == 1 ? L * R : 0) + l;
      const float* srow = S + (f * R) * DX_SS;
      for (int n4 = 0; n4 < nodes; n4 += 4) {
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int j = 0; j < R; ++j) {
          const float tj = T[j * L];
          const float4 sv = *reinterpret_cast<const float4*>(srow + j * DX_SS + n4);
          v.x += tj * sv.x; v.y += tj * sv.y; v.z += tj * sv.z; v.w += tj * sv.w;
        }
        const float vv[4] = {v.x, v.y, v.z, v.w};
        for (int q = 0; q < 4 && n4 + q < nodes; ++q) dst[(size_t)(n4 + q) * K] = vv[q];
      }
    } else {
      const float* srow = S + (Fv * R + (kidx - nvk)) * DX_SS;
      for (int n = 0; n < nodes; ++n) dst[(size_t)n * K] = srow[n];
    }
  }
}

__global__ void k_fill(float* p, size_t n, float v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

// ---------------------------------------------------------------- host side
struct EvalWork {
  void* inter = nullptr;
  size_t inter_bytes = 0;
  void* basis = nullptr;  // B operand of the DFT coefficient pass
  size_t basis_bytes = 0;
  double* zdev = nullptr;
  size_t zcap = 0;
  // caller-provided scratch for one call (null: the buffers above, grown on demand)
  char* ext = nullptr;
  size_t ext_inter = 0, ext_basis = 0;  // capacities: intermediates first, then the basis
  // caller-provided twiddle tables of the grid for one call (null: the handle's cache)
  void* ext_twx = nullptr;
  void* ext_twy = nullptr;
  int ext_gx = 0, ext_gy = 0;
};

namespace {

void check_grid(const swense_hos* h, const swense_grid_desc* gd) {
  SW_REQUIRE(gd != nullptr, "null grid descriptor");
  SW_REQUIRE(gd->gx >= 2 && is_235_smooth(gd->gx), "gx must be >= 2 and 2/3/5-smooth");
  if (h->G.ny > 1) SW_REQUIRE(gd->gy >= 2 && is_235_smooth(gd->gy), "gy must be >= 2 and 2/3/5-smooth");
  else SW_REQUIRE(gd->gy == 1 && gd->wy == 1 && gd->iy0 == 0, "2D grids need gy = wy = 1, iy0 = 0");
  SW_REQUIRE(gd->wx >= 1 && gd->wx <= gd->gx && gd->wy >= 1 && gd->wy <= gd->gy, "window larger than the grid");
  SW_REQUIRE(gd->ix0 >= 0 && gd->ix0 < gd->gx && gd->iy0 >= 0 && gd->iy0 < gd->gy, "window origin outside the grid");
  SW_REQUIRE(gd->nl >= 1 && gd->z != nullptr, "need at least one layer");
  for (int l = 1; l < gd->nl; ++l) SW_REQUIRE(gd->z[l] > gd->z[l - 1], "layer heights must ascend");
}

void ensure(void** p, size_t* cap, size_t bytes) {
  if (*cap >= bytes) return;
  if (*p) SW_HIP(hipFree(*p));
  *p = nullptr;
  *cap = 0;
  SW_HIP(hipMalloc(p, bytes));
  *cap = bytes;
}

EvalWork* work(swense_hos* h) {
  if (!h->ev) h->ev = new EvalWork();
  return h->ev;
}

// Spectral source of a volume field bit.
void vol_source(swense_hos* h, int f, EvField& e) {
  const bool t = f >= F_PHIT;
  const int base = t ? f - F_PHIT : f;  // PHI U V W
  const cd *a, *at, *eta, *etat;
  eval_sources(h, &a, &at, &eta, &etat);
  e.src = t ? at : a;
  e.vf = base == 3 ? 1 : 0;
  e.mult = base == 0 ? 0 : (base == 1 ? 1 : (base == 2 ? 2 : 3));
}

// Plan the evaluation: which spectral fields run, where each lands.
// Output (pre = 0): volume slots in bit order of the mask (incl. P), then
// surface slots.  Coefficients (pre = 1): volume fields in bit order (no P),
// then surface fields.
void plan_fields(swense_hos* h, unsigned mask, bool pre, EvArgs& A, int* out_of_field, int* nvol_out,
                 int* nsurf_out) {
  std::memset(&A, 0, sizeof(A));
  A.p_slot = -1;
  const bool three = h->G.ny > 1;
  int vslot = 0, sslot = 0;
  int vol_slot_of[kNumFields], srf_slot_of[kNumFields];
  for (int f = 0; f < kNumFields; ++f) vol_slot_of[f] = srf_slot_of[f] = -1;
  for (int f = 0; f < kNumFields; ++f) {
    if (!(mask & (1u << f))) continue;
    if (f == F_ETA || f == F_ETAT) srf_slot_of[f] = sslot++;
    else if (f == F_P && pre) continue;
    else vol_slot_of[f] = vslot++;
  }
  *nvol_out = vslot;
  *nsurf_out = sslot;
  const bool need_p = !pre && (mask & SWENSE_P);
  if (need_p) A.p_slot = vol_slot_of[F_P];
  // spectral volume fields
  int nv = 0;
  for (int f : {F_PHI, F_U, F_V, F_W, F_PHIT, F_UT, F_VT, F_WT}) {
    const bool want = vol_slot_of[f] >= 0;
    int prole = 0;
    if (need_p) prole = f == F_PHIT ? 1 : (f == F_U ? 2 : (f == F_V ? 3 : (f == F_W ? 4 : 0)));
    if (!want && !prole) continue;
    if (!three && (f == F_V || f == F_VT)) continue;  // identically zero in 2D
    EvField& e = A.f[nv];
    vol_source(h, f, e);
    e.out_slot = vol_slot_of[f];
    e.p_role = prole;
    if (out_of_field) out_of_field[f] = nv;
    ++nv;
  }
  A.nvol = nv;
  int ns = 0;
  for (int f : {F_ETA, F_ETAT}) {
    if (srf_slot_of[f] < 0) continue;
    EvField& e = A.f[nv + ns];
    const cd *a, *at, *eta, *etat;
    eval_sources(h, &a, &at, &eta, &etat);
    e.src = f == F_ETA ? eta : etat;
    e.vf = 2;
    e.mult = 0;
    e.out_slot = srf_slot_of[f];
    if (out_of_field) out_of_field[f] = ns;
    ++ns;
  }
  A.nsurf = ns;
}

template <typename R>
void eval_t(swense_hos* h, const swense_grid_desc* gd, const double* zdev, unsigned mask, bool pre, float* out,
            const Skel* skel, int* plane_out) {
  launch_modes(h);
  EvArgs A;
  int nvo = 0, nso = 0;
  plan_fields(h, mask, pre, A, nullptr, &nvo, &nso);
  if (plane_out) *plane_out = 0;
  {
    int ns = 0;
    for (int f = 0; f < A.nvol + A.nsurf; ++f) {
      int k = 0;
      while (k < ns && A.srcs[k] != A.f[f].src) ++k;
      if (k == ns) {
        SW_REQUIRE(ns < 4, "too many spectral sources");
        A.srcs[ns++] = A.f[f].src;
      }
      A.sid[f] = k;
    }
  }
  for (int f = 0; f < kMaxEvFields; ++f) A.alias[f] = -1;
  const bool use_skel = pre && skel && skel->R > 0;
  A.z = use_skel ? skel->zeta : zdev;
  A.nl = use_skel ? skel->R : gd->nl;
  A.gx = gd->gx;
  A.gy = h->G.ny > 1 ? gd->gy : 1;
  A.ix0 = gd->ix0;
  A.iy0 = gd->iy0;
  A.wx = gd->wx;
  A.wy = gd->wy;
  A.pre = pre ? 1 : 0;
  A.out = out;
  A.nvol_out = nvo;
  const size_t plane = (size_t)A.wy * A.wx;
  // zero-fill outputs that no transform writes (v, v_t in 2D)
  if (h->G.ny == 1 && !pre) {
    for (int f : {F_V, F_VT}) {
      if (!(mask & (1u << f))) continue;
      int slot = 0;
      for (int g = 0; g < f; ++g)
        if ((mask & (1u << g)) && g != F_ETA && g != F_ETAT && !(pre && g == F_P)) ++slot;
      const size_t n = (size_t)A.nl * plane;
      SW_LAUNCH(h, SWENSE_K_AUX, k_fill, dim3((n + 255) / 256), dim3(256), 0, h->st, out + (size_t)slot * n, n, 0.0f);
      SW_HIP(hipGetLastError());
    }
  }
  const int njobs = A.nvol * A.nl + A.nsurf;
  if (njobs == 0) return;
  EvalWork* w = work(h);
  const size_t csz = sizeof(cpx<R>);
  const size_t inter_need = (size_t)njobs * A.wy * h->G.nxh * csz;
  if (w->ext) {
    if (inter_need > w->ext_inter) throw SwenseError{SWENSE_ENOMEM, "scratch too small for the evaluation rows"};
    A.inter = w->ext;
  } else {
    void* before = w->inter;
    ensure(&w->inter, &w->inter_bytes, inter_need);
    if (w->inter != before) ++h->scratch_epoch;
    A.inter = w->inter;
  }
  TwiddleCache& tc = h->tw;
  FftPlan py = (w->ext_twy && w->ext_gy == A.gy) ? TwiddleCache::plan_with(A.gy, w->ext_twy) : tc.get(A.gy, sizeof(R) == 8);
  FftPlan px = (w->ext_twx && w->ext_gx == A.gx) ? TwiddleCache::plan_with(A.gx, w->ext_twx) : tc.get(A.gx, sizeof(R) == 8);
  int naliased = 0;
  if constexpr (sizeof(R) == 4) {
    // workgroup y pass and plane x pass: an x-derivative field reuses the y
    // transform of the field of the same source and vertical factor
    const bool ygrp = h->G.ny > 1 && grp_len_ok(py.n) && py.n >= h->G.ny && (h->G.ny + 255) / 256 <= 4;
    const bool xplane = pre && !use_skel && grp_len_ok(px.n);
    if (ygrp && xplane)
      for (int f = 0; f < A.nvol; ++f) {
        if (A.f[f].mult != 1) continue;
        for (int g = 0; g < A.nvol; ++g)
          if (A.f[g].mult == 0 && A.f[g].vf == A.f[f].vf && A.sid[g] == A.sid[f] && A.alias[g] < 0) {
            A.alias[f] = g;
            ++naliased;
            break;
          }
      }
  }
  if (h->prof.on) {
    // compulsory: each distinct spectrum read once, the window rows written
    // once and read once by the x pass, the outputs written once; model: the
    // two-pass transform bytes of every (field, layer) job on the refined grid
    int nsrc = 0;
    for (int f = 0; f < A.nvol + A.nsurf; ++f) nsrc = std::max(nsrc, A.sid[f] + 1);
    const double rows = (double)(njobs - naliased * A.nl) * A.wy * h->G.nxh * csz;
    const double outb = (double)(pre ? A.nvol * gd->nl + A.nsurf : (size_t)(nvo * gd->nl + nso)) * plane * 4.0;
    const double tb = (double)njobs * 2.0 * sizeof(R) * (double)A.gx * A.gy;
    h->prof.bytes[SWENSE_K_YINV_EVAL] += (double)nsrc * h->nc * sizeof(cd) + rows;
    h->prof.tbytes[SWENSE_K_YINV_EVAL] += tb;
    h->prof.bytes[SWENSE_K_XEVAL] += rows + outb;
    h->prof.tbytes[SWENSE_K_XEVAL] += tb;
  }
  // y pass
  SW_REQUIRE(njobs <= 65535, "too many (field, layer) pairs");
  const int tq = (h->G.ny + 255) / 256;
  bool ydone = false;
  if constexpr (sizeof(R) == 4) {
    const int ny = h->G.ny, rs = py.n / std::max(ny, 1);
    if ((ny == 256 || ny == 512 || ny == 1024) && rs >= 2 && rs <= 4 && rs * ny == py.n) {
      // residue form: one wavefront per output residue y mod rs
      const size_t lds = (size_t)rs * (ny + ny / 16 + 1) * csz;
      const int nly = (A.nvol > 0 ? A.nl : 0) + (A.nsurf > 0 ? 1 : 0);
      dim3 grid((unsigned)(h->G.nxh * nly));  // nly = 0: no fields, nothing launched
      const cpx<float>* twy = reinterpret_cast<const cpx<float>*>(py.tw);
#define L_YR(RS, NY) sw_launch(h, SWENSE_K_YINV_EVAL, &k_yinv_eval_r<RS, NY, NY / 256>, grid, dim3(256), lds, h->st, A, h->G, twy)
#define L_YRN(RS)                  \
  switch (ny) {                    \
    case 256: L_YR(RS, 256); break;  \
    case 512: L_YR(RS, 512); break;  \
    default: L_YR(RS, 1024); break;  \
  }
      if (nly > 0) switch (rs) {
          case 2: L_YRN(2); break;
          case 3: L_YRN(3); break;
          default: L_YRN(4); break;
        }
#undef L_YRN
#undef L_YR
      ydone = true;
    } else if (ny >= 16 && ny <= 512 && ny % 2 == 0 && rs >= 2 && rs <= 4 && rs * ny == py.n && !grp_len_ok(py.n)) {
      // residue form with a runtime plan of the mode count (refinements of
      // 2-4 times a 2/3/5-smooth count whose refined length has no
      // compile-time transform); its twiddles are read from the refined
      // length's table, so no other table is needed
      FftPlan sub{};
      sub.n = ny;
      sub.tw = py.tw;
      const WPlan pny = make_wplan(sub);
      const size_t lds = (size_t)rs * wbuf_len(ny) * csz;
      const int nly = (A.nvol > 0 ? A.nl : 0) + (A.nsurf > 0 ? 1 : 0);
      dim3 grid((unsigned)(h->G.nxh * nly));
      const cpx<float>* twy = reinterpret_cast<const cpx<float>*>(py.tw);
#define L_RR(RS, TQ)   sw_launch(h, SWENSE_K_YINV_EVAL, &k_yinv_eval_rr<RS, TQ, 8>, grid, dim3(256), lds, h->st, A, h->G, twy, pny)
#define L_RRN(RS)                if (ny <= 256) L_RR(RS, 1);   else L_RR(RS, 2);
      if (nly > 0) switch (rs) {
          case 2: L_RRN(2); break;
          case 3: L_RRN(3); break;
          default: L_RRN(4); break;
        }
#undef L_RRN
#undef L_RR
      ydone = true;
    } else if (h->G.ny > 1 && grp_len_ok(py.n) && py.n >= h->G.ny && tq <= 4) {
    // one workgroup per (column, layer): the layer's fields share the FP64 factors
    const size_t lds = grp_lds_len(py.n) * csz;
    dim3 grid(h->G.nxh, (A.nvol > 0 ? A.nl : 0) + (A.nsurf > 0 ? 1 : 0));
    const cpx<R>* twy = reinterpret_cast<const cpx<R>*>(py.tw);
#define L_YG(N)                                                                                              \
  if (tq <= 1) sw_launch(h, SWENSE_K_YINV_EVAL, &k_yinv_eval_g<R, N, 1>, grid, dim3(256), lds, h->st, A, h->G, twy); \
  else if (tq <= 2) sw_launch(h, SWENSE_K_YINV_EVAL, &k_yinv_eval_g<R, N, 2>, grid, dim3(256), lds, h->st, A, h->G, twy); \
  else sw_launch(h, SWENSE_K_YINV_EVAL, &k_yinv_eval_g<R, N, 4>, grid, dim3(256), lds, h->st, A, h->G, twy);
    SW_B4_DISPATCH(py.n, L_YG);
#undef L_YG
      ydone = true;
    }
  }
  if (ydone) {
  } else if (py.n <= (sizeof(R) == 4 ? 4096 : 2048)) {
    const WPlan wp = make_wplan(py);
    const size_t lds = 4ull * wbuf_len(py.n) * csz;
    dim3 grid((h->G.nxh + 3) / 4, njobs);
#define L_YEV(E, N) sw_launch(h, SWENSE_K_YINV_EVAL, &k_yinv_eval_w<R, E, N>, grid, dim3(256), lds, h->st, A, h->G, wp)
    SW_FFT_DISPATCH(py.n, L_YEV);
#undef L_YEV
  } else {
    int TW = 1;
    long cap = 65536 / (2L * py.n * (long)csz);
    while (TW * 2 <= cap && TW * 2 <= 256) TW *= 2;
    const size_t lds = 2ull * TW * py.n * csz;
    dim3 grid((h->G.nxh + TW - 1) / TW, njobs);
    sw_launch(h, SWENSE_K_YINV_EVAL, &k_yinv_eval<R>, grid, dim3(256), lds, h->st, A, h->G, py, TW);
  }
  if (use_skel) {
    const int Fv = A.nvol;
    const int L = gd->nl;
    const int K = L * Fv + A.nsurf;
    const int nitems = Fv * skel->R + A.nsurf;
    if constexpr (sizeof(R) == 4) {
      const int rows = (nitems + 15) / 16 * 16;
      const size_t lds_dft = ((2ull * L * skel->R + 3) / 4 * 4 +
                              std::max((size_t)rows * DX_SA + (size_t)DX_KC * DX_SB, (size_t)rows * DX_SS)) *
                             sizeof(float);
      if (nitems <= DX_MAXMT * 16 && lds_dft <= 160 * 1024) {
        const int ntx = (A.wx + DX_T - 1) / DX_T;
        const int hx = h->G.nx / 2;
        SW_REQUIRE(dft_last_row_read(hx) < dft_rows(hx), "DFT basis rows do not cover the rows the pass reads");
        const size_t nb = (size_t)ntx * dft_rows(hx) * DX_T;
        SW_REQUIRE(nb < (1ull << 31), "coefficient window too wide");
        float* basis;
        if (w->ext) {
          if (nb * sizeof(float) > w->ext_basis) throw SwenseError{SWENSE_ENOMEM, "scratch too small for the DFT basis"};
          basis = reinterpret_cast<float*>(w->ext + w->ext_inter);
        } else {
          void* before = w->basis;
          ensure(&w->basis, &w->basis_bytes, nb * sizeof(float));
          if (w->basis != before) ++h->scratch_epoch;
          basis = reinterpret_cast<float*>(w->basis);
        }
        const unsigned bblk = (unsigned)std::min<size_t>((nb + 255) / 256, 4096);
        sw_launch(h, SWENSE_K_AUX, &k_dft_basis, dim3(bblk), dim3(256), 0, h->st, reinterpret_cast<const cf*>(px.tw),
                  px.n, A.ix0, hx, ntx, basis);
        dim3 grid(ntx, A.wy);
        sw_launch(h, SWENSE_K_XEVAL, &k_xcoef_dft, grid, dim3(256), lds_dft, h->st, A, h->G, basis, *skel, L, K,
                  nitems, out);
        return;
      }
    }
    const int maxitems = std::max(skel->R, A.nsurf);
    const size_t lds = 4ull * wbuf_len(px.n) * csz + (size_t)A.wx * maxitems * sizeof(float);
    SW_REQUIRE(px.n <= (sizeof(R) == 4 ? 4096 : 2048) && lds <= 160 * 1024, "grid row too long for one workgroup");
    const WPlan wp = make_wplan(px);
    dim3 grid(A.wy, Fv + (A.nsurf > 0 ? 1 : 0));
#define L_XS(E, N) sw_launch(h, SWENSE_K_XEVAL, &k_xcoef_skel<R, E, N>, grid, dim3(256), lds, h->st, A, h->G, wp, *skel, L, K, out)
    SW_FFT_DISPATCH(px.n, L_XS);
#undef L_XS
    return;
  }
  if constexpr (sizeof(R) == 4) {
  const int nxm = h->G.nx, rsx = px.n / std::max(nxm, 1);
  if (pre && (nxm == 256 || nxm == 512 || nxm == 1024) && rsx >= 2 && rsx <= 4 && rsx * nxm == px.n) {
    // plane layout, residue form: one wavefront per output residue x mod rsx
    if (plane_out) *plane_out = 1;
    constexpr int ppb = 4;
    const int npair = (njobs + 1) / 2;
    const size_t lds = (size_t)rsx * (nxm + nxm / 16 + 1) * csz;
    dim3 grid(A.wy, (npair + ppb - 1) / ppb);
    const cpx<float>* twx = reinterpret_cast<const cpx<float>*>(px.tw);
#define L_XR(RS, NX) sw_launch(h, SWENSE_K_XEVAL, &k_xplane_r<RS, NX>, grid, dim3(256), lds, h->st, A, h->G, twx, njobs, ppb, out)
#define L_XRN(RS)                  \
  switch (nxm) {                   \
    case 256: L_XR(RS, 256); break;  \
    case 512: L_XR(RS, 512); break;  \
    default: L_XR(RS, 1024); break;  \
  }
    switch (rsx) {
      case 2: L_XRN(2); break;
      case 3: L_XRN(3); break;
      default: L_XRN(4); break;
    }
#undef L_XRN
#undef L_XR
    return;
  }
  if (pre && grp_len_ok(px.n)) {
    // plane layout: each pair of rows transformed by a whole workgroup
    if (plane_out) *plane_out = 1;
    constexpr int ppb = 4;
    const int npair = (njobs + 1) / 2;
    const size_t lds = grp_lds_len(px.n) * csz;
    dim3 grid(A.wy, (npair + ppb - 1) / ppb);
    const cpx<R>* twx = reinterpret_cast<const cpx<R>*>(px.tw);
#define L_XP(N) sw_launch(h, SWENSE_K_XEVAL, &k_xplane_g<R, N>, grid, dim3(256), lds, h->st, A, h->G, twx, njobs, ppb, out)
    SW_B4_DISPATCH(px.n, L_XP);
#undef L_XP
    return;
  }
  }
  if (pre) {
    const int Fv = A.nvol;
    const int LG = Fv > 0 ? std::max(1, 16 / Fv) : 1;
    const int ngroups = Fv > 0 ? (A.nl + LG - 1) / LG : 0;
    const int K = A.nl * Fv + A.nsurf;
    const int maxitems = std::max(LG * Fv, A.nsurf);
    dim3 grid(A.wy, ngroups + (A.nsurf > 0 ? 1 : 0));
    const size_t ldsw = 4ull * wbuf_len(px.n) * csz + (size_t)A.wx * maxitems * sizeof(float);
    if (px.n <= (sizeof(R) == 4 ? 4096 : 2048) && ldsw <= 160 * 1024) {
      const WPlan wp = make_wplan(px);
#define L_XC(E, N) sw_launch(h, SWENSE_K_XEVAL, &k_xcoef_w<R, E, N>, grid, dim3(256), ldsw, h->st, A, h->G, wp, LG, K, out)
      SW_FFT_DISPATCH(px.n, L_XC);
#undef L_XC
      return;
    }
    const size_t lds = 2ull * px.n * csz + (size_t)A.wx * maxitems * sizeof(float);
    SW_REQUIRE(lds <= 160 * 1024, "grid row too long for one workgroup");
    sw_launch(h, SWENSE_K_XEVAL, &k_xcoef<R>, grid, dim3(256), lds, h->st, A, h->G, px, LG, K, out);
    return;
  }
  if (A.nvol > 0) {
    const size_t lds = 2ull * px.n * csz + 4ull * A.wx * sizeof(R);
    SW_REQUIRE(lds <= 160 * 1024, "grid row too long for one workgroup");
    if (lds > 65536)
      SW_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_xeval_vol<R>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    SW_LAUNCH(h, SWENSE_K_XEVAL, k_xeval_vol<R>, dim3(A.wy, A.nl), dim3(256), lds, h->st, A, h->G, px);
    SW_HIP(hipGetLastError());
  }
  if (A.nsurf > 0) {
    const size_t lds = 2ull * px.n * csz;
    if (lds > 65536)
      SW_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_xeval_surf<R>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    SW_LAUNCH(h, SWENSE_K_XEVAL_SURF, k_xeval_surf<R>, dim3(A.wy), dim3(256), lds, h->st, A, h->G, px);
    SW_HIP(hipGetLastError());
  }
}

void eval_dispatch(swense_hos* h, const swense_grid_desc* gd, const double* zdev, unsigned mask, bool pre,
                   float* out, const Skel* skel = nullptr, int* plane = nullptr) {
  if (h->fp64) eval_t<double>(h, gd, zdev, mask, pre, out, skel, plane);
  else eval_t<float>(h, gd, zdev, mask, pre, out, skel, plane);
}

size_t grid_floats(const swense_hos* h, const swense_grid_desc* gd, unsigned mask, bool pre) {
  size_t nv = 0, ns = 0;
  for (int f = 0; f < kNumFields; ++f) {
    if (!(mask & (1u << f))) continue;
    if (f == F_ETA || f == F_ETAT) ++ns;
    else if (pre && (f == F_P || (h->G.ny == 1 && (f == F_V || f == F_VT)))) continue;
    else ++nv;
  }
  const size_t plane = (size_t)gd->wx * gd->wy;
  return nv * gd->nl * plane + ns * plane;
}

}  // namespace

void check_grid_desc(const swense_hos* h, const swense_grid_desc* gd) { check_grid(h, gd); }

extern "C" int swense_selfcheck_launch_geometry(int max_nx) {
  // host-only: for every even mode count up to max_nx, the DFT coefficient
  // pass reads no basis row past the ones allocated per node tile
  for (int nx = 2; nx <= max_nx; nx += 2) {
    const int hx = nx / 2;
    if (dft_last_row_read(hx) >= dft_rows(hx)) return nx;
  }
  return 0;
}

void eval_scratch_need(swense_hos* h, const swense_grid_desc* gd, unsigned cm, int skel_r, size_t* inter,
                       size_t* basis) {
  EvArgs A;
  int nvo = 0, nso = 0;
  plan_fields(h, cm, true, A, nullptr, &nvo, &nso);
  const int nl = skel_r > 0 ? skel_r : gd->nl;
  const size_t njobs = (size_t)A.nvol * nl + A.nsurf;
  const size_t csz = h->fp64 ? sizeof(cd) : sizeof(cf);
  *inter = njobs * gd->wy * h->G.nxh * csz;
  const size_t ntx = (gd->wx + DX_T - 1) / DX_T;
  *basis = skel_r > 0 ? ntx * dft_rows(h->G.nx / 2) * DX_T * sizeof(float) : 0;
}

void eval_set_scratch(swense_hos* h, void* base, size_t inter, size_t basis) {
  EvalWork* w = work(h);
  w->ext = reinterpret_cast<char*>(base);
  w->ext_inter = inter;
  w->ext_basis = basis;
}

void eval_set_twiddles(swense_hos* h, int gx, void* twx, int gy, void* twy) {
  EvalWork* w = work(h);
  w->ext_twx = twx;
  w->ext_twy = twy;
  w->ext_gx = gx;
  w->ext_gy = gy;
}
void ensure_device(void** p, size_t* cap, size_t bytes) { ensure(p, cap, bytes); }

CoefLayout coef_layout(swense_hos* h, unsigned cm, int nl) {
  EvArgs A;
  int idx[kNumFields];
  for (int f = 0; f < kNumFields; ++f) idx[f] = -1;
  int nvo = 0, nso = 0;
  plan_fields(h, cm, true, A, idx, &nvo, &nso);
  CoefLayout L{};
  L.fv = A.nvol;
  L.fs = A.nsurf;
  L.nl = nl;
  L.k = nl * A.nvol + A.nsurf;
  for (int f = 0; f < kNumFields; ++f) L.idx[f] = (cm & (1u << f)) ? idx[f] : -1;
  return L;
}

void eval_coef(swense_hos* h, const swense_grid_desc* gd, const double* zdev, unsigned cm, float* coef,
               const Skel* sk, int* plane) {
  eval_dispatch(h, gd, zdev, cm, true, coef, sk, plane);
}

size_t coef_floats(swense_hos* h, const swense_grid_desc* gd, unsigned cm) { return grid_floats(h, gd, cm, true); }

void eval_release(swense_hos* h) {
  if (!h->ev) return;
  if (h->ev->inter) (void)hipFree(h->ev->inter);
  if (h->ev->basis) (void)hipFree(h->ev->basis);
  if (h->ev->zdev) (void)hipFree(h->ev->zdev);
  delete h->ev;
  h->ev = nullptr;
}

extern "C" {

size_t swense_eval_grid_size(const swense_hos* h, const swense_grid_desc* gd, unsigned mask) {
  if (!h || !gd) return 0;
  return grid_floats(h, gd, mask & SWENSE_ALL_FIELDS, false);
}

int swense_eval_grid(swense_hos* h, const swense_grid_desc* gd, unsigned mask, float* out) {
  if (!h) return SWENSE_EINVAL;
  return guarded(h, [&] {
    check_grid(h, gd);
    SW_REQUIRE(out != nullptr, "null output");
    SW_REQUIRE((mask & ~(unsigned)SWENSE_ALL_FIELDS) == 0 && mask != 0, "bad field mask");
    EvalWork* w = work(h);
    void* zp = w->zdev;
    ensure(&zp, &w->zcap, (size_t)gd->nl * sizeof(double));
    w->zdev = reinterpret_cast<double*>(zp);
    SW_HIP(hipMemcpyAsync(w->zdev, gd->z, (size_t)gd->nl * sizeof(double), hipMemcpyHostToDevice, h->st));
    eval_dispatch(h, gd, w->zdev, mask, false, out);
    return SWENSE_OK;
  });
}

}  // extern "C"
