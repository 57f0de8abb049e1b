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
};

// y-inverse for evaluation: job = (field, layer) for volume fields, then
// one job per surface field.
template <typename R>
__global__ void __launch_bounds__(256) k_yinv_eval(EvArgs A, Geom G, FftPlan plan, int TW) {
  extern __shared__ unsigned char smem[];
  const int job = blockIdx.y;
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
  jb.dst = reinterpret_cast<cpx<R>*>(A.inter) + (size_t)job * A.wy * G.nxh;
  jb.sym = SYM_EVAL;
  jb.ev.vf = A.f[fi].vf;
  jb.ev.mult = A.f[fi].mult;
  jb.ev.pre = A.pre;
  jb.ev.gx = A.gx;
  jb.ev.gy = A.gy;
  yinv_body<R>(jb, G, plan, TW, A.wy, A.iy0, smem);
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

__global__ void k_fill(float* p, size_t n, float v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------- binding
struct CellsDev {
  int* ix;    // first stencil node, window-local (x)
  int* iy;    // (y)
  float* tx;  // fractional position in [0,1)
  float* ty;
  int* l0;    // first stencil layer, -1: out of range
  float* wz;  // [4][n] Lagrange weights
  float* dwz; // [4][n] their z-derivatives
  float* pz;  // rho g z
};

__global__ void k_bind(const double* xyz, long long n, CellsDev c, const double* zl, int nl, double dx, double dy,
                       int gx, int gy, int ix0, int iy0, int wx, int wy, int three, double rho_g,
                       unsigned long long* nbad) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = xyz[i], y = xyz[n + i], z = xyz[2 * n + i];
  bool ok = isfinite(x) && isfinite(y) && isfinite(z);
  const double sx = x / dx;
  const double fx = floor(sx);
  long long st = (long long)fx - 1 - ix0;
  if (wx == gx) st = ((st % gx) + gx) % gx;
  else ok = ok && st >= 0 && st + 3 < wx;
  long long sty = 0;
  double ty = 0.0;
  if (three) {
    const double sy = y / dy;
    const double fy = floor(sy);
    sty = (long long)fy - 1 - iy0;
    if (wy == gy) sty = ((sty % gy) + gy) % gy;
    else ok = ok && sty >= 0 && sty + 3 < wy;
    ty = sy - fy;
  }
  ok = ok && z >= zl[0] && z <= zl[nl - 1];
  int l0 = -1;
  double w[4] = {0, 0, 0, 0}, dw[4] = {0, 0, 0, 0};
  if (ok) {
    int lo = 0, hi = nl - 1;  // last layer index with zl <= z, clamped to nl-2
    while (hi - lo > 1) {
      int mid = (lo + hi) >> 1;
      if (zl[mid] <= z) lo = mid;
      else hi = mid;
    }
    int l = lo;
    l0 = l - 1;
    if (l0 < 0) l0 = 0;
    if (l0 > nl - 4) l0 = nl - 4;
    double zn[4];
    for (int a = 0; a < 4; ++a) zn[a] = zl[l0 + a];
    for (int a = 0; a < 4; ++a) {
      double wa = 1.0, dwa = 0.0;
      for (int b = 0; b < 4; ++b) {
        if (b == a) continue;
        wa *= (z - zn[b]) / (zn[a] - zn[b]);
      }
      for (int cc = 0; cc < 4; ++cc) {
        if (cc == a) continue;
        double term = 1.0 / (zn[a] - zn[cc]);
        for (int b = 0; b < 4; ++b) {
          if (b == a || b == cc) continue;
          term *= (z - zn[b]) / (zn[a] - zn[b]);
        }
        dwa += term;
      }
      w[a] = wa;
      dw[a] = dwa;
    }
  } else {
    atomicAdd(nbad, 1ull);
  }
  c.ix[i] = (int)st;
  c.iy[i] = (int)sty;
  c.tx[i] = (float)(sx - fx);
  c.ty[i] = (float)ty;
  c.l0[i] = l0;
  for (int a = 0; a < 4; ++a) {
    c.wz[(size_t)a * n + i] = (float)w[a];
    c.dwz[(size_t)a * n + i] = (float)dw[a];
  }
  c.pz[i] = (float)(rho_g * z);
}

__device__ __forceinline__ void bsw(float t, float* w) {
  const float t2 = t * t, t3 = t2 * t, u = 1.0f - t;
  w[0] = u * u * u * (1.0f / 6.0f);
  w[1] = (3.0f * t3 - 6.0f * t2 + 4.0f) * (1.0f / 6.0f);
  w[2] = (-3.0f * t3 + 3.0f * t2 + 3.0f * t + 1.0f) * (1.0f / 6.0f);
  w[3] = t3 * (1.0f / 6.0f);
}
__device__ __forceinline__ void dbsw(float t, float* w) {
  const float t2 = t * t, u = 1.0f - t;
  w[0] = -0.5f * u * u;
  w[1] = 1.5f * t2 - 2.0f * t;
  w[2] = -1.5f * t2 + t + 0.5f;
  w[3] = 0.5f * t2;
}

struct InterpArgs {
  const float* coef;  // volume coefficient grids [nvc][nl][wy][wx], then surface [nsc][wy][wx]
  int nvc, nsc, nl, wx, wy, gx, gy, three;
  int vol_src[kNumFields];  // output slot -> coefficient field (volume), -1 none
  int srf_src[kNumFields];  // output slot -> coefficient field (surface), -1 none
  int p_slot;
  int c_phit, c_u, c_v, c_w;  // coefficient fields used by the pressure (-1 none)
  int nout;
  float rho;
  float* out;
  long long n;
};

__device__ __forceinline__ int wrapi(int i, int w, int g) {
  if (w == g) {
    if (i >= g) i -= g;
  }
  return i;
}

__global__ void __launch_bounds__(256) k_interp(InterpArgs A, CellsDev c) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  const int l0 = c.l0[i];
  const size_t n = (size_t)A.n;
  if (l0 < 0) {
    for (int o = 0; o < A.nout; ++o) A.out[(size_t)o * n + i] = __builtin_nanf("");
    return;
  }
  float wx[4], wy[4] = {1.f, 0.f, 0.f, 0.f}, wz[4];
  bsw(c.tx[i], wx);
  if (A.three) bsw(c.ty[i], wy);
  for (int a = 0; a < 4; ++a) wz[a] = c.wz[(size_t)a * n + i];
  int xs[4], ys[4];
  const int ix = c.ix[i], iy = c.iy[i];
  for (int a = 0; a < 4; ++a) {
    xs[a] = wrapi(ix + a, A.wx, A.gx);
    ys[a] = A.three ? wrapi(iy + a, A.wy, A.gy) : 0;
  }
  const int nyt = A.three ? 4 : 1;
  const size_t plane = (size_t)A.wy * A.wx;
  auto vol = [&](int f) {
    const float* base = A.coef + (size_t)f * A.nl * plane;
    float acc = 0.f;
    for (int cc = 0; cc < 4; ++cc) {
      const float* lay = base + (size_t)(l0 + cc) * plane;
      float h = 0.f;
      for (int b = 0; b < nyt; ++b) {
        const float* row = lay + (size_t)ys[b] * A.wx;
        h += wy[b] * (wx[0] * row[xs[0]] + wx[1] * row[xs[1]] + wx[2] * row[xs[2]] + wx[3] * row[xs[3]]);
      }
      acc += wz[cc] * h;
    }
    return acc;
  };
  auto srf = [&](int f) {
    const float* base = A.coef + (size_t)A.nvc * A.nl * plane + (size_t)f * plane;
    float h = 0.f;
    for (int b = 0; b < nyt; ++b) {
      const float* row = base + (size_t)ys[b] * A.wx;
      h += wy[b] * (wx[0] * row[xs[0]] + wx[1] * row[xs[1]] + wx[2] * row[xs[2]] + wx[3] * row[xs[3]]);
    }
    return h;
  };
  for (int o = 0; o < A.nout; ++o) {
    float v = 0.f;
    if (o == A.p_slot) {
      const float pt = vol(A.c_phit), u = vol(A.c_u), w = vol(A.c_w);
      const float vv = A.c_v >= 0 ? vol(A.c_v) : 0.f;
      v = -A.rho * (pt + 0.5f * (u * u + vv * vv + w * w)) - c.pz[i];
    } else if (A.vol_src[o] >= 0) {
      v = vol(A.vol_src[o]);
    } else if (A.srf_src[o] >= 0) {
      v = srf(A.srf_src[o]);
    }
    A.out[(size_t)o * n + i] = v;
  }
}

__global__ void __launch_bounds__(256) k_interp_div(InterpArgs A, CellsDev c, double dx, double dy, float* div) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  const int l0 = c.l0[i];
  const size_t n = (size_t)A.n;
  if (l0 < 0) {
    div[i] = __builtin_nanf("");
    return;
  }
  float wx[4], dwx[4], wy[4] = {1.f, 0.f, 0.f, 0.f}, dwy[4] = {0.f, 0.f, 0.f, 0.f}, wz[4], dwz[4];
  bsw(c.tx[i], wx);
  dbsw(c.tx[i], dwx);
  if (A.three) {
    bsw(c.ty[i], wy);
    dbsw(c.ty[i], dwy);
  }
  for (int a = 0; a < 4; ++a) {
    wz[a] = c.wz[(size_t)a * n + i];
    dwz[a] = c.dwz[(size_t)a * n + i];
    dwx[a] *= (float)(1.0 / dx);
    dwy[a] *= (float)(1.0 / dy);
  }
  int xs[4], ys[4];
  for (int a = 0; a < 4; ++a) {
    xs[a] = wrapi(c.ix[i] + a, A.wx, A.gx);
    ys[a] = A.three ? wrapi(c.iy[i] + a, A.wy, A.gy) : 0;
  }
  const int nyt = A.three ? 4 : 1;
  const size_t plane = (size_t)A.wy * A.wx;
  float d = 0.f;
  for (int cc = 0; cc < 4; ++cc) {
    for (int b = 0; b < nyt; ++b) {
      for (int a = 0; a < 4; ++a) {
        const size_t off = (size_t)(l0 + cc) * plane + (size_t)ys[b] * A.wx + xs[a];
        d += wz[cc] * wy[b] * dwx[a] * A.coef[(size_t)A.c_u * A.nl * plane + off];
        if (A.c_v >= 0) d += wz[cc] * dwy[b] * wx[a] * A.coef[(size_t)A.c_v * A.nl * plane + off];
        d += dwz[cc] * wy[b] * wx[a] * A.coef[(size_t)A.c_w * A.nl * plane + off];
      }
    }
  }
  div[i] = d;
}

}  // namespace

// ---------------------------------------------------------------- host side
struct EvalWork {
  void* inter = nullptr;
  size_t inter_bytes = 0;
  double* zdev = nullptr;
  size_t zcap = 0;
};

struct swense_cells {
  swense_hos* h = nullptr;
  swense_grid_desc gd{};
  std::vector<double> z;
  long long n = 0;
  unsigned long long nbad = 0;
  void* mem = nullptr;
  CellsDev dev{};
  double* zdev = nullptr;
  float* coef = nullptr;
  size_t coef_bytes = 0;
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
  e.src = t ? h->atmod : h->amod;
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
    e.src = f == F_ETA ? h->xn[0] : h->kk[0];
    e.vf = 2;
    e.mult = 0;
    e.out_slot = srf_slot_of[f];
    if (out_of_field) out_of_field[f] = ns;
    ++ns;
  }
  A.nsurf = ns;
}

template <typename R>
void eval_t(swense_hos* h, const swense_grid_desc* gd, const double* zdev, unsigned mask, bool pre, float* out) {
  launch_modes(h);
  EvArgs A;
  int nvo = 0, nso = 0;
  plan_fields(h, mask, pre, A, nullptr, &nvo, &nso);
  A.z = zdev;
  A.nl = gd->nl;
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
  if (h->G.ny == 1) {
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
  ensure(&w->inter, &w->inter_bytes, (size_t)njobs * A.wy * h->G.nxh * csz);
  A.inter = w->inter;
  TwiddleCache& tc = h->tw;
  FftPlan py = tc.get(A.gy, sizeof(R) == 8);
  FftPlan px = tc.get(A.gx, sizeof(R) == 8);
  // y pass; jobs may exceed the grid's y limit -> chunk
  {
    int TW = 1;
    long cap = 65536 / (2L * py.n * (long)csz);
    while (TW * 2 <= cap && TW * 2 <= 256) TW *= 2;
    const size_t lds = 2ull * TW * py.n * csz;
    dim3 grid((h->G.nxh + TW - 1) / TW, njobs);
    SW_REQUIRE(njobs <= 65535, "too many (field, layer) pairs");
    SW_LAUNCH(h, SWENSE_K_YINV_EVAL, k_yinv_eval<R>, grid, dim3(256), lds, h->st, A, h->G, py, TW);
    SW_HIP(hipGetLastError());
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
                   float* out) {
  if (h->fp64) eval_t<double>(h, gd, zdev, mask, pre, out);
  else eval_t<float>(h, gd, zdev, mask, pre, out);
}

size_t grid_floats(const swense_hos* h, const swense_grid_desc* gd, unsigned mask, bool pre) {
  size_t nv = 0, ns = 0;
  for (int f = 0; f < kNumFields; ++f) {
    if (!(mask & (1u << f))) continue;
    if (f == F_ETA || f == F_ETAT) ++ns;
    else if (!(pre && f == F_P)) ++nv;
  }
  const size_t plane = (size_t)gd->wx * gd->wy;
  return nv * gd->nl * plane + ns * plane;
}

// coefficient fields an interpolation of `mask` needs (volume fields incl.
// the inputs of the pressure; surface fields)
unsigned coef_mask(unsigned mask, bool three) {
  unsigned m = mask & ~(unsigned)SWENSE_P;
  if (mask & SWENSE_P) m |= SWENSE_PHI_T | SWENSE_U | SWENSE_W | (three ? SWENSE_V : 0u);
  return m;
}

void interp_args(swense_hos* h, swense_cells* c, unsigned mask, float* out, InterpArgs& A) {
  std::memset(&A, 0, sizeof(A));
  const bool three = h->G.ny > 1;
  const unsigned cm = coef_mask(mask, three);
  // coefficient field index of each bit in the coefficient grid layout
  int cidx[kNumFields];
  int nv = 0, ns = 0;
  for (int f = 0; f < kNumFields; ++f) {
    cidx[f] = -1;
    if (!(cm & (1u << f))) continue;
    if (f == F_ETA || f == F_ETAT) cidx[f] = ns++;
    else cidx[f] = nv++;
  }
  A.coef = c->coef;
  A.nvc = nv;
  A.nsc = ns;
  A.nl = c->gd.nl;
  A.wx = c->gd.wx;
  A.wy = c->gd.wy;
  A.gx = c->gd.gx;
  A.gy = three ? c->gd.gy : 1;
  A.three = three ? 1 : 0;
  A.p_slot = -1;
  A.c_phit = cidx[F_PHIT];
  A.c_u = cidx[F_U];
  A.c_v = three ? cidx[F_V] : -1;
  A.c_w = cidx[F_W];
  int o = 0;
  for (int f = 0; f < kNumFields; ++f) {
    if (!(mask & (1u << f))) continue;
    A.vol_src[o] = -1;
    A.srf_src[o] = -1;
    if (f == F_P) A.p_slot = o;
    else if (f == F_ETA || f == F_ETAT) A.srf_src[o] = cidx[f];
    else A.vol_src[o] = cidx[f];
    ++o;
  }
  A.nout = o;
  A.rho = (float)h->G.rho;
  A.out = out;
  A.n = c->n;
}

void refresh_coef(swense_hos* h, swense_cells* c, unsigned cm) {
  const size_t nfl = grid_floats(h, &c->gd, cm, true);
  ensure(reinterpret_cast<void**>(&c->coef), &c->coef_bytes, std::max<size_t>(nfl, 1) * sizeof(float));
  eval_dispatch(h, &c->gd, c->zdev, cm, true, c->coef);
}

}  // namespace

void eval_release(swense_hos* h) {
  if (!h->ev) return;
  if (h->ev->inter) (void)hipFree(h->ev->inter);
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

int swense_cells_bind(swense_hos* h, const swense_grid_desc* gd, long long n, const double* xyz,
                      swense_cells** out) {
  if (!h || !out) return SWENSE_EINVAL;
  *out = nullptr;
  swense_cells* c = nullptr;
  int rc = guarded(h, [&] {
    check_grid(h, gd);
    SW_REQUIRE(n >= 0, "negative point count");
    SW_REQUIRE(n == 0 || xyz != nullptr, "null coordinates");
    SW_REQUIRE(gd->nl >= 4, "interpolation needs at least 4 layers");
    c = new swense_cells();
    c->h = h;
    c->gd = *gd;
    c->z.assign(gd->z, gd->z + gd->nl);
    c->gd.z = c->z.data();
    c->n = n;
    const size_t nn = (size_t)std::max<long long>(n, 1);
    // carve: counter, layer heights, then the per-point arrays (each 256-B aligned)
    const size_t sizes[] = {sizeof(unsigned long long), gd->nl * sizeof(double), nn * 4, nn * 4, nn * 4, nn * 4,
                            nn * 4, nn * 16, nn * 16, nn * 4};
    size_t bytes = 0;
    for (size_t b : sizes) bytes += (b + 255) & ~size_t(255);
    SW_HIP(hipMalloc(&c->mem, bytes));
    char* p = reinterpret_cast<char*>(c->mem);
    int k = 0;
    auto take = [&](size_t b) {
      SW_REQUIRE(b == sizes[k], "internal carve mismatch");
      ++k;
      void* r = p;
      p += (b + 255) & ~size_t(255);
      return r;
    };
    unsigned long long* dbad = reinterpret_cast<unsigned long long*>(take(sizeof(unsigned long long)));
    c->zdev = reinterpret_cast<double*>(take(gd->nl * sizeof(double)));
    c->dev.ix = reinterpret_cast<int*>(take(nn * 4));
    c->dev.iy = reinterpret_cast<int*>(take(nn * 4));
    c->dev.tx = reinterpret_cast<float*>(take(nn * 4));
    c->dev.ty = reinterpret_cast<float*>(take(nn * 4));
    c->dev.l0 = reinterpret_cast<int*>(take(nn * 4));
    c->dev.wz = reinterpret_cast<float*>(take(nn * 16));
    c->dev.dwz = reinterpret_cast<float*>(take(nn * 16));
    c->dev.pz = reinterpret_cast<float*>(take(nn * 4));
    SW_REQUIRE(k == (int)(sizeof(sizes) / sizeof(sizes[0])) && p <= reinterpret_cast<char*>(c->mem) + bytes,
               "internal carve overflow");
    SW_HIP(hipMemcpyAsync(c->zdev, gd->z, gd->nl * sizeof(double), hipMemcpyHostToDevice, h->st));
    SW_HIP(hipMemsetAsync(dbad, 0, sizeof(unsigned long long), h->st));
    if (n > 0) {
      const double dx = h->G.lx / gd->gx;
      const double dy = h->G.ny > 1 ? h->G.ly / gd->gy : 1.0;
      SW_LAUNCH(h, SWENSE_K_BIND, k_bind, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->st, xyz, n, c->dev, c->zdev,
                         gd->nl, dx, dy, gd->gx, h->G.ny > 1 ? gd->gy : 1, gd->ix0, gd->iy0, gd->wx, gd->wy,
                         h->G.ny > 1 ? 1 : 0, h->G.rho * h->G.g, dbad);
      SW_HIP(hipGetLastError());
    }
    SW_HIP(hipMemcpyAsync(&c->nbad, dbad, sizeof(unsigned long long), hipMemcpyDeviceToHost, h->st));
    SW_HIP(hipStreamSynchronize(h->st));
    *out = c;
    return SWENSE_OK;
  });
  if (rc != SWENSE_OK && c) swense_cells_destroy(c);
  return rc;
}

int swense_interp_cells(swense_hos* h, swense_cells* c, unsigned mask, float* out, long long* n_out_of_range) {
  if (!h || !c || c->h != h) return SWENSE_EINVAL;
  return guarded(h, [&] {
    SW_REQUIRE(out != nullptr || c->n == 0, "null output");
    SW_REQUIRE((mask & ~(unsigned)SWENSE_ALL_FIELDS) == 0 && mask != 0, "bad field mask");
    if (c->n > 0) {
      const unsigned cm = coef_mask(mask, h->G.ny > 1);
      refresh_coef(h, c, cm);
      InterpArgs A;
      interp_args(h, c, mask, out, A);
      SW_LAUNCH(h, SWENSE_K_INTERP, k_interp, dim3((unsigned)((c->n + 255) / 256)), dim3(256), 0, h->st, A, c->dev);
      SW_HIP(hipGetLastError());
    }
    if (n_out_of_range) {
      *n_out_of_range = (long long)c->nbad;
      if (c->nbad) return (int)SWENSE_ERANGE;
    }
    return (int)SWENSE_OK;
  });
}

int swense_interp_divergence(swense_hos* h, swense_cells* c, float* div) {
  if (!h || !c || c->h != h) return SWENSE_EINVAL;
  return guarded(h, [&] {
    SW_REQUIRE(div != nullptr || c->n == 0, "null output");
    if (c->n == 0) return (int)SWENSE_OK;
    const bool three = h->G.ny > 1;
    const unsigned m = SWENSE_U | SWENSE_W | (three ? SWENSE_V : 0u);
    refresh_coef(h, c, m);
    InterpArgs A;
    interp_args(h, c, m, nullptr, A);
    const double dx = h->G.lx / c->gd.gx;
    const double dy = three ? h->G.ly / c->gd.gy : 1.0;
    SW_LAUNCH(h, SWENSE_K_INTERP_DIV, k_interp_div, dim3((unsigned)((c->n + 255) / 256)), dim3(256), 0, h->st, A, c->dev, dx, dy,
                       div);
    SW_HIP(hipGetLastError());
    return (int)SWENSE_OK;
  });
}

void swense_cells_destroy(swense_cells* c) {
  if (!c) return;
  if (c->mem) (void)hipFree(c->mem);
  if (c->coef) (void)hipFree(c->coef);
  delete c;
}

}  // extern "C"
