// Interpolation of the incident fields to CFD cell centres (Sec. 3.2.2) and
// the divergence of the interpolant (Sec. 3.2.3), gfx950.
//
// Scheme: periodic cubic spline horizontally (uniform cubic B-spline on a
// coefficient grid whose modes were divided by the B-spline symbol
// (4 + 2 cos(k dx))/6 per axis, so that the spline interpolates the node
// values), 4-point Lagrange vertically on the arbitrary layer heights.
//
// Binding (once per static mesh, host FP64): every point gets its horizontal
// stencil (first node, fractional offset) and its vertical stencil (first
// layer, 4 weights and their z-derivatives).  Points sharing one exact (x, y)
// - the columns of structured and extruded CFD meshes - are grouped, and the
// columns are ordered by stencil node so neighbouring columns share cache
// lines.
//
// Gather (every call), two forms chosen at binding:
// * shared columns: one 64-lane wavefront per column contracts the 16
//   horizontal taps once for every (layer, field) the column's points need -
//   the coefficient grid is node-major, so each tap is one contiguous vector
//   load across the wavefront - keeps the column profile in LDS, then each
//   point takes 4 vertical taps per field;
// * no shared columns (unstructured and jittered meshes, random clouds): the
//   points are binned by a tile of stencil start nodes and a band of first
//   layers; a workgroup stages its tile's coefficient block (tile + 3-node
//   halo, band + 3 layers, every field) in LDS once, then one thread per
//   point takes its 4 x 4 x 4 taps per field from LDS.  The tile shape is the
//   one with the fewest staged bytes for the cloud's own point density.
// Pressure is formed at the point from phi_t, u, v, w:
// p = -rho (phi_t + |u|^2/2) - rho g z.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "internal.h"
#include "wfft.h"

namespace {

struct Col {
  int start, count;  // range in the sorted point arrays
  int ix, iy;        // first stencil node, window-local
  float tx, ty;      // fractional offsets
  int lmin, nlc;     // first layer and number of layers the column needs (0: all out of range)
};

struct PtDev {
  int* perm;   // caller index of sorted point i
  int* l0;     // first stencil layer (-1: out of range)
  float* wz;   // [4][n] Lagrange weights
  float* dwz;  // [4][n] d/dz of the weights
  float* pz;   // rho g z
};

constexpr int kColsPerBlock = 4;

// Work item of the tiled gather: the points [start, start + count) of the
// sorted arrays whose stencil starts lie in the tile at (ix0, iy0) and whose
// first layers lie in the band starting at layer lb (lb < 0: points outside
// the grid or the layers, written as NaN); nlb layers are staged.
struct TileItem {
  int start, count;
  int ix0, iy0;
  int lb, nlb;
};
constexpr int kTileThreads = 256;
constexpr int kTileMaxPts = 1024;  // points per item (larger bins are split)

struct TileDev {
  const TileItem* items;
  const unsigned* hxy;  // per sorted point: stencil start ix | iy << 16 (window-local)
  const float2* txy;    // per sorted point: fractional offsets
  int nitems;
  int sx, sy;           // staged nodes per axis (tile + 3)
  int stride;           // LDS floats per staged node
};

struct GatherArgs {
  const float* coef;  // coefficient c of window node nd at nd ns + c ps
  long long ns, ps;
  int K, fv, fs, nl;
  int wx, wy, gx, gy, three;
  int nout;
  int vol[11];  // output slot -> volume field index (-1: none)
  int srf[11];  // output slot -> surface field index (-1: none)
  int zero[11]; // output slot is identically zero (v, v_t in 2D)
  int p_slot;
  int vslot[8];   // volume field of the coefficient grid -> output slot (-1: none)
  int sslot[2];   // surface field -> output slot (-1: none)
  unsigned zmask; // output slots that are identically zero
  int c_phit, c_u, c_v, c_w;
  float rho;
  float* out;
  long long n;
  int kmax;  // LDS floats per column
};

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
__device__ __forceinline__ int wrapn(int i, int w, int g) { return (w == g && i >= g) ? i - g : i; }

// Node offsets (in floats) of the 4 x 4 (or 4 x 1) horizontal stencil.
__device__ __forceinline__ void stencil(const Col& c, const GatherArgs& A, long long* off) {
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int yy = A.three ? wrapn(c.iy + b, A.wy, A.gy) : 0;
      const int xx = wrapn(c.ix + a, A.wx, A.gx);
      off[b * 4 + a] = ((long long)yy * A.wx + xx) * A.ns;
    }
}

__global__ void __launch_bounds__(256) k_gather_col(GatherArgs A, const Col* __restrict__ cols, int ncols, PtDev pd) {
  extern __shared__ float hbuf[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // neighbouring columns share coefficient nodes: consecutive column groups
  // go to the workgroups of one XCD, so its L2 serves the shared nodes
  const int ci = xcd_tile(blockIdx.x, gridDim.x) * kColsPerBlock + wave;
  float* h = hbuf + wave * A.kmax;
  Col c{};
  const bool valid = ci < ncols;
  if (valid) c = cols[ci];
  const int nv = c.nlc * A.fv;
  if (valid && c.nlc > 0) {
    float wx[4], wy[4] = {1.f, 0.f, 0.f, 0.f};
    bsw(c.tx, wx);
    if (A.three) bsw(c.ty, wy);
    long long off[16];
    stencil(c, A, off);
    const int nb = A.three ? 4 : 1;
    for (int j = lane; j < nv + A.fs; j += 64) {
      // column profile h[(l - lmin) fv + f] (the node record's layers lmin..
      // contiguous), then the surface fields
      const int jj = j < nv ? c.lmin * A.fv + j : A.nl * A.fv + (j - nv);
      // all 16 taps read before any is used (in 2D the rows b >= 1 repeat
      // row 0's nodes and are not summed)
      float tap[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) tap[t] = A.coef[off[t] + jj * A.ps];
      float acc = 0.f;
#pragma unroll
      for (int b = 0; b < 4; ++b) {  // unrolled so the weights stay in registers
        if (b < nb) {
          float r = 0.f;
#pragma unroll
          for (int a = 0; a < 4; ++a) r += wx[a] * tap[b * 4 + a];
          acc += wy[b] * r;
        }
      }
      h[j] = acc;
    }
  }
  __syncthreads();
  if (!valid) return;
  const size_t n = (size_t)A.n;
  for (int i = lane; i < c.count; i += 64) {
    const int sp = c.start + i;
    // every per-point value is read before any is used
    const int orig = pd.perm[sp];
    const int l0 = c.nlc > 0 ? pd.l0[sp] : -1;
    float wz[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) wz[a] = pd.wz[(size_t)a * n + sp];
    const float pz = A.p_slot >= 0 ? pd.pz[sp] : 0.f;
    if (l0 < 0) {
      for (int o = 0; o < A.nout; ++o) A.out[(size_t)o * n + orig] = __builtin_nanf("");
      continue;
    }
    const int base = l0 - c.lmin;
    auto vol = [&](int f) {
      const float* hf = h + base * A.fv + f;
      return wz[0] * hf[0] + wz[1] * hf[A.fv] + wz[2] * hf[2 * A.fv] + wz[3] * hf[3 * A.fv];
    };
    // unrolled over the output slots, so their field indices are read once
#pragma unroll
    for (int o = 0; o < 11; ++o) {
      if (o >= A.nout) break;
      float v = 0.f;
      if (o == A.p_slot) {
        const float pt = vol(A.c_phit), u = vol(A.c_u), w = vol(A.c_w);
        const float vv = A.c_v >= 0 ? vol(A.c_v) : 0.f;
        v = -A.rho * (pt + 0.5f * (u * u + vv * vv + w * w)) - pz;
      } else if (A.vol[o] >= 0) {
        v = vol(A.vol[o]);
      } else if (A.srf[o] >= 0) {
        v = h[nv + A.srf[o]];
      }
      A.out[(size_t)o * n + orig] = v;
    }
  }
}

// Tiled gather for clouds without shared columns: one workgroup per work
// item.  Staging: the item's nodes (tile + halo) x (the band's layers of
// every field - one contiguous run of each node record - then the surface
// fields), node-major in LDS with `stride` floats per node, eight global
// loads in flight per thread.
// Points: one thread each, 4 x 4 horizontal taps (4 x 1 in 2D) of 4 layers
// per volume field, 16 (4) taps per surface field.
template <int THREE>
__global__ void __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(5))) k_gather_tile(GatherArgs A, TileDev T, PtDev pd) {
  extern __shared__ float lds[];
  const int it = xcd_tile(blockIdx.x, gridDim.x);
  if (it >= T.nitems) return;  // uniform over the workgroup
  const TileItem I = T.items[it];
  const size_t n = (size_t)A.n;
  if (I.lb < 0) {
    for (int i = threadIdx.x; i < I.count; i += kTileThreads) {
      const int orig = pd.perm[I.start + i];
      for (int o = 0; o < A.nout; ++o) A.out[(size_t)o * n + orig] = __builtin_nanf("");
    }
    return;
  }
  const int tl = I.nlb;
  const int nvr = A.fv * tl;  // the band's layers of every volume field: one run of the node record
  const int rec = nvr + A.fs;
  const int nodes = T.sx * T.sy;
  int* nidx = reinterpret_cast<int*>(lds + (size_t)nodes * T.stride);  // window node of each staged node, -1: none
  for (int nd = threadIdx.x; nd < nodes; nd += kTileThreads) {
    const int by = THREE ? nd / T.sx : 0;
    const int bx = nd - by * T.sx;
    // full-period windows wrap; nodes past a partial window are never read
    const int gxn = wrapn(I.ix0 + bx, A.wx, A.gx);
    const int gyn = THREE ? wrapn(I.iy0 + by, A.wy, A.gy) : 0;
    nidx[nd] = (gxn < A.wx && gyn < A.wy) ? gyn * A.wx + gxn : -1;
  }
  __syncthreads();
  const bool plane = A.ps != 1;
  const int vbase = I.lb * A.fv, sbase = A.nl * A.fv - nvr;
  if (plane) {
    // plane layout (a row of nodes contiguous for each field-layer): thread
    // -> (node nd, residue class rg of r modulo G), consecutive threads on
    // consecutive nodes; each thread walks its node's record with pointer
    // steps, eight loads in flight before their stores
    const int G = nodes < kTileThreads ? kTileThreads / nodes : 1;
    for (int slot = threadIdx.x; slot < G * nodes; slot += kTileThreads) {
      const int nd = slot % nodes, rg = slot / nodes;
      const int ni = nidx[nd];
      if (ni < 0) continue;
      const long long step = (long long)G * A.ps;
      const float* src = A.coef + ni + (long long)(vbase + rg) * A.ps;
      float* dst = lds + nd * T.stride + rg;
      int r = rg;
      for (; r + 7 * G < nvr; r += 8 * G) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = src[u * step];
#pragma unroll
        for (int u = 0; u < 8; ++u) dst[u * G] = v[u];
        src += 8 * step;
        dst += 8 * G;
      }
      for (; r < nvr; r += G) {
        *dst = *src;
        src += step;
        dst += G;
      }
      // the surface fields (r in [nvr, rec), at sbase + r)
      for (; r < rec; r += G) lds[nd * T.stride + r] = A.coef[ni + (long long)(sbase + r) * A.ps];
    }
  }
  if (!plane) {
    // node-major layout (a node's record contiguous): a wavefront reads one
    // record in 64-lane runs, four nodes at a time (eight loads in flight)
    constexpr int NW = kTileThreads / 64;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int nd0 = wave; nd0 < nodes; nd0 += 4 * NW) {
      long long nb[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int nd = nd0 + j * NW;
        const int ni = nd < nodes ? nidx[nd] : -1;
        nb[j] = ni >= 0 ? (long long)ni * A.ns : -1;
      }
      for (int r0 = 0; r0 < rec; r0 += 128) {
        float v[4][2];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int hh = 0; hh < 2; ++hh) {
            const int r = r0 + lane + 64 * hh;
            v[j][hh] = nb[j] >= 0 && r < rec ? A.coef[nb[j] + (r < nvr ? vbase : sbase) + r] : 0.f;
          }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int hh = 0; hh < 2; ++hh) {
            const int r = r0 + lane + 64 * hh;
            if (nb[j] >= 0 && r < rec) lds[(nd0 + j * NW) * T.stride + r] = v[j][hh];
          }
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < I.count; i += kTileThreads) {
    const int sp = I.start + i;
    // every per-point value is read before any is used
    const int orig = pd.perm[sp];
    const int l0 = pd.l0[sp];
    const unsigned hp = T.hxy[sp];
    const float2 t = T.txy[sp];
    float wz[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) wz[a] = pd.wz[(size_t)a * n + sp];
    const float pz = A.p_slot >= 0 ? pd.pz[sp] : 0.f;
    float wx[4], wy[4] = {1.f, 0.f, 0.f, 0.f};
    bsw(t.x, wx);
    if (THREE) bsw(t.y, wy);
    // the start node lies in the item's tile: local offsets in [0, tile)
    const int lx = (int)(hp & 0xffffu) - I.ix0;
    const int ly = THREE ? (int)(hp >> 16) - I.iy0 : 0;
    const float* nb = lds + (ly * T.sx + lx) * T.stride;
    const int lo = l0 - I.lb;
    const int fv = A.fv;
    auto vol = [&](int f) {
      const float* q0 = nb + lo * fv + f;
      float acc = 0.f;
#pragma unroll
      for (int b = 0; b < (THREE ? 4 : 1); ++b) {
        float rb = 0.f;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const float* q = q0 + (b * T.sx + a) * T.stride;
          rb += wx[a] * (wz[0] * q[0] + wz[1] * q[fv] + wz[2] * q[2 * fv] + wz[3] * q[3 * fv]);
        }
        acc += wy[b] * rb;
      }
      return acc;
    };
    auto srf = [&](int s) {
      const float* q0 = nb + nvr + s;
      float acc = 0.f;
#pragma unroll
      for (int b = 0; b < (THREE ? 4 : 1); ++b) {
        float rb = 0.f;
#pragma unroll
        for (int a = 0; a < 4; ++a) rb += wx[a] * q0[(b * T.sx + a) * T.stride];
        acc += wy[b] * rb;
      }
      return acc;
    };
    float pt = 0.f, u = 0.f, vv = 0.f, w = 0.f;
    auto put = [&](int f, float v) {
      const int o = A.vslot[f];
      if (o >= 0) A.out[(size_t)o * n + orig] = v;
      pt = f == A.c_phit ? v : pt;
      u = f == A.c_u ? v : u;
      vv = f == A.c_v ? v : vv;
      w = f == A.c_w ? v : w;
    };
    if (fv == 8 && (T.stride & 3) == 0) {
      // all 8 volume fields: each (node, layer) record read as two 16-byte
      // loads, the 8 fields accumulated together
      float acc[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) acc[k] = 0.f;
      auto pick = [](const float* w4, int i) { return i == 0 ? w4[0] : i == 1 ? w4[1] : i == 2 ? w4[2] : w4[3]; };
#pragma unroll 1
      for (int b = 0; b < (THREE ? 4 : 1); ++b) {
        float rb[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) rb[k] = 0.f;
#pragma unroll 1
        for (int a = 0; a < 4; ++a) {
          const float4* q = reinterpret_cast<const float4*>(nb + (b * T.sx + a) * T.stride + lo * 8);
          float rl[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) rl[k] = 0.f;
#pragma unroll
          for (int l = 0; l < 4; ++l) {
            const float4 v0 = q[2 * l], v1 = q[2 * l + 1];
            rl[0] += wz[l] * v0.x;
            rl[1] += wz[l] * v0.y;
            rl[2] += wz[l] * v0.z;
            rl[3] += wz[l] * v0.w;
            rl[4] += wz[l] * v1.x;
            rl[5] += wz[l] * v1.y;
            rl[6] += wz[l] * v1.z;
            rl[7] += wz[l] * v1.w;
          }
          const float wa = pick(wx, a);
#pragma unroll
          for (int k = 0; k < 8; ++k) rb[k] += wa * rl[k];
        }
        const float wb = pick(wy, b);
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] += wb * rb[k];
      }
#pragma unroll
      for (int f = 0; f < 8; ++f) put(f, acc[f]);
    } else {
      // one field at a time (registers: one field's 64 taps in flight); the
      // pressure's inputs are kept as they pass
#pragma unroll 1
      for (int f = 0; f < A.fv; ++f) put(f, vol(f));
    }
#pragma unroll 1
    for (int s2 = 0; s2 < A.fs; ++s2) {
      const int o = A.sslot[s2];
      if (o >= 0) A.out[(size_t)o * n + orig] = srf(s2);
    }
    if (A.p_slot >= 0) A.out[(size_t)A.p_slot * n + orig] = -A.rho * (pt + 0.5f * (u * u + vv * vv + w * w)) - pz;
    for (unsigned zm = A.zmask; zm; zm &= zm - 1) A.out[(size_t)__builtin_ctz(zm) * n + orig] = 0.f;
  }
}

// du/dx + dv/dy + dw/dz of the interpolant: per column the horizontal
// derivative contractions of u (x) and v (y) and the plain contraction of w
// per layer, then the vertical weights (and their derivatives) per point.
__global__ void __launch_bounds__(256) k_div_col(GatherArgs A, const Col* __restrict__ cols, int ncols, PtDev pd,
                                                 float inv_dx, float inv_dy, float* div) {
  extern __shared__ float hbuf[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ci = blockIdx.x * kColsPerBlock + wave;
  float* h = hbuf + wave * A.kmax;  // [3][nlc]: d/dx u + d/dy v, w
  Col c{};
  const bool valid = ci < ncols;
  if (valid) c = cols[ci];
  if (valid && c.nlc > 0) {
    float wx[4], dwx[4], wy[4] = {1.f, 0.f, 0.f, 0.f}, dwy[4] = {0.f, 0.f, 0.f, 0.f};
    bsw(c.tx, wx);
    dbsw(c.tx, dwx);
    if (A.three) {
      bsw(c.ty, wy);
      dbsw(c.ty, dwy);
    }
    long long off[16];
    stencil(c, A, off);
    const int nb = A.three ? 4 : 1;
    for (int l = lane; l < c.nlc; l += 64) {
      const int lay = c.lmin + l;
      float hdx = 0.f, hw = 0.f;
#pragma unroll
      for (int b = 0; b < 4; ++b) {  // unrolled so the weights stay in registers
        if (b >= nb) continue;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const long long o = off[b * 4 + a] + (long long)lay * A.fv * A.ps;
          hdx += wy[b] * dwx[a] * inv_dx * A.coef[o + A.c_u * A.ps];
          if (A.c_v >= 0) hdx += dwy[b] * wx[a] * inv_dy * A.coef[o + A.c_v * A.ps];
          hw += wy[b] * wx[a] * A.coef[o + A.c_w * A.ps];
        }
      }
      h[l] = hdx;
      h[c.nlc + l] = hw;
    }
  }
  __syncthreads();
  if (!valid) return;
  const size_t n = (size_t)A.n;
  for (int i = lane; i < c.count; i += 64) {
    const int sp = c.start + i;
    const int orig = pd.perm[sp];
    const int l0 = c.nlc > 0 ? pd.l0[sp] : -1;
    if (l0 < 0) {
      div[orig] = __builtin_nanf("");
      continue;
    }
    const int b = l0 - c.lmin;
    float d = 0.f;
    for (int a = 0; a < 4; ++a)
      d += pd.wz[(size_t)a * n + sp] * h[b + a] + pd.dwz[(size_t)a * n + sp] * h[c.nlc + b + a];
    div[orig] = d;
  }
}

}  // namespace

struct swense_cells {
  swense_hos* h = nullptr;
  swense_grid_desc gd{};
  std::vector<double> z;
  long long n = 0;
  unsigned long long nbad = 0;
  int ncols = 0;
  int max_nlc = 0;
  void* mem = nullptr;
  Col* cols = nullptr;
  PtDev pd{};
  double* zdev = nullptr;
  void* coef = nullptr;
  size_t coef_bytes = 0;
  Skel skel{};            // skeleton heights of the layers (R = 0: none)
  void* skel_mem = nullptr;
  // caller-owned workspace (swense_cells_bind_ws): every device buffer of
  // the handle and of its interpolation calls lives there
  bool ws_mode = false;
  unsigned ws_mask = 0;
  float* ws_coef = nullptr;
  size_t ws_coef_cap = 0;
  char* ws_eval = nullptr;
  size_t ws_inter_cap = 0, ws_basis_cap = 0;
  void* ws_twx = nullptr;
  void* ws_twy = nullptr;
  // tiled gather (clouds without shared columns): tile of stencil start
  // nodes per horizontal axis (1 in y for 2D), band of first layers
  bool tiled = false;
  bool coef_plane = false;  // layout the last evaluation wrote (plane or node-major)
  const float* coef_cur = nullptr;  // the grid the last evaluation wrote
  int tile = 0, tile_l = 0;
  int nitems = 0;
  TileItem* items = nullptr;
  unsigned* hxy = nullptr;
  float2* txy = nullptr;
};

namespace {

// Skeleton heights (host, FP64).  Rows: |k| sampled on [0, kmax] for both
// factor families C = cosh k(z+h)/cosh kh and S = sinh k(z+h)/cosh kh (deep
// water: e^{kz} for both); columns: the layers.  Picks: greedy
// column-pivoted Gram-Schmidt on the rows scaled by max(1, max_l |factor|)
// until every remaining column is reproduced to `tol`.  Coefficients: each
// layer is a weighted least-squares combination of the picks with row i
// weighted by 1 / max(1, |factor_i(z_l)|), so that the layer's own factors
// are met to `tol` of their size (floored at the mean-level size 1) - above
// the mean level the factors grow as e^{kz}, and a bound relative to the
// largest layer would leave the deeper layers with errors of that size.
// Accepted when, with the coefficients rounded to FP32, every layer's
// weighted error is within 10 tol and the weighted sum of |coefficient| x
// |pick factor| within 30: a worst case over wavenumbers of the growth of
// the picks' own FP32 rounding, whose errors are independent, so that the
// typical growth is several times smaller.  Failing layers join the picks,
// at most four more.  Returns false if no
// worthwhile reduction exists.
bool build_skeleton(const std::vector<double>& z, double kmax, double depth, double tol, std::vector<int>& sel,
                    std::vector<float>& tc, std::vector<float>& ts) {
  const int L = (int)z.size();
  const int nk = 1024;
  const bool deep = !(depth > 0);
  std::vector<double> FC((size_t)nk * L), FS((size_t)nk * L);  // raw factors, [l][i]
  for (int i = 0; i < nk; ++i) {
    const double k = kmax * i / (nk - 1);
    for (int l = 0; l < L; ++l) {
      double c, sv;
      if (deep) {
        c = sv = std::exp(k * z[l]);
      } else {
        const double a = std::exp(k * z[l]), b = std::exp(-k * (z[l] + 2 * depth)), d = 1.0 + std::exp(-2 * k * depth);
        c = (a + b) / d;
        sv = (a - b) / d;
      }
      FC[(size_t)l * nk + i] = c;
      FS[(size_t)l * nk + i] = sv;
    }
  }
  // joint residual matrix [BC; BS] of row-scaled factors, column-major, 2 nk rows
  const int m = 2 * nk;
  std::vector<double> Rm((size_t)m * L);
  for (int i = 0; i < nk; ++i) {
    double sc = 1.0, ss = 1.0;
    for (int l = 0; l < L; ++l) {
      sc = std::max(sc, std::fabs(FC[(size_t)l * nk + i]));
      ss = std::max(ss, std::fabs(FS[(size_t)l * nk + i]));
    }
    for (int l = 0; l < L; ++l) {
      Rm[(size_t)l * m + i] = FC[(size_t)l * nk + i] / sc;
      Rm[(size_t)l * m + nk + i] = FS[(size_t)l * nk + i] / ss;
    }
  }
  sel.clear();
  std::vector<char> used(L, 0);
  for (int it = 0; it < L; ++it) {
    int jb = -1;
    double best = 0.0, bmax = 0.0;
    for (int l = 0; l < L; ++l) {
      if (used[l]) continue;
      double nn = 0.0, mx = 0.0;
      for (int i = 0; i < m; ++i) {
        nn += Rm[(size_t)l * m + i] * Rm[(size_t)l * m + i];
        mx = std::max(mx, std::fabs(Rm[(size_t)l * m + i]));
      }
      if (nn > best) { best = nn; jb = l; }
      bmax = std::max(bmax, mx);
    }
    if (jb < 0 || bmax <= tol) break;
    used[jb] = 1;
    sel.push_back(jb);
    const double inv = 1.0 / std::sqrt(best);
    std::vector<double> q(m);
    for (int i = 0; i < m; ++i) q[i] = Rm[(size_t)jb * m + i] * inv;
    for (int pass = 0; pass < 2; ++pass)  // deflate twice (orthogonality at this conditioning)
      for (int l = 0; l < L; ++l) {
        double dp = 0.0;
        for (int i = 0; i < m; ++i) dp += q[i] * Rm[(size_t)l * m + i];
        for (int i = 0; i < m; ++i) Rm[(size_t)l * m + i] -= dp * q[i];
      }
  }
  if (sel.empty()) return false;
  std::sort(sel.begin(), sel.end());
  // per-layer weighted least squares (modified Gram-Schmidt, reorthogonalised);
  // returns the worst layer's badness (> 1: fails) and that layer
  auto solve = [&](const std::vector<double>& F, std::vector<float>& T, int& worst) -> double {
    const int R = (int)sel.size();
    T.assign((size_t)L * R, 0.f);
    std::vector<double> Q((size_t)nk * R), Rr((size_t)R * R), w(nk), c(R);
    double bad = 0.0;
    worst = -1;
    for (int l = 0; l < L; ++l) {
      const double* f = &F[(size_t)l * nk];
      const int self = int(std::find(sel.begin(), sel.end(), l) - sel.begin());
      if (self < R) {
        T[(size_t)l * R + self] = 1.f;
        continue;
      }
      for (int i = 0; i < nk; ++i) w[i] = 1.0 / std::max(1.0, std::fabs(f[i]));
      std::fill(Rr.begin(), Rr.end(), 0.0);
      for (int j = 0; j < R; ++j) {
        double* qj = &Q[(size_t)j * nk];
        const double* pj = &F[(size_t)sel[j] * nk];
        for (int i = 0; i < nk; ++i) qj[i] = pj[i] * w[i];
        for (int pass = 0; pass < 2; ++pass)
          for (int p = 0; p < j; ++p) {
            const double* qp = &Q[(size_t)p * nk];
            double dp = 0.0;
            for (int i = 0; i < nk; ++i) dp += qp[i] * qj[i];
            Rr[(size_t)p * R + j] += dp;
            for (int i = 0; i < nk; ++i) qj[i] -= dp * qp[i];
          }
        double nn = 0.0;
        for (int i = 0; i < nk; ++i) nn += qj[i] * qj[i];
        nn = std::sqrt(nn);
        Rr[(size_t)j * R + j] = nn;
        if (nn > 0)
          for (int i = 0; i < nk; ++i) qj[i] /= nn;
      }
      for (int j = 0; j < R; ++j) {
        double dp = 0.0;
        for (int i = 0; i < nk; ++i) dp += Q[(size_t)j * nk + i] * f[i] * w[i];
        c[j] = dp;
      }
      for (int j = R - 1; j >= 0; --j) {  // back substitution R t = Q^T b
        double v = c[j];
        for (int p = j + 1; p < R; ++p) v -= Rr[(size_t)j * R + p] * c[p];
        c[j] = Rr[(size_t)j * R + j] != 0 ? v / Rr[(size_t)j * R + j] : 0.0;
      }
      for (int j = 0; j < R; ++j) T[(size_t)l * R + j] = (float)c[j];
      double e = 0.0, g = 0.0;
      for (int i = 0; i < nk; ++i) {
        double v = 0.0, a = 0.0;
        for (int j = 0; j < R; ++j) {
          const double t = (double)T[(size_t)l * R + j], pf = F[(size_t)sel[j] * nk + i];
          v += t * pf;
          a += std::fabs(t * pf);
        }
        e = std::max(e, std::fabs(v - f[i]) * w[i]);
        g = std::max(g, a * w[i]);
      }
      const double b = std::max(e / (10 * tol), g / 30.0);
      if (b > bad) { bad = b; worst = l; }
    }
    return bad;
  };
  const size_t r0 = sel.size();
  for (;;) {
    if (4 * sel.size() > 3 * (size_t)L || sel.size() > r0 + 4) return false;
    int wc = -1, ws = -1;
    const double bc = solve(FC, tc, wc);
    const double bs = deep ? bc : solve(FS, ts, ws);
    if (deep) ts = tc;
    if (bc <= 1.0 && bs <= 1.0) return true;
    sel.push_back(bc >= bs ? wc : ws);
    std::sort(sel.begin(), sel.end());
  }
}

// LDS floats per staged node of the tiled gather: odd (the scalar reads of
// neighbouring nodes then fall in different banks), or, with all 8 volume
// fields, a multiple of 4 that is not a multiple of 8 so that each (node,
// layer) record of 8 fields is two aligned 16-byte reads.
long long tile_stride(int fv, int tl, int fs) {
  const long long rec = (long long)fv * tl + fs;
  if (fv != 8) return rec | 1;
  long long s4 = (rec + 3) & ~3ll;
  return (s4 & 7) ? s4 : s4 + 4;
}

// Tile shape of the tiled gather: the candidate (tile of stencil start
// nodes, band of first layers) with the least staged data over the cloud's
// own bins (a sample of at most ~400k points), each item charged the cache
// lines its staging reads plus a fixed 16 KB for its launch slot, so that
// sparse clouds take large tiles and dense ones small tiles with less halo.  Sized
// for the full field set (8 volume and 2 surface fields in 3D, 6 and 2 in
// 2D); one block at most 31 KB, so that five workgroups share a CU (the
// kernel is held to five wavefronts per SIMD: measured on the 20M-point hex
// cloud, 1.77 ms with three 53 KB workgroups per CU, 1.34 ms with five).
void choose_tile(swense_cells* c, const std::vector<int>& ixs, const std::vector<int>& iys,
                 const std::vector<char>& okh, const std::vector<int>& l0, bool three) {
  const int nl = c->gd.nl, wx = c->gd.wx, wy = three ? c->gd.wy : 1;
  const long long n = c->n;
  const long long step = std::max<long long>(1, n / 400000);
  const int fv = three ? 8 : 6, fs = 2;
  static const int t3[] = {4, 6, 8, 12, 16, 24, 32};
  static const int t2[] = {16, 32, 64, 128, 256, 512};
  static const int tls[] = {1, 2, 4, 8, 16, 32, 64};
  double best = -1.0;
  c->tile = three ? 8 : 64;
  c->tile_l = 8;
  std::vector<int> cnt;
  for (int ti = 0; ti < (three ? 7 : 6); ++ti) {
    const int T = three ? t3[ti] : t2[ti], TY = three ? T : 1;
    for (int TL : tls) {
      if (TL > nl - 3) continue;
      const int tl = std::min(TL + 3, nl);
      const long long stride = tile_stride(fv, tl, fs);
      const long long nodes = (long long)(T + 3) * (three ? T + 3 : 1);
      const long long lds = nodes * (stride + 1) * 4;
      if (lds > 31 * 1024) continue;
      // bytes the staging moves through the caches: each node's band is one
      // run of fv tl floats (whole 128-byte lines), its surface floats one more line
      const double staged = (double)nodes * (std::ceil((fv * tl * 4.0 + 124.0) / 128.0) + 1.0) * 128.0;
      const long long ntx = (wx + T - 1) / T, nty = (wy + TY - 1) / TY, nband = (nl - 4) / TL + 1;
      if (ntx * nty * nband > (1ll << 24)) continue;
      cnt.assign((size_t)(ntx * nty * nband), 0);
      for (long long i = 0; i < n; i += step) {
        if (!okh[i] || l0[i] < 0) continue;
        ++cnt[(size_t)(((long long)(iys[i] / TY) * ntx + ixs[i] / T) * nband + l0[i] / TL)];
      }
      double items = 0.0;
      for (int k : cnt)
        if (k) items += std::ceil((double)k * step / kTileMaxPts);
      const double cost = items * (staged + 16384.0);
      if (best < 0 || cost < best) {
        best = cost;
        c->tile = T;
        c->tile_l = TL;
      }
    }
  }
}

// Host binding in FP64: stencils, column grouping, ordering.
void bind_host(swense_cells* c, const std::vector<double>& xyz, double lx, double ly, bool three,
               std::vector<Col>& cols, std::vector<int>& perm, std::vector<int>& l0v, std::vector<float>& wzv,
               std::vector<float>& dwzv, std::vector<float>& pzv, double rho_g, std::vector<TileItem>& items,
               std::vector<unsigned>& hxy, std::vector<float2>& txy) {
  const long long n = c->n;
  const swense_grid_desc& gd = c->gd;
  const int gx = gd.gx, gy = three ? gd.gy : 1;
  const double dx = lx / gx, dy = three ? ly / gy : 1.0;
  const double* X = xyz.data();
  const double* Y = X + n;
  const double* Z = Y + n;
  const int nl = gd.nl;
  const double* zl = c->z.data();
  std::vector<int> ixs(n), iys(n);
  std::vector<float> txs(n), tys(n);
  std::vector<char> okh(n);
  l0v.assign(n, -1);
  wzv.assign(4 * n, 0.f);
  dwzv.assign(4 * n, 0.f);
  pzv.assign(n, 0.f);
  std::vector<int> l0_orig(n, -1);
  std::vector<float> w_orig(4 * n, 0.f), dw_orig(4 * n, 0.f);
  for (long long i = 0; i < n; ++i) {
    const double x = X[i], y = Y[i], z = Z[i];
    bool ok = std::isfinite(x) && std::isfinite(y) && std::isfinite(z);
    long long st = 0, sty = 0;
    double fx = 0, fy = 0, sx = 0, sy = 0;
    if (ok) {
      sx = x / dx;
      fx = std::floor(sx);
      st = (long long)fx - 1 - gd.ix0;
      if (gd.wx == gx) st = ((st % gx) + gx) % gx;
      else ok = st >= 0 && st + 3 < gd.wx;
      if (three) {
        sy = y / dy;
        fy = std::floor(sy);
        sty = (long long)fy - 1 - gd.iy0;
        if (gd.wy == gy) sty = ((sty % gy) + gy) % gy;
        else ok = ok && sty >= 0 && sty + 3 < gd.wy;
      }
    }
    okh[i] = ok;
    ixs[i] = ok ? (int)st : 0;
    iys[i] = ok ? (int)sty : 0;
    txs[i] = ok ? (float)(sx - fx) : 0.f;
    tys[i] = (ok && three) ? (float)(sy - fy) : 0.f;
    if (ok && z >= zl[0] && z <= zl[nl - 1]) {
      int l = int(std::upper_bound(zl, zl + nl, z) - zl) - 1;
      l = std::min(std::max(l, 0), nl - 2);
      int b0 = std::min(std::max(l - 1, 0), nl - 4);
      double zn[4];
      for (int a = 0; a < 4; ++a) zn[a] = zl[b0 + a];
      for (int a = 0; a < 4; ++a) {
        double wa = 1.0, dwa = 0.0;
        for (int b = 0; b < 4; ++b)
          if (b != a) wa *= (z - zn[b]) / (zn[a] - zn[b]);
        for (int cc = 0; cc < 4; ++cc) {
          if (cc == a) continue;
          double term = 1.0 / (zn[a] - zn[cc]);
          for (int b = 0; b < 4; ++b)
            if (b != a && b != cc) term *= (z - zn[b]) / (zn[a] - zn[b]);
          dwa += term;
        }
        w_orig[4 * i + a] = (float)wa;
        dw_orig[4 * i + a] = (float)dwa;
      }
      l0_orig[i] = b0;
    }
  }
  // order: by stencil node (iy, ix), then exact (x, y), then z; columns are
  // runs of identical (x, y)
  perm.resize(n);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) {
    if (okh[a] != okh[b]) return okh[a] > okh[b];
    if (!okh[a]) return false;  // out-of-range points keep their order (coordinates may be NaN)
    if (iys[a] != iys[b]) return iys[a] < iys[b];
    if (ixs[a] != ixs[b]) return ixs[a] < ixs[b];
    if (X[a] != X[b]) return X[a] < X[b];
    if (Y[a] != Y[b]) return Y[a] < Y[b];
    return Z[a] < Z[b];
  });
  long long nrun = 0;
  for (long long i = 0; i < n;) {
    const int p0 = perm[i];
    long long j = i + 1;
    while (okh[p0] && j < n && okh[perm[j]] && X[perm[j]] == X[p0] && Y[perm[j]] == Y[p0]) ++j;
    ++nrun;
    i = j;
  }
  // fewer than 4 points per exact column: the tiled gather (stencil-start
  // tiles x first-layer bands, sorted by caller index within each bin)
  c->tiled = 4 * nrun > n && gd.wx < 65536 && gd.wy < 65536;
  items.clear();
  if (c->tiled) {
    choose_tile(c, ixs, iys, okh, l0_orig, three);
    const int T = c->tile, TY = three ? c->tile : 1, TL = c->tile_l;
    const long long ntx = (gd.wx + T - 1) / T;
    const long long nband = (nl - 4) / TL + 1;
    std::vector<unsigned long long> key(n);
    for (long long i = 0; i < n; ++i) {
      if (!okh[i] || l0_orig[i] < 0) {
        key[i] = ~0ull;
        continue;
      }
      const long long tile = (long long)(iys[i] / TY) * ntx + ixs[i] / T;
      key[i] = (unsigned long long)(tile * nband + l0_orig[i] / TL);
    }
    std::sort(perm.begin(), perm.end(), [&](int a, int b) { return key[a] != key[b] ? key[a] < key[b] : a < b; });
    for (long long i = 0; i < n;) {
      const unsigned long long k0 = key[perm[i]];
      long long j = i + 1;
      while (j < n && key[perm[j]] == k0 && j - i < kTileMaxPts) ++j;
      TileItem it{};
      it.start = (int)i;
      it.count = (int)(j - i);
      if (k0 == ~0ull) {
        it.lb = -1;
      } else {
        const long long tile = (long long)(k0 / nband), band = (long long)(k0 % nband);
        it.ix0 = (int)(tile % ntx) * T;
        it.iy0 = (int)(tile / ntx) * TY;
        it.lb = (int)band * TL;
        it.nlb = std::min(TL + 3, nl - it.lb);
      }
      items.push_back(it);
      i = j;
    }
  }
  cols.clear();
  unsigned long long bad = 0;
  long long i = 0;
  while (i < n) {
    const int p0 = perm[i];
    long long j = i + 1;
    while (okh[p0] && j < n && okh[perm[j]] && X[perm[j]] == X[p0] && Y[perm[j]] == Y[p0]) ++j;
    Col col{};
    col.start = (int)i;
    col.count = (int)(j - i);
    col.ix = ixs[p0];
    col.iy = iys[p0];
    col.tx = txs[p0];
    col.ty = tys[p0];
    int lmin = nl, lmax = -1;
    for (long long k = i; k < j; ++k) {
      const int q = perm[k];
      const int l0 = okh[q] ? l0_orig[q] : -1;
      l0v[k] = l0;
      for (int a = 0; a < 4; ++a) {
        wzv[(size_t)a * n + k] = w_orig[4 * q + a];
        dwzv[(size_t)a * n + k] = dw_orig[4 * q + a];
      }
      pzv[k] = (float)(rho_g * Z[q]);
      if (l0 < 0) {
        ++bad;
        continue;
      }
      lmin = std::min(lmin, l0);
      lmax = std::max(lmax, l0);
    }
    if (lmax >= 0) {
      col.lmin = lmin;
      col.nlc = lmax - lmin + 4;
    } else {
      col.lmin = 0;
      col.nlc = 0;
    }
    cols.push_back(col);
    i = j;
  }
  if (c->tiled) {
    hxy.resize(n);
    txy.resize(n);
    for (long long k = 0; k < n; ++k) {
      const int q = perm[k];
      hxy[k] = (unsigned)ixs[q] | ((unsigned)iys[q] << 16);
      txy[k] = make_float2(txs[q], tys[q]);
    }
  }
  c->nbad = bad;
}

void gather_args(swense_hos* h, swense_cells* c, unsigned mask, const CoefLayout& L, float* out, GatherArgs& A) {
  std::memset(&A, 0, sizeof(A));
  const bool three = h->G.ny > 1;
  A.coef = c->coef_cur;
  A.ns = c->coef_plane ? 1 : L.k;
  A.ps = c->coef_plane ? (long long)c->gd.wx * (three ? c->gd.wy : 1) : 1;
  A.K = L.k;
  A.fv = L.fv;
  A.fs = L.fs;
  A.nl = L.nl;
  A.wx = c->gd.wx;
  A.wy = three ? c->gd.wy : 1;
  A.gx = c->gd.gx;
  A.gy = three ? c->gd.gy : 1;
  A.three = three ? 1 : 0;
  A.p_slot = -1;
  A.c_phit = L.idx[5];
  A.c_u = L.idx[1];
  A.c_v = three ? L.idx[2] : -1;
  A.c_w = L.idx[3];
  int o = 0;
  for (int f = 0; f < 11; ++f) {
    if (!(mask & (1u << f))) continue;
    A.vol[o] = -1;
    A.srf[o] = -1;
    if (f == 4) A.p_slot = o;
    else if (f == 9 || f == 10) A.srf[o] = L.idx[f];
    else A.vol[o] = L.idx[f];
    ++o;
  }
  A.nout = o;
  for (int f = 0; f < 8; ++f) A.vslot[f] = -1;
  A.sslot[0] = A.sslot[1] = -1;
  A.zmask = 0;
  for (int q = 0; q < o; ++q) {
    if (q == A.p_slot) continue;
    if (A.vol[q] >= 0) A.vslot[A.vol[q]] = q;
    else if (A.srf[q] >= 0) A.sslot[A.srf[q]] = q;
    else A.zmask |= 1u << q;
  }
  A.rho = (float)h->G.rho;
  A.out = out;
  A.n = c->n;
  A.kmax = std::max(c->max_nlc * L.fv + L.fs, 3 * c->max_nlc);
}

// Coefficient grid of the current modes for the fields cm: into the cells'
// own buffer (grown on demand), or into coef_ext when given.
void refresh(swense_hos* h, swense_cells* c, unsigned cm, CoefLayout* L, float* coef_ext = nullptr) {
  *L = coef_layout(h, cm, c->gd.nl);
  float* coef = coef_ext;
  if (!coef) {
    const size_t nfl = std::max<size_t>(coef_floats(h, &c->gd, cm), 1);
    void* before = c->coef;
    ensure_device(&c->coef, &c->coef_bytes, nfl * sizeof(float));
    if (c->coef != before) ++h->scratch_epoch;
    coef = reinterpret_cast<float*>(c->coef);
  }
  int plane = 0;
  eval_coef(h, &c->gd, c->zdev, cm, coef, c->skel.R > 0 ? &c->skel : nullptr, &plane);
  c->coef_plane = plane != 0;
  c->coef_cur = coef;
}

unsigned coef_mask(unsigned mask, bool three) {
  unsigned m = mask & ~(unsigned)SWENSE_P;
  if (mask & SWENSE_P) m |= SWENSE_PHI_T | SWENSE_U | SWENSE_W | (three ? SWENSE_V : 0u);
  return m;
}

}  // namespace

// Finite-volume divergence on a structured box mesh from the normal
// velocity at the face centres (Sec. 3.2.3): per cell, the outflow through
// its six (2D: four) faces over its volume, i.e. the differences of the face
// velocities over the cell widths.  Face values f: rows of the interpolation
// output (U, [V,] W) at the face-centre points ordered x faces
// [nz][ny][nx+1], then y faces [nz][ny+1][nx] (3D), then z faces [nz+1][ny][nx].
__global__ void k_fv_div(const float* __restrict__ f, long long nf, int three, int nx, int ny, int nz,
                         const double* __restrict__ xe, const double* __restrict__ ye, const double* __restrict__ ze,
                         float* __restrict__ div, double* __restrict__ sums) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long ncell = (long long)nx * ny * nz;
  double d2 = 0.0, dm = 0.0;
  if (c < ncell) {
    const int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / ((long long)nx * ny));
    const long long nxf = (long long)nz * ny * (nx + 1);
    const long long nyf = three ? (long long)nz * (ny + 1) * nx : 0;
    const float* fu = f;                        // U row
    const float* fv = three ? f + nf : nullptr; // V row
    const float* fw = f + (three ? 2 : 1) * nf; // W row
    const long long ux = ((long long)k * ny + j) * (nx + 1) + i;
    double v = ((double)fu[ux + 1] - (double)fu[ux]) / (xe[i + 1] - xe[i]);
    if (three) {
      const long long uy = nxf + ((long long)k * (ny + 1) + j) * nx + i;
      v += ((double)fv[uy + nx] - (double)fv[uy]) / (ye[j + 1] - ye[j]);
    }
    const long long uz = nxf + nyf + ((long long)k * ny + j) * nx + i;
    v += ((double)fw[uz + (long long)ny * nx] - (double)fw[uz]) / (ze[k + 1] - ze[k]);
    div[c] = (float)v;
    d2 = v * v;
    dm = fabs(v);
  }
  __shared__ double r2[256], rm[256];
  r2[threadIdx.x] = d2;
  rm[threadIdx.x] = dm;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      r2[threadIdx.x] += r2[threadIdx.x + w];
      rm[threadIdx.x] = fmax(rm[threadIdx.x], rm[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&sums[0], r2[0]);
    // non-negative doubles order like their bit patterns
    atomicMax(reinterpret_cast<unsigned long long*>(&sums[1]), (unsigned long long)__double_as_longlong(rm[0]));
  }
}

__global__ void k_zero2(double* s) {
  s[0] = 0.0;
  s[1] = 0.0;
}

// Grid evaluation + gather of the current modes into out (on h->st).
// Scratch of a cells handle bound on a caller's workspace: the coefficient
// grid, the evaluation rows, the DFT basis and the grid's twiddle tables
// come from it for the duration of the evaluation (restored on exit).
struct WsScope {
  swense_hos* h;
  bool on;
  WsScope(swense_hos* hh, swense_cells* c, bool use_tw) : h(hh), on(c->ws_mode) {
    if (!on) return;
    eval_set_scratch(h, c->ws_eval, c->ws_inter_cap, c->ws_basis_cap);
    if (use_tw) eval_set_twiddles(h, c->gd.gx, c->ws_twx, c->gd.gy, c->ws_twy);
  }
  ~WsScope() {
    if (!on) return;
    eval_set_scratch(h, nullptr, 0, 0);
    eval_set_twiddles(h, 0, nullptr, 0, nullptr);
  }
};

void interp_body(swense_hos* h, swense_cells* c, unsigned mask, float* out, float* coef_ext = nullptr) {
  if (c->n == 0) return;
  CoefLayout L;
  const unsigned cm0 = coef_mask(mask, h->G.ny > 1);
  WsScope scope(h, c, true);
  if (c->ws_mode && !coef_ext) {
    if (coef_floats(h, &c->gd, cm0) * sizeof(float) > c->ws_coef_cap)
      throw SwenseError{SWENSE_ENOMEM, "field mask needs a larger coefficient grid than the cells' workspace holds"};
    coef_ext = c->ws_coef;
  }
  refresh(h, c, cm0, &L, coef_ext);
  GatherArgs A;
  gather_args(h, c, mask, L, out, A);
  if (h->prof.on) {
    // compulsory: every point's stencil data read once, its outputs written
    // once, the coefficient grid read once; model: 12 B of coordinates + 4 B of
    // index + 4 B per output field per point, plus the grid
    const double grid = (double)L.k * c->gd.wx * (h->G.ny > 1 ? c->gd.wy : 1) * 4.0;
    const double per = 4.0 + 4.0 + 16.0 + (A.p_slot >= 0 ? 4.0 : 0.0) + (c->tiled ? 12.0 : 0.0);
    h->prof.bytes[SWENSE_K_INTERP] += (double)c->n * (per + 4.0 * A.nout) + grid;
    h->prof.tbytes[SWENSE_K_INTERP] += (double)c->n * (16.0 + 4.0 * A.nout) + grid;
  }
  if (c->tiled) {
    const bool three = h->G.ny > 1;
    TileDev T{c->items, c->hxy, c->txy, c->nitems, c->tile + 3, three ? c->tile + 3 : 1, 0};
    T.stride = (int)tile_stride(L.fv, std::min(c->tile_l + 3, L.nl), L.fs);
    const size_t lds = (size_t)T.sx * T.sy * (T.stride + 1) * sizeof(float);
    SW_REQUIRE(lds <= 64 * 1024, "tile block too large for LDS");
    if (three)
      SW_LAUNCH(h, SWENSE_K_INTERP, k_gather_tile<1>, dim3((unsigned)c->nitems), dim3(kTileThreads), lds, h->st, A,
                T, c->pd);
    else
      SW_LAUNCH(h, SWENSE_K_INTERP, k_gather_tile<0>, dim3((unsigned)c->nitems), dim3(kTileThreads), lds, h->st, A,
                T, c->pd);
    return;
  }
  const size_t lds = (size_t)kColsPerBlock * A.kmax * sizeof(float);
  SW_REQUIRE(lds <= 160 * 1024, "column profile too long for LDS");
  if (lds > 65536)
    SW_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gather_col),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  const unsigned nblk = (unsigned)((c->ncols + kColsPerBlock - 1) / kColsPerBlock);
  SW_LAUNCH(h, SWENSE_K_INTERP, k_gather_col, dim3(nblk), dim3(64 * kColsPerBlock), lds, h->st, A, c->cols,
            c->ncols, c->pd);
}

// Device scratch of the allocation-free interpolation: one array per GPU the
// library runs on, resident until the process ends.  Host code never passes
// the array's name to a kernel: its address on each device is looked up
// once, with that device current, and kept.
constexpr size_t kNoAllocScratchBytes = 128ull << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // device -> address of `scratch` on it

// caller must have made `dev` current
void* noalloc_scratch(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  void* ptr = nullptr;
  SW_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  SW_REQUIRE(ptr != nullptr, "no device address for the scratch array");
  g_scratch_ptr[dev] = ptr;
  return ptr;
}

}  // namespace

void noalloc_scratch_setup(int dev) { (void)noalloc_scratch(dev); }

namespace {
// makes `dev` current for a scope and restores the previous device
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    SW_HIP(hipGetDevice(&prev));
    if (prev != dev) SW_HIP(hipSetDevice(dev));
  }
  ~DeviceGuard() {
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
  }
};
}  // namespace

namespace {
// Byte offsets of a cells workspace (all 256-aligned), upper bounds that
// need no binning: per point its stencil records (and, tiled, its tile
// position), one column and one tile item per point at most, skeleton
// coefficients for every layer, the coefficient grid of `mask`, the
// evaluation rows without skeleton heights, the DFT basis, two twiddle tables.
struct WsPlan {
  size_t points = 0, points_bytes = 0, skel = 0, skel_bytes = 0, coef = 0, coef_bytes = 0, eval = 0,
         inter_bytes = 0, basis_bytes = 0, twx = 0, twy = 0, total = 0;
};

WsPlan cells_ws_plan(swense_hos* h, const swense_grid_desc* gd, long long n, unsigned mask) {
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  const bool three = h->G.ny > 1;
  const size_t nn = (size_t)std::max<long long>(n, 1), L = gd->nl;
  WsPlan w;
  size_t o = 0;
  w.points = o;
  w.points_bytes = up(L * sizeof(double)) + up(nn * sizeof(Col)) + 2 * up(nn * 4) + 2 * up(nn * 16) + up(nn * 4) +
                   up(nn * sizeof(TileItem)) + up(nn * 4) + up(nn * 8);
  o += w.points_bytes;
  w.skel = o;
  w.skel_bytes = up(L * sizeof(double)) + 2 * up(L * L * sizeof(float));
  o += w.skel_bytes;
  const unsigned cm = coef_mask(mask, three);
  w.coef = o;
  w.coef_bytes = up(std::max<size_t>(coef_floats(h, gd, cm), 1) * sizeof(float));
  o += w.coef_bytes;
  size_t inter = 0, basis = 0;
  eval_scratch_need(h, gd, cm, 0, &inter, &basis);
  size_t inter_s = 0, basis_s = 0;
  eval_scratch_need(h, gd, cm, 1, &inter_s, &basis_s);  // a skeleton's basis (any R)
  w.eval = o;
  w.inter_bytes = up(inter);
  w.basis_bytes = up(basis_s);
  o += w.inter_bytes + w.basis_bytes;
  w.twx = o;
  o += TwiddleCache::table_bytes(gd->gx, h->fp64);
  w.twy = o;
  o += three ? TwiddleCache::table_bytes(gd->gy, h->fp64) : 0;
  w.total = o;
  return w;
}

int cells_bind_impl(swense_hos* h, const swense_grid_desc* gd, long long n, const double* xyz, unsigned ws_mask,
                    char* ws, size_t ws_bytes, swense_cells** out);
}  // namespace

extern "C" {

int swense_cells_bind(swense_hos* h, const swense_grid_desc* gd, long long n, const double* xyz,
                      swense_cells** out) {
  return cells_bind_impl(h, gd, n, xyz, 0u, nullptr, 0, out);
}

int swense_cells_workspace_bytes(swense_hos* h, const swense_grid_desc* gd, long long n, unsigned mask,
                                 size_t* bytes) {
  if (!h || !bytes) return SWENSE_EINVAL;
  *bytes = 0;
  return guarded(h, [&] {
    check_grid_desc(h, gd);
    SW_REQUIRE(n >= 0 && n < (1ll << 31), "point count must be in [0, 2^31)");
    SW_REQUIRE((mask & ~(unsigned)SWENSE_ALL_FIELDS) == 0 && mask != 0, "bad field mask");
    *bytes = cells_ws_plan(h, gd, n, mask).total;
    return (int)SWENSE_OK;
  });
}

int swense_cells_bind_ws(swense_hos* h, const swense_grid_desc* gd, long long n, const double* xyz, unsigned mask,
                         void* ws, size_t ws_bytes, swense_cells** out) {
  if (!h || !out || !ws || (reinterpret_cast<uintptr_t>(ws) & 255)) return SWENSE_EINVAL;
  if ((mask & ~(unsigned)SWENSE_ALL_FIELDS) != 0 || mask == 0) return SWENSE_EINVAL;
  return cells_bind_impl(h, gd, n, xyz, mask, reinterpret_cast<char*>(ws), ws_bytes, out);
}

}  // extern "C"

namespace {
int cells_bind_impl(swense_hos* h, const swense_grid_desc* gd, long long n, const double* xyz, unsigned ws_mask,
                    char* ws, size_t ws_bytes, swense_cells** out) {
  if (!h || !out) return SWENSE_EINVAL;
  *out = nullptr;
  swense_cells* c = nullptr;
  int rc = guarded(h, [&] {
    if (ws) {
      check_grid_desc(h, gd);
      SW_REQUIRE(n >= 0 && n < (1ll << 31), "point count must be in [0, 2^31)");
      if (ws_bytes < cells_ws_plan(h, gd, n, ws_mask).total)
        throw SwenseError{SWENSE_ENOMEM, "cells workspace smaller than swense_cells_workspace_bytes"};
    }
    check_grid_desc(h, gd);
    SW_REQUIRE(n >= 0 && n < (1ll << 31), "point count must be in [0, 2^31)");
    SW_REQUIRE(n == 0 || xyz != nullptr, "null coordinates");
    SW_REQUIRE(gd->nl >= 4, "interpolation needs at least 4 layers");
    // a stencil of 4 nodes wraps at most once round a full period
    SW_REQUIRE(gd->gx >= 4 && (h->G.ny == 1 || gd->gy >= 4), "interpolation needs at least 4 nodes per period");
    // the grid's twiddle tables now, so that interpolation calls allocate
    // nothing for them (in the caller's workspace when there is one)
    const WsPlan wp = ws ? cells_ws_plan(h, gd, n, ws_mask) : WsPlan{};
    c = new swense_cells();
    if (ws) {
      c->ws_mode = true;
      c->ws_mask = ws_mask;
      c->ws_coef = reinterpret_cast<float*>(ws + wp.coef);
      c->ws_coef_cap = wp.coef_bytes;
      c->ws_eval = ws + wp.eval;
      c->ws_inter_cap = wp.inter_bytes;
      c->ws_basis_cap = wp.basis_bytes;
      TwiddleCache::fill(gd->gx, h->fp64, ws + wp.twx);
      c->ws_twx = ws + wp.twx;
      if (h->G.ny > 1) {
        TwiddleCache::fill(gd->gy, h->fp64, ws + wp.twy);
        c->ws_twy = ws + wp.twy;
      }
    } else {
      h->tw.get(gd->gx, h->fp64);
      if (h->G.ny > 1) h->tw.get(gd->gy, h->fp64);
    }
    c->h = h;
    c->gd = *gd;
    c->z.assign(gd->z, gd->z + gd->nl);
    c->gd.z = c->z.data();
    c->n = n;
    std::vector<double> hx((size_t)3 * n);
    if (n > 0) {
      SW_HIP(hipMemcpyAsync(hx.data(), xyz, hx.size() * sizeof(double), hipMemcpyDeviceToHost, h->st));
      SW_HIP(hipStreamSynchronize(h->st));
    }
    std::vector<Col> cols;
    std::vector<int> perm, l0v;
    std::vector<float> wz, dwz, pz;
    std::vector<TileItem> items;
    std::vector<unsigned> hxy;
    std::vector<float2> txy;
    const bool three = h->G.ny > 1;
    bind_host(c, hx, h->G.lx, h->G.ly, three, cols, perm, l0v, wz, dwz, pz, h->G.rho * h->G.g, items, hxy, txy);
    c->ncols = (int)cols.size();
    c->nitems = (int)items.size();
    for (const Col& col : cols) c->max_nlc = std::max(c->max_nlc, col.nlc);
    const size_t nn = (size_t)std::max<long long>(n, 1);
    const size_t nc = std::max<size_t>(cols.size(), 1);
    const size_t nt = c->tiled ? nn : 0, ni = c->tiled ? std::max<size_t>(items.size(), 1) : 0;
    const size_t sizes[] = {gd->nl * sizeof(double), nc * sizeof(Col), nn * 4, nn * 4, nn * 16, nn * 16, nn * 4,
                            ni * sizeof(TileItem), nt * 4, nt * 8};
    size_t bytes = 0;
    for (size_t b : sizes) bytes += (b + 255) & ~size_t(255);
    char* p;
    if (ws) {
      SW_REQUIRE(bytes <= wp.points_bytes, "internal: point records exceed their workspace bound");
      p = ws + wp.points;
    } else {
      SW_HIP(hipMalloc(&c->mem, bytes));
      p = reinterpret_cast<char*>(c->mem);
    }
    char* const p0 = p;
    auto take = [&](size_t b) {
      void* r = p;
      p += (b + 255) & ~size_t(255);
      return r;
    };
    c->zdev = reinterpret_cast<double*>(take(sizes[0]));
    c->cols = reinterpret_cast<Col*>(take(sizes[1]));
    c->pd.perm = reinterpret_cast<int*>(take(sizes[2]));
    c->pd.l0 = reinterpret_cast<int*>(take(sizes[3]));
    c->pd.wz = reinterpret_cast<float*>(take(sizes[4]));
    c->pd.dwz = reinterpret_cast<float*>(take(sizes[5]));
    c->pd.pz = reinterpret_cast<float*>(take(sizes[6]));
    c->items = reinterpret_cast<TileItem*>(take(sizes[7]));
    c->hxy = reinterpret_cast<unsigned*>(take(sizes[8]));
    c->txy = reinterpret_cast<float2*>(take(sizes[9]));
    SW_REQUIRE(p <= p0 + bytes, "internal carve overflow");
    SW_HIP(hipMemcpy(c->zdev, gd->z, gd->nl * sizeof(double), hipMemcpyHostToDevice));
    if (n > 0) {
      SW_HIP(hipMemcpy(c->cols, cols.data(), cols.size() * sizeof(Col), hipMemcpyHostToDevice));
      SW_HIP(hipMemcpy(c->pd.perm, perm.data(), n * 4, hipMemcpyHostToDevice));
      SW_HIP(hipMemcpy(c->pd.l0, l0v.data(), n * 4, hipMemcpyHostToDevice));
      SW_HIP(hipMemcpy(c->pd.wz, wz.data(), n * 16, hipMemcpyHostToDevice));
      SW_HIP(hipMemcpy(c->pd.dwz, dwz.data(), n * 16, hipMemcpyHostToDevice));
      SW_HIP(hipMemcpy(c->pd.pz, pz.data(), n * 4, hipMemcpyHostToDevice));
      if (c->tiled) {
        SW_HIP(hipMemcpy(c->items, items.data(), items.size() * sizeof(TileItem), hipMemcpyHostToDevice));
        SW_HIP(hipMemcpy(c->hxy, hxy.data(), n * 4, hipMemcpyHostToDevice));
        SW_HIP(hipMemcpy(c->txy, txy.data(), n * 8, hipMemcpyHostToDevice));
      }
    }
    // skeleton heights for the coefficient grids: factors reproduced to 1e-7
    // of each wavenumber's scale, below the FP32 rounding of the transforms
    {
      const double kx = M_PI * h->G.nx / h->G.lx, ky = three ? M_PI * h->G.ny / h->G.ly : 0.0;
      std::vector<int> sel;
      std::vector<float> tc, ts;
      if (gd->nl >= 8 && build_skeleton(c->z, std::sqrt(kx * kx + ky * ky), h->G.depth, 1e-7, sel, tc, ts)) {
        const int R = (int)sel.size(), L = gd->nl;
        std::vector<double> zeta(R);
        for (int j = 0; j < R; ++j) zeta[j] = c->z[sel[j]];
        const size_t b0 = ((R * sizeof(double)) + 255) & ~size_t(255);
        const size_t b1 = ((size_t)L * R * sizeof(float) + 255) & ~size_t(255);
        char* q;
        if (ws) {
          SW_REQUIRE(b0 + 2 * b1 <= wp.skel_bytes, "internal: skeleton exceeds its workspace bound");
          q = ws + wp.skel;
        } else {
          SW_HIP(hipMalloc(&c->skel_mem, b0 + 2 * b1));
          q = reinterpret_cast<char*>(c->skel_mem);
        }
        SW_HIP(hipMemcpy(q, zeta.data(), R * sizeof(double), hipMemcpyHostToDevice));
        SW_HIP(hipMemcpy(q + b0, tc.data(), (size_t)L * R * sizeof(float), hipMemcpyHostToDevice));
        SW_HIP(hipMemcpy(q + b0 + b1, ts.data(), (size_t)L * R * sizeof(float), hipMemcpyHostToDevice));
        c->skel = Skel{R, reinterpret_cast<const double*>(q), reinterpret_cast<const float*>(q + b0),
                       reinterpret_cast<const float*>(q + b0 + b1)};
      }
    }
    *out = c;
    return SWENSE_OK;
  });
  if (rc != SWENSE_OK && c) swense_cells_destroy(c);
  return rc;
}
}  // namespace

extern "C" {

int swense_interp_cells(swense_hos* h, swense_cells* c, unsigned mask, float* out, long long* n_out_of_range) {
  if (!h || !c || c->h != h) return SWENSE_EINVAL;
  return guarded(h, [&] {
    SW_REQUIRE(out != nullptr || c->n == 0, "null output");
    SW_REQUIRE((mask & ~(unsigned)SWENSE_ALL_FIELDS) == 0 && mask != 0, "bad field mask");
    interp_body(h, c, mask, out);
    if (n_out_of_range) {
      *n_out_of_range = (long long)c->nbad;
      if (c->nbad) return (int)SWENSE_ERANGE;
    }
    return (int)SWENSE_OK;
  });
}

int swense_interp_step(swense_hos* h, swense_cells* c, unsigned mask, float* out, int nsteps) {
  if (!h || !c || c->h != h || nsteps < 0) return SWENSE_EINVAL;
  return guarded(h, [&] {
    SW_REQUIRE(out != nullptr || c->n == 0, "null output");
    SW_REQUIRE((mask & ~(unsigned)SWENSE_ALL_FIELDS) == 0 && mask != 0, "bad field mask");
    if (!h->aux) {
      SW_HIP(hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking));
      SW_HIP(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
      SW_HIP(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
    }
    if (!h->eta_snap) SW_HIP(hipMalloc(&h->eta_snap, h->nc * sizeof(cd)));
    // modes (and right-hand side) of the current state, and a copy of eta that
    // the evaluation reads while the step rewrites the state (a set
    // evaluation time does not apply: this call maps the current state)
    h->herm_on = false;
    launch_modes(h);
    SW_HIP(hipMemcpyAsync(h->eta_snap, h->xn[0], h->nc * sizeof(cd), hipMemcpyDeviceToDevice, h->st));
    SW_HIP(hipEventRecord(h->ev_fork, h->st));
    SW_HIP(hipStreamWaitEvent(h->aux, h->ev_fork, 0));
    hipStream_t main = h->st;
    h->st = h->aux;
    h->eta_src = h->eta_snap;
    try {
      interp_body(h, c, mask, out);
    } catch (...) {
      h->st = main;
      h->eta_src = nullptr;
      throw;
    }
    h->st = main;
    h->eta_src = nullptr;
    SW_HIP(hipEventRecord(h->ev_join, h->aux));
    hos_step(h, nsteps);
    SW_HIP(hipStreamWaitEvent(h->st, h->ev_join, 0));
    return (int)SWENSE_OK;
  });
}

int swense_fv_divergence(swense_hos* h, const swense_grid_desc* gd, const double* xe, int nx, const double* ye,
                         int ny, const double* ze, int nz, float* div, double* rms, double* maxabs) {
  if (!h || !gd || !xe || !ze || !div) return SWENSE_EINVAL;
  swense_cells* c = nullptr;
  void* mem = nullptr;
  const int rc = guarded(h, [&] {
    const bool three = h->G.ny > 1;
    SW_REQUIRE(nx >= 1 && nz >= 1 && (three ? (ny >= 1 && ye != nullptr) : ny == 1), "mesh sizes");
    for (int i = 0; i < nx; ++i) SW_REQUIRE(xe[i + 1] > xe[i], "x edges must increase");
    for (int k = 0; k < nz; ++k) SW_REQUIRE(ze[k + 1] > ze[k], "z edges must increase");
    if (three)
      for (int j = 0; j < ny; ++j) SW_REQUIRE(ye[j + 1] > ye[j], "y edges must increase");
    const long long nxf = (long long)nz * ny * (nx + 1), nyf = three ? (long long)nz * (ny + 1) * nx : 0;
    const long long nzf = (long long)(nz + 1) * ny * nx, nf = nxf + nyf + nzf;
    SW_REQUIRE(nf < (1ll << 31), "too many faces");
    // face centres [3][nf]
    std::vector<double> xyz((size_t)3 * nf);
    auto put = [&](long long idx, double x, double y, double z) {
      xyz[idx] = x;
      xyz[nf + idx] = y;
      xyz[2 * nf + idx] = z;
    };
    std::vector<double> yedge(three ? ye : nullptr, three ? ye + ny + 1 : nullptr);
    if (!three) yedge = {0.0, 0.0};
    long long o = 0;
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i <= nx; ++i)
          put(o++, xe[i], 0.5 * (yedge[j] + yedge[j + 1]), 0.5 * (ze[k] + ze[k + 1]));
    if (three)
      for (int k = 0; k < nz; ++k)
        for (int j = 0; j <= ny; ++j)
          for (int i = 0; i < nx; ++i)
            put(o++, 0.5 * (xe[i] + xe[i + 1]), ye[j], 0.5 * (ze[k] + ze[k + 1]));
    for (int k = 0; k <= nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
          put(o++, 0.5 * (xe[i] + xe[i + 1]), 0.5 * (yedge[j] + yedge[j + 1]), ze[k]);
    const int nfields = three ? 3 : 2;
    const size_t b_xyz = xyz.size() * sizeof(double), b_out = (size_t)nfields * nf * sizeof(float);
    const size_t b_e = (size_t)(nx + 1 + (three ? ny + 1 : 0) + nz + 1) * sizeof(double);
    SW_HIP(hipMalloc(&mem, b_xyz + b_out + b_e + 2 * sizeof(double) + 1024));
    char* p = reinterpret_cast<char*>(mem);
    auto take = [&](size_t b) {
      void* r = p;
      p += (b + 255) & ~size_t(255);
      return r;
    };
    double* dxyz = reinterpret_cast<double*>(take(b_xyz));
    float* fout = reinterpret_cast<float*>(take(b_out));
    double* de = reinterpret_cast<double*>(take(b_e));
    double* sums = reinterpret_cast<double*>(take(2 * sizeof(double)));
    SW_HIP(hipMemcpyAsync(dxyz, xyz.data(), b_xyz, hipMemcpyHostToDevice, h->st));
    std::vector<double> edges(xe, xe + nx + 1);
    if (three) edges.insert(edges.end(), ye, ye + ny + 1);
    edges.insert(edges.end(), ze, ze + nz + 1);
    SW_HIP(hipMemcpyAsync(de, edges.data(), b_e, hipMemcpyHostToDevice, h->st));
    int brc = swense_cells_bind(h, gd, nf, dxyz, &c);
    if (brc != SWENSE_OK) throw SwenseError{brc, "binding the face centres: " + h->err};
    const unsigned mask = SWENSE_U | SWENSE_W | (three ? SWENSE_V : 0u);
    SW_REQUIRE(c->nbad == 0, "face centres outside the grid window or layers");
    interp_body(h, c, mask, fout);
    hipLaunchKernelGGL(k_zero2, dim3(1), dim3(1), 0, h->st, sums);
    const long long ncell = (long long)nx * ny * nz;
    hipLaunchKernelGGL(k_fv_div, dim3((unsigned)((ncell + 255) / 256)), dim3(256), 0, h->st, fout, nf, three ? 1 : 0,
                       nx, ny, nz, de, three ? de + nx + 1 : de, de + nx + 1 + (three ? ny + 1 : 0), div, sums);
    SW_HIP(hipGetLastError());
    double hs[2];
    SW_HIP(hipMemcpyAsync(hs, sums, sizeof(hs), hipMemcpyDeviceToHost, h->st));
    SW_HIP(hipStreamSynchronize(h->st));
    if (rms) *rms = std::sqrt(hs[0] / (double)ncell);
    if (maxabs) *maxabs = hs[1];
    return (int)SWENSE_OK;
  });
  if (c) swense_cells_destroy(c);
  if (mem) {
    (void)hipStreamSynchronize(h->st);
    (void)hipFree(mem);
  }
  return rc;
}

int swense_interp_divergence(swense_hos* h, swense_cells* c, float* div) {
  if (!h || !c || c->h != h) return SWENSE_EINVAL;
  return guarded(h, [&] {
    SW_REQUIRE(div != nullptr || c->n == 0, "null output");
    if (c->n == 0) return (int)SWENSE_OK;
    const bool three = h->G.ny > 1;
    const unsigned m = SWENSE_U | SWENSE_W | (three ? SWENSE_V : 0u);
    CoefLayout L;
    WsScope scope(h, c, true);
    float* cx = nullptr;
    if (c->ws_mode) {
      if (coef_floats(h, &c->gd, m) * sizeof(float) > c->ws_coef_cap)
        throw SwenseError{SWENSE_ENOMEM, "the divergence needs a larger coefficient grid than the cells' workspace holds"};
      cx = c->ws_coef;
    }
    refresh(h, c, m, &L, cx);
    GatherArgs A;
    gather_args(h, c, m, L, nullptr, A);
    const float inv_dx = (float)(c->gd.gx / h->G.lx);
    const float inv_dy = three ? (float)(c->gd.gy / h->G.ly) : 0.f;
    const size_t lds = (size_t)kColsPerBlock * A.kmax * sizeof(float);
    SW_REQUIRE(lds <= 160 * 1024, "column profile too long for LDS");
    if (lds > 65536)
      SW_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_div_col),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const unsigned nblk = (unsigned)((c->ncols + kColsPerBlock - 1) / kColsPerBlock);
    SW_LAUNCH(h, SWENSE_K_INTERP_DIV, k_div_col, dim3(nblk), dim3(64 * kColsPerBlock), lds, h->st, A, c->cols,
              c->ncols, c->pd, inv_dx, inv_dy, div);
    return (int)SWENSE_OK;
  });
}

int swense_interp_cells_noalloc(swense_hos* h, swense_cells* c, unsigned mask, float* out,
                                long long* n_out_of_range) {
  if (!h || !c || c->h != h) return SWENSE_EINVAL;
  return guarded(h, [&] {
    SW_REQUIRE(out != nullptr || c->n == 0, "null output");
    SW_REQUIRE((mask & ~(unsigned)SWENSE_ALL_FIELDS) == 0 && mask != 0, "bad field mask");
    const bool three = h->G.ny > 1;
    SW_REQUIRE(h->tw.has(c->gd.gx, h->fp64) && (!three || h->tw.has(c->gd.gy, h->fp64)),
               "twiddle tables missing (the cells were not bound on this handle)");
    const unsigned cm = coef_mask(mask, three);
    size_t inter = 0, basis = 0;
    eval_scratch_need(h, &c->gd, cm, c->skel.R, &inter, &basis);
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t cbytes = up(std::max<size_t>(coef_floats(h, &c->gd, cm), 1) * sizeof(float));
    const size_t need = cbytes + up(inter) + up(basis);
    if (need > kNoAllocScratchBytes)
      throw SwenseError{SWENSE_ENOMEM, "interpolation needs " + std::to_string(need) +
                                           " bytes of scratch; the allocation-free entry point holds " +
                                           std::to_string(kNoAllocScratchBytes)};
    DeviceGuard dg(h->device);
    char* base = reinterpret_cast<char*>(noalloc_scratch(h->device));
    eval_set_scratch(h, base + cbytes, up(inter), up(basis));
    try {
      interp_body(h, c, mask, out, reinterpret_cast<float*>(base));
    } catch (...) {
      eval_set_scratch(h, nullptr, 0, 0);
      throw;
    }
    eval_set_scratch(h, nullptr, 0, 0);
    if (n_out_of_range) {
      *n_out_of_range = (long long)c->nbad;
      if (c->nbad) return (int)SWENSE_ERANGE;
    }
    return (int)SWENSE_OK;
  });
}

void swense_cells_destroy(swense_cells* c) {
  if (!c) return;
  if (c->mem) (void)hipFree(c->mem);      // null when bound on a caller's workspace
  if (c->coef) (void)hipFree(c->coef);
  if (c->skel_mem) (void)hipFree(c->skel_mem);
  delete c;
}

}  // extern "C"
