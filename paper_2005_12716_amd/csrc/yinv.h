// Inverse transform along y of symbol-weighted half spectra (shared by the
// HOS step and the grid evaluation).
#pragma once

#include "internal.h"
#include "wfft.h"

__device__ __forceinline__ cd symbol_of(const Geom& G, const YInvJob& jb, int p, int qs) {
  const double kx = 2.0 * M_PI * (double)p / G.lx;
  const double ky = G.ny > 1 ? 2.0 * M_PI * (double)qs / G.ly : 0.0;
  const double k = sqrt(kx * kx + ky * ky);
  switch (jb.sym) {
    case SYM_ONE: return mk(1.0, 0.0);
    case SYM_IKX: return mk(0.0, kx);
    case SYM_IKY: return mk(0.0, ky);
    case SYM_DZ: {
      double s = 1.0;
      for (int i = 0; i < jb.jpow; ++i) s *= k;
      if ((jb.jpow & 1) && G.depth > 0.0) s *= tanh(k * G.depth);
      return mk(s, 0.0);
    }
    default: {
      double C = 1.0, S = 1.0;
      if (jb.ev.vf != 2) vfactors(k, jb.z, G.depth, C, S);
      const double f = jb.ev.vf == 0 ? C : (jb.ev.vf == 1 ? S : 1.0);
      cd m;
      switch (jb.ev.mult) {
        case 0: m = mk(f, 0.0); break;
        case 1: m = mk(0.0, kx * f); break;
        case 2: m = mk(0.0, ky * f); break;
        default: m = mk(k * f, 0.0); break;
      }
      if (jb.ev.pre) {
        double bx = (4.0 + 2.0 * cos(2.0 * M_PI * (double)p / (double)jb.ev.gx)) / 6.0;
        double by = G.ny > 1 ? (4.0 + 2.0 * cos(2.0 * M_PI * (double)qs / (double)jb.ev.gy)) / 6.0 : 1.0;
        m = cscale(m, 1.0 / (bx * by));
      }
      return m;
    }
  }
}

// Evaluation symbol in single precision, for FP32 transforms: the factors of
// symbol_of's evaluation branch (vertical factor, multiplier, prefilter) in
// float arithmetic.  Per column: kx, the x prefilter factor bx and the scale
// kys = 2 pi / ly of ky.
__device__ __forceinline__ cpx<float> symbol_eval_f32(const Geom& G, const YInvJob& jb, float kx, float bx, float kys,
                                                      int qs) {
  const float ky = G.ny > 1 ? kys * (float)qs : 0.f;
  const float k = sqrtf(kx * kx + ky * ky);
  float C = 1.f, S = 1.f;
  if (jb.ev.vf != 2) {
    const float z = (float)jb.z;
    if (!(G.depth > 0.0)) {
      C = S = expf(k * z);
    } else {
      const float h = (float)G.depth;
      const float a = expf(k * z), b = expf(-k * (z + 2.f * h)), d = 1.f + expf(-2.f * k * h);
      C = (a + b) / d;
      S = (a - b) / d;
    }
  }
  const float f = jb.ev.vf == 0 ? C : (jb.ev.vf == 1 ? S : 1.f);
  cpx<float> m;
  switch (jb.ev.mult) {
    case 0: m = mk(f, 0.f); break;
    case 1: m = mk(0.f, kx * f); break;
    case 2: m = mk(0.f, ky * f); break;
    default: m = mk(k * f, 0.f); break;
  }
  if (jb.ev.pre) {
    const float by = G.ny > 1 ? (4.f + 2.f * cospif(2.f * (float)qs / (float)jb.ev.gy)) / 6.f : 1.f;
    const float s = 1.f / (bx * by);
    m = mk(m.x * s, m.y * s);
  }
  return m;
}

// y-inverse: grid (ceil(nxh / TW), njobs).  Slot s of the length-Ly
// sequence gathers every kept mode q whose signed index is = s (mod Ly):
// zero-padding when Ly >= ny, alias-folding when Ly < ny.  Rows
// (row0 + r) mod Ly, r < nrows, are stored.
// Value of slot s of column p: the sum over kept modes q with signed index
// = s (mod Ly) of spectrum x symbol (zero-padding or alias-folding in y).
__device__ __forceinline__ cd yinv_slot(const YInvJob& jb, const Geom& G, int Ly, int p, int s) {
  double ax = 0.0, ay = 0.0;
  if (p < G.nxh && 2 * p != G.nx) {
    if (G.ny == 1) {
      if (s == 0) {
        cd v = cmul(jb.src[p], symbol_of(G, jb, p, 0));
        ax = v.x;
        ay = v.y;
      }
    } else {
      const int half = G.ny / 2;
      for (int qs = s - ((s + half - 1) / Ly) * Ly; qs <= half - 1; qs += Ly) {
        const int q = qs >= 0 ? qs : qs + G.ny;
        cd v = cmul(jb.src[(size_t)q * G.nxh + p], symbol_of(G, jb, p, qs));
        ax += v.x;
        ay += v.y;
      }
    }
  }
  return mk(ax, ay);
}

// Wavefront version: the calling wavefront transforms column p in its LDS
// buffer (wbuf_len(Ly) complex, skewed index) and stores rows
// (row0 + r) mod Ly, r < nrows.
template <typename R, int MAXE, int NS0>
__device__ __forceinline__ void yinv_wave(const YInvJob& jb, const Geom& G, const WPlan& plan, int nrows, int row0,
                                          int p, cpx<R>* buf, int lane) {
  const int Ly = plan.n;
  bool filled = false;
  if constexpr (NS0 > 0) {
    // Zero-padding in y (Ly >= ny): each kept mode q has a slot of its own,
    // so the wavefront walks the modes instead of the slots, issuing a batch
    // of column loads before the symbols are formed; slots no mode maps to
    // are cleared.  Same values as the slot walk below.
    if (G.ny > 1 && Ly >= G.ny) {
      constexpr int E = NS0 / 64, B = E < 4 ? E : 4;
      const int half = G.ny / 2;
      const bool col = p < G.nxh && 2 * p != G.nx;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int s = lane + 64 * j;
        if (!col || (s >= half && s <= Ly - half)) buf[sk(s)] = mk((R)0, (R)0);
      }
      if (col) {
        // FP32 transforms of evaluation jobs take the single-precision symbol
        const bool f32sym = sizeof(R) == 4 && jb.sym == SYM_EVAL;
        float kxf = 0.f, bxf = 1.f, kys = 0.f;
        if (f32sym) {
          kxf = (float)(2.0 * M_PI * (double)p / G.lx);
          if (jb.ev.pre) bxf = (float)((4.0 + 2.0 * cos(2.0 * M_PI * (double)p / (double)jb.ev.gx)) / 6.0);
          kys = (float)(2.0 * M_PI / G.ly);
        }
        for (int k0 = 0; k0 < E && 64 * k0 < G.ny; k0 += B) {
          cd v[B];
#pragma unroll
          for (int k = 0; k < B; ++k) {
            const int q = lane + 64 * (k0 + k);
            const int qs = q >= half ? q - G.ny : q;  // kept: -ny/2 < qs < ny/2
            v[k] = mk(0.0, 0.0);
            if (q < G.ny && qs > -half) v[k] = jb.src[(size_t)q * G.nxh + p];
          }
#pragma unroll
          for (int k = 0; k < B; ++k) {
            const int q = lane + 64 * (k0 + k);
            const int qs = q >= half ? q - G.ny : q;
            if (q < G.ny && qs > -half) {
              cpx<R> o;
              if (f32sym) {
                const cpx<float> sy = symbol_eval_f32(G, jb, kxf, bxf, kys, qs);
                const float vx = (float)v[k].x, vy = (float)v[k].y;
                o = mk((R)(vx * sy.x - vy * sy.y), (R)(vx * sy.y + vy * sy.x));
              } else {
                const cd w = cmul(v[k], symbol_of(G, jb, p, qs));
                double ax = 0.0, ay = 0.0;
                ax += w.x;
                ay += w.y;
                o = mk((R)ax, (R)ay);
              }
              buf[sk(qs >= 0 ? qs : qs + Ly)] = o;
            }
          }
        }
      }
      filled = true;
    }
  }
  if (!filled) {
    for (int s = lane; s < Ly; s += 64) {
      cd v = yinv_slot(jb, G, Ly, p, s);
      buf[sk(s)] = mk((R)v.x, (R)v.y);
    }
  }
  wave_sync();
  wave_fft_any<R, MAXE, NS0>(buf, plan, +1, lane);
  cpx<R>* dst = reinterpret_cast<cpx<R>*>(jb.dst);
  for (int r = lane; r < nrows; r += 64) {
    int y = row0 + r;
    if (y >= Ly) y -= Ly * (y / Ly);
    dst[(size_t)r * G.nxh + p] = buf[sk(y)];
  }
}

template <typename R>
__device__ __forceinline__ void yinv_body(const YInvJob& jb, const Geom& G, const FftPlan& plan, int TW, int nrows,
                                          int row0, unsigned char* smem) {
  using C = cpx<R>;
  const int Ly = plan.n;
  C* a = reinterpret_cast<C*>(smem);
  C* b = a + (size_t)TW * Ly;
  const int p0 = blockIdx.x * TW;
  const int half = G.ny / 2;
  for (int e = threadIdx.x; e < Ly * TW; e += blockDim.x) {
    const int s = e / TW, c = e - s * TW, p = p0 + c;
    double ax = 0.0, ay = 0.0;
    if (p < G.nxh && 2 * p != G.nx) {
      if (G.ny == 1) {
        if (s == 0) {
          cd v = cmul(jb.src[p], symbol_of(G, jb, p, 0));
          ax = v.x;
          ay = v.y;
        }
      } else {
        for (int qs = s - ((s + half - 1) / Ly) * Ly; qs <= half - 1; qs += Ly) {
          const int q = qs >= 0 ? qs : qs + G.ny;
          cd v = cmul(jb.src[(size_t)q * G.nxh + p], symbol_of(G, jb, p, qs));
          ax += v.x;
          ay += v.y;
        }
      }
    }
    a[(size_t)c * Ly + s] = mk((R)ax, (R)ay);
  }
  __syncthreads();
  C* res = block_fft<R>(a, b, plan, TW, +1);
  C* dst = reinterpret_cast<C*>(jb.dst);
  for (int e = threadIdx.x; e < nrows * TW; e += blockDim.x) {
    const int r = e / TW, c = e - r * TW, p = p0 + c;
    if (p < G.nxh) {
      const int y = (row0 + r) % Ly;
      dst[(size_t)r * G.nxh + p] = res[(size_t)c * Ly + y];
    }
  }
}

