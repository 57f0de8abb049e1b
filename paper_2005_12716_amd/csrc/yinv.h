// Inverse transform along y of symbol-weighted half spectra (shared by the
// HOS step and the grid evaluation).
#pragma once

#include "internal.h"
#include "wfft.h"

// Workgroup transforms (one sequence per 256-thread workgroup) exist for
// power-of-two lengths in [256, 4096] (block4_fft) and for 768, 1536 and
// 3072 points (block3_fft).
__host__ __device__ constexpr bool b4_len_ok(int n) { return n >= 256 && n <= 4096 && (n & (n - 1)) == 0; }
__host__ __device__ constexpr bool b3_len_ok(int n) { return n == 768 || n == 1536 || n == 3072; }
__host__ __device__ constexpr bool grp_len_ok(int n) { return b4_len_ok(n) || b3_len_ok(n); }
// LDS elements of a workgroup transform of length n
inline size_t grp_lds_len(int n) {
  if (b3_len_ok(n)) return n == 768 ? b3_len<256>() : (n == 1536 ? b3_len<512>() : b3_len<1024>());
  return 4ull * wbuf_len(n / 4);
}

// Slot of element n of a workgroup transform's input, of element k of its
// output, and the transform itself.
template <int N>
__device__ __forceinline__ int grp_in(int n) {
  if constexpr (N % 3 == 0) return b3_in<N / 3>(n); else return b4_in<N / 4>(n);
}
template <int N>
__device__ __forceinline__ int grp_out(int k) {
  if constexpr (N % 3 == 0) return b3_out<N / 3>(k); else return b4_out<N / 4>(k);
}
template <typename R, int N>
__device__ __forceinline__ void grp_fft(cpx<R>* buf, const cpx<R>* __restrict__ tw, int sign) {
  // twiddles read ahead of each pass's LDS loads for the long transforms
  // (measured faster at 3072 and 4096 points; the shorter ones keep their
  // occupancy instead)
  constexpr bool HT = N >= 3072;
  if constexpr (N % 3 == 0) block3_fft<R, N / 3, 256, HT>(buf, tw, sign); else block4_fft<R, N, HT>(buf, tw, sign);
}

#define SW_B4_DISPATCH(n, LAUNCH) \
  switch (n) {                    \
    case 256: LAUNCH(256); break;   \
    case 512: LAUNCH(512); break;   \
    case 1024: LAUNCH(1024); break; \
    case 2048: LAUNCH(2048); break; \
    case 768: LAUNCH(768); break;   \
    case 1536: LAUNCH(1536); break; \
    case 3072: LAUNCH(3072); break; \
    default: LAUNCH(4096); break;   \
  }

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
              // symbol (vertical factor, multiplier, prefilter) in FP64
              const cd w = cmul(v[k], symbol_of(G, jb, p, qs));
              buf[sk(qs >= 0 ? qs : qs + Ly)] = mk((R)w.x, (R)w.y);
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

