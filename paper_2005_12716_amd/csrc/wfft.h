// Wavefront-level FFT: one 64-lane wavefront transforms one sequence held in
// its own LDS buffer, in place, with mixed-radix self-sorting (Stockham)
// passes of radix 16, 8, 4, 2, 3 or 5.  In every pass each lane first loads
// all of its butterflies into registers, the wavefront synchronises, then each
// lane twiddles, transforms and stores; no workgroup barrier is involved, so
// the waves of a workgroup run independent transforms.
//
// MAXE is the largest number of elements per lane (n <= 64 MAXE); register
// arrays are sized by it.  Twiddles come from a table exp(-2 pi i m / n)
// computed in FP64 and rounded to the transform precision.
#pragma once

#include "common.h"

// LDS index of element i of a wavefront FFT buffer: one pad slot every 16
// elements, so the strided stores of the early Stockham passes spread over
// the banks.  Buffers hold wbuf_len(n) elements.
__host__ __device__ __forceinline__ int sk(int i) { return i + (i >> 4); }
__host__ __device__ __forceinline__ int wbuf_len(int n) { return n + (n >> 4) + 1; }

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// exp(sign i pi m / 8) for the inner twiddles of the radix-16 butterfly
template <typename R>
__device__ __forceinline__ cpx<R> w16(int m, int sign) {
  const R c1 = (R)0.92387953251128675613, s1 = (R)0.38268343236508977173, h = (R)0.70710678118654752440;
  switch (m) {
    case 1: return mk(c1, sign * s1);
    case 2: return mk(h, sign * h);
    case 3: return mk(s1, sign * c1);
    case 4: return mk((R)0, (R)sign);
    case 6: return mk(-h, sign * h);
    case 9: return mk(-c1, -sign * s1);
    default: return mk((R)1, (R)0);
  }
}

// 16-point DFT as 4 x 4 with inner twiddles exp(sign 2 pi i n2 k1 / 16).
template <typename R>
__device__ __forceinline__ void dft16(cpx<R>* v, int sign) {
  cpx<R> a[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    cpx<R> t[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
    dft4(t, sign);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) a[n2][k1] = (n2 * k1 == 0) ? t[k1] : cmul(t[k1], w16<R>(n2 * k1, sign));
  }
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cpx<R> t[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
    dft4(t, sign);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
  }
}

template <typename R, int RAD>
__device__ __forceinline__ void dft_any(cpx<R>* v, int sign) {
  if (RAD == 2) dft2(v);
  else if (RAD == 3) dft3(v, sign);
  else if (RAD == 4) dft4(v, sign);
  else if (RAD == 5) dft5(v, sign);
  else if (RAD == 8) dft8(v, sign);
  else dft16(v, sign);
}

// ts: twiddle stride (the table holds the twiddles of a length ts n)
template <typename R, int RAD, int MAXE>
__device__ __forceinline__ void wave_pass(cpx<R>* buf, int n, int Ns, const cpx<R>* __restrict__ tw, int sign,
                                          int lane, int ts = 1) {
  constexpr int MAXB = (MAXE + RAD - 1) / RAD;
  const int nb = n / RAD;
  const int twstep = n / (Ns * RAD);
  const bool pow2 = (Ns & (Ns - 1)) == 0;
  cpx<R> v[MAXB][RAD];
#pragma unroll
  for (int m = 0; m < MAXB; ++m) {
    const int j = lane + 64 * m;
    if (j < nb) {
#pragma unroll
      for (int r = 0; r < RAD; ++r) v[m][r] = buf[sk(j + r * nb)];
    }
  }
  wave_sync();
#pragma unroll
  for (int m = 0; m < MAXB; ++m) {
    const int j = lane + 64 * m;
    if (j < nb) {
      const int k = pow2 ? (j & (Ns - 1)) : (j % Ns);
      if (k > 0) {
#pragma unroll
        for (int r = 1; r < RAD; ++r) {
          cpx<R> w = tw[k * r * twstep * ts];
          if (sign > 0) w.y = -w.y;
          v[m][r] = cmul(v[m][r], w);
        }
      }
      dft_any<R, RAD>(v[m], sign);
      const int o = (j - k) * RAD + k;
#pragma unroll
      for (int r = 0; r < RAD; ++r) buf[sk(o + r * Ns)] = v[m][r];
    }
  }
  wave_sync();
}

// Plan for the wavefront FFT: radices 16 first, then one of 8/4/2, then 3s
// and 5s.
struct WPlan {
  int n;
  int nrad;
  int rad[kMaxRad];
  const void* tw;
};

inline WPlan make_wplan(const FftPlan& p) {
  WPlan w{};
  w.n = p.n;
  w.tw = p.tw;
  int n = p.n;
  int np = 0;
  while (n % 16 == 0) { w.rad[np++] = 16; n /= 16; }
  if (n % 8 == 0) { w.rad[np++] = 8; n /= 8; }
  if (n % 4 == 0) { w.rad[np++] = 4; n /= 4; }
  if (n % 2 == 0) { w.rad[np++] = 2; n /= 2; }
  while (n % 3 == 0) { w.rad[np++] = 3; n /= 3; }
  while (n % 5 == 0) { w.rad[np++] = 5; n /= 5; }
  w.nrad = np;
  return w;
}

// Elements per lane a kernel instantiation must hold for length n.
inline int wave_maxe(int n) {
  const int e = (n + 63) / 64;
  if (e <= 8) return 8;
  if (e <= 16) return 16;
  if (e <= 32) return 32;
  if (e <= 48) return 48;
  return 64;
}

// ts: twiddle stride, for a plan whose table is that of a length ts n
template <typename R, int MAXE>
__device__ void wave_fft(cpx<R>* buf, const WPlan& plan, int sign, int lane, int ts = 1) {
  const cpx<R>* tw = reinterpret_cast<const cpx<R>*>(plan.tw);
  int Ns = 1;
  for (int p = 0; p < plan.nrad; ++p) {
    switch (plan.rad[p]) {
      case 16: wave_pass<R, 16, MAXE>(buf, plan.n, Ns, tw, sign, lane, ts); break;
      case 8: wave_pass<R, 8, MAXE>(buf, plan.n, Ns, tw, sign, lane, ts); break;
      case 4: wave_pass<R, 4, MAXE>(buf, plan.n, Ns, tw, sign, lane, ts); break;
      case 2: wave_pass<R, 2, MAXE>(buf, plan.n, Ns, tw, sign, lane, ts); break;
      case 3: wave_pass<R, 3, MAXE>(buf, plan.n, Ns, tw, sign, lane, ts); break;
      default: wave_pass<R, 5, MAXE>(buf, plan.n, Ns, tw, sign, lane, ts); break;
    }
    Ns *= plan.rad[p];
  }
}

// ---------------------------------------------------------------------------
// Compile-time-length version for powers of two (64 ... 4096): radix-16
// passes with Ns = 1, 16, 256, then one radix 2/4/8/16 pass.  Every stride is
// a constant, so the skewed LDS addresses reduce to one base register plus
// immediate offsets.
// HT: read the pass's twiddles before its LDS loads, so that their latency
// overlaps the loads (the wavefront fence after them keeps the compiler from
// issuing later global reads early); costs the registers that hold them, so
// it is chosen per kernel.
template <typename R, int N, int RAD, int NS, int TS = 1, bool HT = false>
__device__ __forceinline__ void spass(cpx<R>* buf, const cpx<R>* __restrict__ tw, int sign, int lane) {
  constexpr int NB = N / RAD;
  constexpr int MB = (NB + 63) / 64;
  constexpr int TWS = N / (NS * RAD);
  static_assert(16 % RAD == 0 || RAD == 16, "radix must divide 16");
  static_assert(NS == 1 || NS % 16 == 0, "pass stride must be 1 or a multiple of 16");
  cpx<R> v[MB][RAD];
  // twiddles read before the LDS loads: the wavefront fence after those
  // loads keeps later global reads from being issued early
  cpx<R> tws[MB][NS > 1 && HT ? RAD : 1];
  if constexpr (NS > 1 && HT) {
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      const int k = (lane + 64 * m) & (NS - 1);
#pragma unroll
      for (int r = 1; r < RAD; ++r) tws[m][r] = tw[k * r * TWS * TS];
    }
  }
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int j = lane + 64 * m;
    if (NB % 64 == 0 || j < NB) {
      if constexpr (NB % 16 == 0) {
        constexpr int SB = NB + NB / 16;
        const int b = sk(j);
#pragma unroll
        for (int r = 0; r < RAD; ++r) v[m][r] = buf[b + r * SB];
      } else {
#pragma unroll
        for (int r = 0; r < RAD; ++r) v[m][r] = buf[sk(j + r * NB)];
      }
    }
  }
  wave_sync();
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int j = lane + 64 * m;
    if (NB % 64 == 0 || j < NB) {
      const int k = j & (NS - 1);
      if constexpr (NS > 1) {
        if (k > 0) {
#pragma unroll
          for (int r = 1; r < RAD; ++r) {
            cpx<R> w;
            if constexpr (HT) w = tws[m][r];
            else w = tw[k * r * TWS * TS];
            if (sign > 0) w.y = -w.y;
            v[m][r] = cmul(v[m][r], w);
          }
        }
      }
      dft_any<R, RAD>(v[m], sign);
      const int o = (j - k) * RAD + k;
      if constexpr (NS == 1) {
        const int b = o + (o >> 4);
#pragma unroll
        for (int r = 0; r < RAD; ++r) buf[b + r] = v[m][r];
      } else {
        constexpr int SS = NS + NS / 16;
        const int b = sk(o);
#pragma unroll
        for (int r = 0; r < RAD; ++r) buf[b + r * SS] = v[m][r];
      }
    }
  }
  wave_sync();
}

// TS: stride of the twiddle table (the N TS-point table of a larger transform).
template <typename R, int N, int TS = 1, bool HT = false>
__device__ __forceinline__ void wave_fft_static(cpx<R>* buf, const cpx<R>* __restrict__ tw, int sign, int lane) {
  static_assert(N >= 64 && N <= 4096 && (N & (N - 1)) == 0, "power of two in [64, 4096]");
  spass<R, N, 16, 1, TS, HT>(buf, tw, sign, lane);
  if constexpr (N == 64) spass<R, N, 4, 16, TS, HT>(buf, tw, sign, lane);
  else if constexpr (N == 128) spass<R, N, 8, 16, TS, HT>(buf, tw, sign, lane);
  else {
    spass<R, N, 16, 16, TS, HT>(buf, tw, sign, lane);
    if constexpr (N == 512) spass<R, N, 2, 256, TS, HT>(buf, tw, sign, lane);
    else if constexpr (N == 1024) spass<R, N, 4, 256, TS, HT>(buf, tw, sign, lane);
    else if constexpr (N == 2048) spass<R, N, 8, 256, TS, HT>(buf, tw, sign, lane);
    else if constexpr (N == 4096) spass<R, N, 16, 256, TS, HT>(buf, tw, sign, lane);
  }
}

// Transform with compile-time length NS0 when NS0 > 0, else the runtime plan.
template <typename R, int MAXE, int NS0, bool HT = false>
__device__ __forceinline__ void wave_fft_any(cpx<R>* buf, const WPlan& plan, int sign, int lane) {
  if constexpr (NS0 > 0) wave_fft_static<R, NS0, 1, HT>(buf, reinterpret_cast<const cpx<R>*>(plan.tw), sign, lane);
  else wave_fft<R, MAXE>(buf, plan, sign, lane);
}

// ---------------------------------------------------------------------------
// Workgroup FFT of N = 4Q points (Q a power of two, 64 <= Q <= 1024) by the
// four wavefronts of a 256-thread workgroup, decimating in time by 4:
// wavefront w transforms the decimated sequence x[4m + w] (m < Q) in its own
// sub-buffer with radix-4 (and one radix-2) Stockham passes, so that every
// lane holds one butterfly per pass; then every thread combines the four
// sub-spectra at frequencies k' < Q with the twiddles W_N^(w k') and a
// 4-point DFT:  X[k' + Q j] = sum_w W_4^(w j) W_N^(w k') Y_w[k'].  Four
// times the lanes of a single-wavefront transform work on one sequence.
// Input element n sits at b4_in<Q>(n), output element k at b4_out<Q>(k);
// sub-buffer w holds wbuf_len(Q) elements at w wbuf_len(Q).  The table `tw`
// is the N-point one (the sub-transforms read every fourth entry).

template <int Q>
__device__ __forceinline__ int b4_in(int n) { return (n & 3) * (Q + Q / 16 + 1) + sk(n >> 2); }
template <int Q>
__device__ __forceinline__ int b4_out(int k) { return (k / Q) * (Q + Q / 16 + 1) + sk(k % Q); }

// One Stockham pass of a length-Q wavefront transform, twiddles tw[TS m].
template <typename R, int Q, int RAD, int NS, int TS, bool HT = false>
__device__ __forceinline__ void qpass(cpx<R>* buf, const cpx<R>* __restrict__ tw, int sign, int lane) {
  constexpr int NB = Q / RAD;
  constexpr int MB = (NB + 63) / 64;
  constexpr int TWS = Q / (NS * RAD);
  cpx<R> v[MB][RAD];
  cpx<R> tws[MB][NS > 1 && HT ? RAD : 1];  // twiddles read before the LDS loads (HT)
  if constexpr (NS > 1 && HT) {
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      const int k = (lane + 64 * m) & (NS - 1);
#pragma unroll
      for (int r = 1; r < RAD; ++r) tws[m][r] = tw[k * r * TWS * TS];
    }
  }
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int j = lane + 64 * m;
    if (NB % 64 == 0 || j < NB) {
#pragma unroll
      for (int r = 0; r < RAD; ++r) v[m][r] = buf[sk(j + r * NB)];
    }
  }
  wave_sync();
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int j = lane + 64 * m;
    if (NB % 64 == 0 || j < NB) {
      const int k = j & (NS - 1);
      if constexpr (NS > 1) {
        if (k > 0) {
#pragma unroll
          for (int r = 1; r < RAD; ++r) {
            cpx<R> w;
            if constexpr (HT) w = tws[m][r];
            else w = tw[k * r * TWS * TS];
            if (sign > 0) w.y = -w.y;
            v[m][r] = cmul(v[m][r], w);
          }
        }
      }
      dft_any<R, RAD>(v[m], sign);
      const int o = (j - k) * RAD + k;
#pragma unroll
      for (int r = 0; r < RAD; ++r) buf[sk(o + r * NS)] = v[m][r];
    }
  }
  wave_sync();
}

template <typename R, int Q, int TS, int NS = 1, bool HT = false>
__device__ __forceinline__ void wave_fft_r4(cpx<R>* buf, const cpx<R>* __restrict__ tw, int sign, int lane) {
  if constexpr (NS * 4 <= Q) {
    qpass<R, Q, 4, NS, TS, HT>(buf, tw, sign, lane);
    wave_fft_r4<R, Q, TS, NS * 4, HT>(buf, tw, sign, lane);
  } else if constexpr (NS * 2 == Q) {
    qpass<R, Q, 2, NS, TS, HT>(buf, tw, sign, lane);
  }
}

// All 256 threads of the workgroup must call this; it starts with a block
// barrier (the inputs may have been written by any thread) and ends with one.
template <typename R, int N, bool HT = false>
__device__ __forceinline__ void block4_fft(cpx<R>* buf, const cpx<R>* __restrict__ tw, int sign) {
  constexpr int Q = N / 4;
  static_assert(Q >= 64 && Q <= 1024 && (Q & (Q - 1)) == 0, "N = 4Q with Q a power of two in [64, 1024]");
  constexpr int WL = Q + Q / 16 + 1;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lane = threadIdx.x & 63;
  __syncthreads();
  wave_fft_r4<R, Q, 4, 1, HT>(buf + wave * WL, tw, sign, lane);
  __syncthreads();
#pragma unroll
  for (int k0 = 0; k0 < Q; k0 += 256) {
    const int kq = k0 + (int)threadIdx.x;
    if (Q % 256 == 0 || kq < Q) {
      cpx<R> a[4];
#pragma unroll
      for (int w = 0; w < 4; ++w) a[w] = buf[w * WL + sk(kq)];
#pragma unroll
      for (int w = 1; w < 4; ++w) {
        cpx<R> t = tw[w * kq];
        if (sign > 0) t.y = -t.y;
        a[w] = cmul(a[w], t);
      }
      dft4(a, sign);
#pragma unroll
      for (int j = 0; j < 4; ++j) buf[j * WL + sk(kq)] = a[j];
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Transforms of N = 3Q points (Q a power of two, 64 <= Q <= 1024),
// decimating in time by 3: the sequence x[3m + r] (m < Q) is transformed in
// sub-buffer r with the compile-time radix-16 passes (every third entry of
// the N-point table), then X[k' + Q j] = sum_r W_3^(r j) W_N^(r k') Y_r[k'] for k' < Q.
// Input element n sits at b3_in<Q>(n), output element k at b3_out<Q>(k); the
// three sub-buffers take b3_len<Q>() elements.  Each k' is combined in place
// by one thread (it reads and writes the same three slots).
// Sub-buffer stride: the skewed length Q + Q/16 + 1 rounded up to 11 mod 32
// (8-byte elements), so that the consecutive elements n of b3_in, which
// cycle through the three sub-buffers, fall into distinct banks for 16 as
// for 32 lanes of 8-byte accesses per cycle (offsets 11 r + n/3 are distinct
// mod 16 for n < 16 and mod 32 for n < 32).
template <int Q>
__host__ __device__ constexpr int b3_stride() {
  return (Q + Q / 16 + 1) + ((11 - (Q + Q / 16 + 1) % 32) + 32) % 32;
}
template <int Q>
__host__ __device__ constexpr int b3_len() { return 3 * b3_stride<Q>(); }
template <int Q>
__device__ __forceinline__ int b3_in(int n) { return (n % 3) * b3_stride<Q>() + sk(n / 3); }
template <int Q>
__device__ __forceinline__ int b3_out(int k) { return (k / Q) * b3_stride<Q>() + sk(k % Q); }

template <typename R, int Q>
__device__ __forceinline__ void b3_combine(cpx<R>* buf, const cpx<R>* __restrict__ tw, int sign, int kq) {
  constexpr int WL = b3_stride<Q>();
  cpx<R> a[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) a[r] = buf[r * WL + sk(kq)];
#pragma unroll
  for (int r = 1; r < 3; ++r) {
    cpx<R> t = tw[r * kq];
    if (sign > 0) t.y = -t.y;
    a[r] = cmul(a[r], t);
  }
  dft3(a, sign);
#pragma unroll
  for (int j = 0; j < 3; ++j) buf[j * WL + sk(kq)] = a[j];
}

// One wavefront: the three sub-transforms, then the combine.
template <typename R, int Q>
__device__ __forceinline__ void wave_fft3(cpx<R>* buf, const cpx<R>* __restrict__ tw, int sign, int lane) {
  static_assert(Q >= 64 && Q <= 1024 && (Q & (Q - 1)) == 0, "N = 3Q with Q a power of two in [64, 1024]");
  constexpr int WL = b3_stride<Q>();
#pragma unroll
  for (int r = 0; r < 3; ++r) wave_fft_static<R, Q, 3>(buf + r * WL, tw, sign, lane);
#pragma unroll
  for (int k0 = 0; k0 < Q; k0 += 64) b3_combine<R, Q>(buf, tw, sign, k0 + lane);
  wave_sync();
}

// The workgroup (NT threads, all must call; NT a multiple of 64, at least
// 192): wavefronts 0-2 take one sub-transform each, every thread combines.
// Starts and ends with a block barrier.
template <typename R, int Q, int NT = 256, bool HT = false>
__device__ __forceinline__ void block3_fft(cpx<R>* buf, const cpx<R>* __restrict__ tw, int sign) {
  static_assert(Q >= 64 && Q <= 1024 && (Q & (Q - 1)) == 0, "N = 3Q with Q a power of two in [64, 1024]");
  static_assert(NT % 64 == 0 && NT >= 192, "three wavefronts at least");
  constexpr int WL = b3_stride<Q>();
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lane = threadIdx.x & 63;
  __syncthreads();
  if (wave < 3) wave_fft_static<R, Q, 3, HT>(buf + wave * WL, tw, sign, lane);
  __syncthreads();
#pragma unroll
  for (int k0 = 0; k0 < Q; k0 += NT) {
    const int kq = k0 + (int)threadIdx.x;
    if (Q % NT == 0 || kq < Q) b3_combine<R, Q>(buf, tw, sign, kq);
  }
  __syncthreads();
}

// Host: choose (MAXE, N) template arguments for a length n.
#define SW_FFT_DISPATCH(n, LAUNCH)          \
  switch (n) {                              \
    case 64: LAUNCH(8, 64); break;          \
    case 128: LAUNCH(8, 128); break;        \
    case 256: LAUNCH(8, 256); break;        \
    case 512: LAUNCH(8, 512); break;        \
    case 1024: LAUNCH(16, 1024); break;     \
    case 2048: LAUNCH(32, 2048); break;     \
    case 4096: LAUNCH(64, 4096); break;     \
    default:                                \
      switch (wave_maxe(n)) {               \
        case 8: LAUNCH(8, 0); break;        \
        case 16: LAUNCH(16, 0); break;      \
        case 32: LAUNCH(32, 0); break;      \
        case 48: LAUNCH(48, 0); break;      \
        default: LAUNCH(64, 0); break;      \
      }                                     \
  }

// Block index remapped so that the blocks resident on one XCD (blocks are
// dealt round-robin over the 8 XCDs) process a contiguous range of tiles.
__device__ __forceinline__ int xcd_tile(int b, int nblocks) {
  const int q = nblocks >> 3, r = nblocks & 7;
  const int xcd = b & 7, k = b >> 3;
  return xcd * q + min(xcd, r) + k;
}

// Block b of a one-dimensional grid of ncol x nly blocks -> (column p, slot
// ly), a bijection: each XCD takes a contiguous run of the sequence (group of
// GW adjacent columns, slot, column in the group), so a group's per-column
// inputs stay in that XCD's L2 across the slots and the GW blocks that write
// one slot's rows at adjacent columns run back to back.
template <int GW>
__device__ __forceinline__ void grouped_tile(int b, int ncol, int nly, int& p, int& ly) {
  const int seq = xcd_tile(b, ncol * nly);
  const int per = GW * nly;
  const int cg = seq / per;
  const int rem = seq - cg * per;
  const int w = min(GW, ncol - cg * GW);
  ly = rem / w;
  p = cg * GW + (rem - ly * w);
}
