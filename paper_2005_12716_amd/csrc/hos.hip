// High-Order Spectral free-surface step on gfx950 (Sec. 3.1.2).
//
// State: FP64 half spectra (eta_hat, phis_hat) [ny][nx/2+1].  One right-hand
// side is a chain of three kinds of launches:
//   y-inverse : per column tile of kx, multiply the FP64 spectrum by a FP64
//               symbol (1, i ky, Dz^j = k^j (tanh kh)^{j odd}, ...), zero-pad
//               ny -> Py, inverse transform along y in LDS, store rows
//               [Py][nx/2+1] (x still spectral) in the transform precision;
//   x pass    : one block per physical row; builds every needed physical field
//               by an inverse x transform (two real fields packed in one
//               complex transform), forms the order-M products in LDS and
//               transforms the result(s) forward again, keeping the nx/2 kept
//               modes - the padded physical grid never touches HBM;
//   y-forward : forward y transform, truncation to the ny kept modes, and an
//               epilogue that stores a series mode or adds the exact linear
//               part of the right-hand side in FP64 and performs the RK4 stage
//               update in place.
// Series (West et al. expansion of the vertical velocity, order M):
//   phi^(1) = phis, phi^(m+1) = -sum_{j=1..m} eta^j/j! g(m+1-j, j),
//   W^(m) = sum_{j=0..m-1} eta^j/j! g(m-j, j+1),  g(m,j) = F^-1(Dz^j phi^(m)).
// Only the nonlinear remainders eta_t - W^(1) and phis_t + g eta pass through
// the reduced-precision transforms; Dz phis and -g eta are added exactly.
#include "internal.h"
#include "yinv.h"

#include <algorithm>
#include <cstring>
#include <vector>

namespace {

// ------------------------------------------------------------------ device
template <typename R>
__global__ void __launch_bounds__(256) k_yinv(YInvArgs args, Geom G, FftPlan plan, int TW, int nrows, int row0) {
  extern __shared__ unsigned char smem[];
  yinv_body<R>(args.job[blockIdx.y], G, plan, TW, nrows, row0, smem);
}

// v times i kx for mode p (kx rounded once from FP64 to the row precision)
template <typename R>
__device__ __forceinline__ cpx<R> times_ikx(cpx<R> v, int p, const Geom& G) {
  const R kx = (R)(2.0 * M_PI * (double)p / G.lx);
  return mk(-kx * v.y, kx * v.x);
}

template <typename R>
__device__ __forceinline__ cpx<R> load_row(const XIn& f, int y, int p, const Geom& G) {
  cpx<R> v = reinterpret_cast<const cpx<R>*>(f.src)[(size_t)y * G.nxh + p];
  if (f.dx) v = times_ikx<R>(v, p, G);
  return v;
}

template <typename R>
__device__ __forceinline__ void apply_role(const XIn& f, R v, R other, int x, int Px, R* acc, const XArgs& A) {
  switch (f.role) {
    case XR_ETA: acc[A.s_eta * Px + x] = v; break;
    case XR_GRADPAIR:
      acc[A.s_ge2 * Px + x] += v * v;
      acc[A.s_dot * Px + x] += v * other;
      acc[A.s_gp2 * Px + x] += other * other;
      break;
    case XR_G: {
      const R e = acc[A.s_eta * Px + x];
      R c = (R)1;
      for (int k = 1; k <= f.pw; ++k) c *= e / (R)k;
      acc[f.slot * Px + x] += c * v;
    } break;
    case XR_ETAT: acc[A.s_etat * Px + x] = v; break;
    case XR_PHIT: acc[A.s_phit * Px + x] = v; break;
    default: break;
  }
}

template <typename R>
__device__ __forceinline__ R w2sum(const R* W, int K) {
  // [W^2]_K = sum_{m=2..K} sum_{l=1..m-1} W^(l) W^(m-l); unrolled to constant indices
  R s = (R)0;
#pragma unroll
  for (int m = 2; m <= kMaxM; ++m)
#pragma unroll
    for (int l = 1; l < m; ++l)
      if (m <= K) s += W[l - 1] * W[m - l - 1];
  return s;
}

// Fused x pass: one block per physical row y of the product grid.
template <typename R>
__global__ void __launch_bounds__(256) k_xpass(XArgs A, Geom G, FftPlan plan) {
  extern __shared__ unsigned char smem[];
  using C = cpx<R>;
  const int Px = plan.n;
  const int y = blockIdx.x;
  const int hx = G.nx / 2;
  C* za = reinterpret_cast<C*>(smem);
  C* zb = za + Px;
  R* acc = reinterpret_cast<R*>(zb + Px);
  for (int e = threadIdx.x; e < A.nslots * Px; e += blockDim.x) acc[e] = (R)0;
  for (int i = 0; i < A.nin; i += 2) {
    const XIn& fa = A.in[i];
    const bool hasb = (i + 1) < A.nin;
    const XIn& fb = A.in[hasb ? i + 1 : i];
    for (int s = threadIdx.x; s < Px; s += blockDim.x) {
      C z = mk((R)0, (R)0);
      if (s < hx) {
        C va = load_row<R>(fa, y, s, G);
        C vb = hasb ? load_row<R>(fb, y, s, G) : mk((R)0, (R)0);
        z = mk(va.x - vb.y, va.y + vb.x);  // va + i vb
      } else if (s > Px - hx) {
        const int p = Px - s;
        C va = conjg(load_row<R>(fa, y, p, G));
        C vb = hasb ? conjg(load_row<R>(fb, y, p, G)) : mk((R)0, (R)0);
        z = mk(va.x - vb.y, va.y + vb.x);
      }
      za[s] = z;
    }
    __syncthreads();
    C* res = block_fft<R>(za, zb, plan, 1, +1);
    for (int x = threadIdx.x; x < Px; x += blockDim.x) {
      const R va = res[x].x, vb = res[x].y;
      apply_role<R>(fa, va, vb, x, Px, acc, A);
      if (hasb && fa.role != XR_GRADPAIR) apply_role<R>(fb, vb, (R)0, x, Px, acc, A);
    }
    __syncthreads();
  }
  const int M = A.M;
  for (int x = threadIdx.x; x < Px; x += blockDim.x) {
    R o0 = (R)0, o1 = (R)0;
    if (A.stage == XS_SERIES) {
      o0 = -acc[A.s_w[0] * Px + x];
    } else if (A.stage == XS_FTILDE) {
      o0 = acc[A.s_phit * Px + x];
      if (M >= 2) o0 -= acc[A.s_w[0] * Px + x] * acc[A.s_etat * Px + x];
    } else {
      R W[kMaxM];
      R wm = (R)0, wm2 = (R)0;
      for (int m = 0; m < M; ++m) {
        W[m] = acc[A.s_w[m] * Px + x];
        wm += W[m];
        if (m < M - 2) wm2 += W[m];
      }
      const R ge2 = acc[A.s_ge2 * Px + x];
      const R dot = acc[A.s_dot * Px + x];
      const R gp2 = acc[A.s_gp2 * Px + x];
      o0 = wm - W[0];
      if (M >= 3) o0 += ge2 * wm2;
      if (M >= 2) o0 -= dot;
      o1 = (R)0.5 * w2sum(W, M);
      if (M >= 2) o1 -= (R)0.5 * gp2;
      if (M >= 4) o1 += (R)0.5 * ge2 * w2sum(W, M - 2);
    }
    za[x] = mk(o0, o1);
  }
  __syncthreads();
  C* res = block_fft<R>(za, zb, plan, 1, -1);
  const R sc = (R)(0.5 / (double)Px);
  C* d0 = reinterpret_cast<C*>(A.out0);
  C* d1 = reinterpret_cast<C*>(A.out1);
  for (int p = threadIdx.x; p < G.nxh; p += blockDim.x) {
    C o0 = mk((R)0, (R)0), o1 = mk((R)0, (R)0);
    if (p < hx) {
      C zp = res[p];
      C zm = conjg(res[(Px - p) % Px]);
      C s = zp + zm, t = zp - zm;
      o0 = cscale(s, sc);
      o1 = mk(t.y * sc, -t.x * sc);
    }
    d0[(size_t)y * G.nxh + p] = o0;
    if (d1) d1[(size_t)y * G.nxh + p] = o1;
  }
}

// Epilogue of the forward y transform for mode (p, q) with value v, in two
// halves: the state operands the mode needs are read first (so a caller can
// issue the reads of several modes before it uses any), then the results
// are formed and stored.  Each mode touches only its own index.
struct EpiOps {
  cd s;  // other field of the stage input (linear part)
  cd x;  // base state
  cd a;  // RK accumulator (or the YE_STORE accumulate target)
};

__device__ __forceinline__ EpiOps yfwd_epi_load(const YFwdJob& jb, const RkArgs& rk, size_t idx) {
  EpiOps o;
  o.s = o.x = o.a = mk(0.0, 0.0);
  if (jb.epi == YE_STORE) {
    if (jb.acc_mode == 1) o.a = jb.acc[idx];
    return o;
  }
  if (jb.epi == YE_NL_ETA || jb.epi == YE_NL_PHI) return o;
  const int w = jb.epi == YE_RHS_ETA ? 0 : 1;
  o.s = rk.sin[1 - w][idx];
  if (rk.stage != 0) o.x = rk.xn[w][idx];
  if (rk.stage != 0 && rk.stage != 1) o.a = rk.acc[w][idx];
  return o;
}

__device__ __forceinline__ void yfwd_epi_store(const YFwdJob& jb, const RkArgs& rk, const Geom& G, int p, int q,
                                               int qs, cd v, const EpiOps& o) {
  const size_t idx = (size_t)q * G.nxh + p;
  if (jb.epi == YE_STORE) {
    jb.dst[idx] = v;
    if (jb.acc_mode == 1) jb.acc[idx] = o.a + v;
    else if (jb.acc_mode == 2) jb.acc[idx] = v;
    return;
  }
  if (jb.epi == YE_NL_ETA || jb.epi == YE_NL_PHI) {
    const bool eta = jb.epi == YE_NL_ETA;
    rk.kout[eta ? 0 : 1][idx] = (eta && p == 0 && q == 0) ? mk(0.0, 0.0) : v;
    return;
  }
  const int w = jb.epi == YE_RHS_ETA ? 0 : 1;
  cd k = v;
  if (w == 0) {
    const double kx = 2.0 * M_PI * (double)p / G.lx;
    const double ky = G.ny > 1 ? 2.0 * M_PI * (double)qs / G.ly : 0.0;
    const double kk = sqrt(kx * kx + ky * ky);
    const double dz1 = G.depth > 0.0 ? kk * tanh(kk * G.depth) : kk;
    k = k + cscale(o.s, dz1);
    if (p == 0 && q == 0) k = mk(0.0, 0.0);
  } else {
    k = k + cscale(o.s, -G.g);
  }
  switch (rk.stage) {
    case 0: rk.kout[w][idx] = k; break;
    case 1:
      rk.acc[w][idx] = k;
      rk.sout[w][idx] = o.x + cscale(k, 0.5 * rk.dt);
      break;
    case 2:
      rk.acc[w][idx] = o.a + cscale(k, 2.0);
      rk.sout[w][idx] = o.x + cscale(k, 0.5 * rk.dt);
      break;
    case 3:
      rk.acc[w][idx] = o.a + cscale(k, 2.0);
      rk.sout[w][idx] = o.x + cscale(k, rk.dt);
      break;
    default:
      rk.xn[w][idx] = o.x + cscale(o.a + k, rk.dt / 6.0);
      break;
  }
}

__device__ __forceinline__ void yfwd_epilogue(const YFwdJob& jb, const RkArgs& rk, const Geom& G, int p, int q, int qs,
                                              cd v) {
  yfwd_epi_store(jb, rk, G, p, q, qs, v, yfwd_epi_load(jb, rk, (size_t)q * G.nxh + p));
}

// y-forward: grid (ceil(nxh / TW), njobs).  Keeps modes |q| < ny/2, zeroes the
// Nyquist row and column, scales by 1/Ly, then applies the epilogue.
template <typename R>
__global__ void __launch_bounds__(256) k_yfwd(YFwdArgs A, Geom G, FftPlan plan, int TW) {
  extern __shared__ unsigned char smem[];
  using C = cpx<R>;
  const int Ly = plan.n;
  C* a = reinterpret_cast<C*>(smem);
  C* b = a + (size_t)TW * Ly;
  const YFwdJob& jb = A.job[blockIdx.y];
  const int p0 = blockIdx.x * TW;
  const C* src = reinterpret_cast<const C*>(jb.src);
  for (int e = threadIdx.x; e < Ly * TW; e += blockDim.x) {
    const int s = e / TW, c = e - s * TW, p = p0 + c;
    a[(size_t)c * Ly + s] = p < G.nxh ? src[(size_t)s * G.nxh + p] : mk((R)0, (R)0);
  }
  __syncthreads();
  C* res = block_fft<R>(a, b, plan, TW, -1);
  const double inv = 1.0 / (double)Ly;
  const RkArgs& rk = A.rk;
  for (int e = threadIdx.x; e < G.ny * TW; e += blockDim.x) {
    const int q = e / TW, c = e - q * TW, p = p0 + c;
    if (p >= G.nxh) continue;
    const int qs = signed_q(q, G.ny);
    cd v = mk(0.0, 0.0);
    if (2 * p != G.nx && !(G.ny > 1 && 2 * q == G.ny)) {
      const int slot = ((qs % Ly) + Ly) % Ly;
      C r = res[(size_t)c * Ly + slot];
      v = mk((double)r.x * inv, (double)r.y * inv);
    }
    yfwd_epilogue(jb, A.rk, G, p, q, qs, v);
  }
}

// Wavefront versions of the y transforms: one wavefront per kx column, four
// columns per block, tiles ordered XCD by XCD.
template <typename R, int MAXE, int NS0>
__global__ void __launch_bounds__(256) k_yinv_w(YInvArgs args, Geom G, WPlan plan, int nrows, int row0) {
  extern __shared__ unsigned char smem[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int p = xcd_tile(blockIdx.x, gridDim.x) * 4 + wave;
  if (p >= G.nxh) return;
  cpx<R>* buf = reinterpret_cast<cpx<R>*>(smem) + (size_t)wave * wbuf_len(plan.n);
  yinv_wave<R, MAXE, NS0>(args.job[blockIdx.y], G, plan, nrows, row0, p, buf, lane);
}

template <typename R, int MAXE, int NS0>
__global__ void __launch_bounds__(256) k_yfwd_w(YFwdArgs A, Geom G, WPlan plan) {
  extern __shared__ unsigned char smem[];
  using C = cpx<R>;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int p = xcd_tile(blockIdx.x, gridDim.x) * 4 + wave;
  if (p >= G.nxh) return;
  const int Ly = plan.n;
  C* buf = reinterpret_cast<C*>(smem) + (size_t)wave * wbuf_len(Ly);
  const YFwdJob& jb = A.job[blockIdx.y];
  const C* src = reinterpret_cast<const C*>(jb.src);
  const double inv = 1.0 / (double)Ly;
  if constexpr (NS0 > 0) {
    // The column and the state operands of the first batch of modes (which
    // do not depend on the transform) are all read before any is used;
    // later batches read theirs before forming their results.
    constexpr int E = NS0 / 64, B = E < 4 ? E : 4;
    EpiOps o[B];
    auto load_ops = [&](int q0) {
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int q = q0 + lane + 64 * k;
        if (q < G.ny) o[k] = yfwd_epi_load(jb, A.rk, (size_t)q * G.nxh + p);
      }
    };
    C colv[NS0 / 64];
#pragma unroll
    for (int j = 0; j < NS0 / 64; ++j) colv[j] = src[(size_t)(lane + 64 * j) * G.nxh + p];
    load_ops(0);
#pragma unroll
    for (int j = 0; j < NS0 / 64; ++j) buf[sk(lane + 64 * j)] = colv[j];
    wave_sync();
    wave_fft_any<R, MAXE, NS0>(buf, plan, -1, lane);
    for (int q0 = 0; q0 < G.ny; q0 += 64 * B) {
      if (q0 > 0) load_ops(q0);
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int q = q0 + lane + 64 * k;
        if (q >= G.ny) continue;
        const int qs = signed_q(q, G.ny);
        cd v = mk(0.0, 0.0);
        if (2 * p != G.nx && !(G.ny > 1 && 2 * q == G.ny)) {
          const int slot = ((qs % Ly) + Ly) % Ly;
          C r = buf[sk(slot)];
          v = mk((double)r.x * inv, (double)r.y * inv);
        }
        yfwd_epi_store(jb, A.rk, G, p, q, qs, v, o[k]);
      }
    }
  } else {
    for (int s = lane; s < Ly; s += 64) buf[sk(s)] = src[(size_t)s * G.nxh + p];
    wave_sync();
    wave_fft_any<R, MAXE, NS0>(buf, plan, -1, lane);
    for (int q = lane; q < G.ny; q += 64) {
      const int qs = signed_q(q, G.ny);
      cd v = mk(0.0, 0.0);
      if (2 * p != G.nx && !(G.ny > 1 && 2 * q == G.ny)) {
        const int slot = ((qs % Ly) + Ly) % Ly;
        C r = buf[sk(slot)];
        v = mk((double)r.x * inv, (double)r.y * inv);
      }
      yfwd_epilogue(jb, A.rk, G, p, q, qs, v);
    }
  }
}

// Workgroup versions of the y transforms for power-of-two lengths N in
// [256, 4096]: one kx column per 256-thread workgroup (columns ordered XCD by
// XCD), the column's transform done by all four wavefronts (block4_fft), and
// the loads and epilogue spread over the 256 threads.
// Lengths 768, 1536 and 3072 (three times a power of two) take the same
// kernels with the three-way workgroup transform (block3_fft).
template <typename R, int N>
__global__ void __launch_bounds__(256) k_yinv_b4(YInvArgs args, Geom G, WPlan plan, int nrows, int row0) {
  extern __shared__ unsigned char smem[];
  using C = cpx<R>;
  constexpr int T = N / 256;  // slots per thread
  C* buf = reinterpret_cast<C*>(smem);
  const int p = xcd_tile(blockIdx.x, gridDim.x);
  const YInvJob& jb = args.job[blockIdx.y];
  const int tid = threadIdx.x;
  const int half = G.ny / 2;
  const bool col = p < G.nxh && 2 * p != G.nx;
  // zero-padding in y (N >= ny): kept mode q (-ny/2 < qs < ny/2) goes to
  // slot qs mod N; every other slot is zero
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int s = tid + 256 * t;
    if (!col || (s >= half && s <= N - half)) buf[grp_in<N>(s)] = mk((R)0, (R)0);
  }
  if (col) {
    cd v[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int q = tid + 256 * t;
      const int qs = q >= half ? q - G.ny : q;
      v[t] = mk(0.0, 0.0);
      if (q < G.ny && qs > -half) v[t] = jb.src[(size_t)q * G.nxh + p];
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int q = tid + 256 * t;
      const int qs = q >= half ? q - G.ny : q;
      if (q < G.ny && qs > -half) {
        const cd w = cmul(v[t], symbol_of(G, jb, p, qs));
        double ax = 0.0, ay = 0.0;
        ax += w.x;
        ay += w.y;
        buf[grp_in<N>(qs >= 0 ? qs : qs + N)] = mk((R)ax, (R)ay);
      }
    }
  }
  grp_fft<R, N>(buf, reinterpret_cast<const C*>(plan.tw), +1);
  if (p >= G.nxh) return;
  C* dst = reinterpret_cast<C*>(jb.dst);
  for (int r = tid; r < nrows; r += 256) {
    int y = row0 + r;
    if (y >= N) y -= N * (y / N);
    dst[(size_t)r * G.nxh + p] = buf[grp_out<N>(y)];
  }
}

template <typename R, int N>
__global__ void __launch_bounds__(256) k_yfwd_b4(YFwdArgs A, Geom G, WPlan plan) {
  extern __shared__ unsigned char smem[];
  using C = cpx<R>;
  constexpr int T = N / 256;
  constexpr int TQ = 4;  // modes per thread held at once (ny <= 1024 in one batch)
  C* buf = reinterpret_cast<C*>(smem);
  const int p = xcd_tile(blockIdx.x, gridDim.x);
  const YFwdJob& jb = A.job[blockIdx.y];
  const int tid = threadIdx.x;
  const bool colp = p < G.nxh;
  // the column and the state operands of the first modes, all read first
  const C* src = reinterpret_cast<const C*>(jb.src);
  C colv[T];
  EpiOps o[TQ];
  if (colp) {
#pragma unroll
    for (int t = 0; t < T; ++t) colv[t] = src[(size_t)(tid + 256 * t) * G.nxh + p];
#pragma unroll
    for (int k = 0; k < TQ; ++k) {
      const int q = tid + 256 * k;
      if (q < G.ny) o[k] = yfwd_epi_load(jb, A.rk, (size_t)q * G.nxh + p);
    }
#pragma unroll
    for (int t = 0; t < T; ++t) buf[grp_in<N>(tid + 256 * t)] = colv[t];
  }
  grp_fft<R, N>(buf, reinterpret_cast<const C*>(plan.tw), -1);
  if (!colp) return;
  const double inv = 1.0 / (double)N;
  for (int q0 = 0; q0 < G.ny; q0 += 256 * TQ) {
    if (q0 > 0) {
#pragma unroll
      for (int k = 0; k < TQ; ++k) {
        const int q = q0 + tid + 256 * k;
        if (q < G.ny) o[k] = yfwd_epi_load(jb, A.rk, (size_t)q * G.nxh + p);
      }
    }
#pragma unroll
    for (int k = 0; k < TQ; ++k) {
      const int q = q0 + tid + 256 * k;
      if (q >= G.ny) continue;
      const int qs = signed_q(q, G.ny);
      cd v = mk(0.0, 0.0);
      if (2 * p != G.nx && !(G.ny > 1 && 2 * q == G.ny)) {
        const int slot = ((qs % N) + N) % N;
        const C r = buf[grp_out<N>(slot)];
        v = mk((double)r.x * inv, (double)r.y * inv);
      }
      yfwd_epi_store(jb, A.rk, G, p, q, qs, v, o[k]);
    }
  }
}

// Residue forms of the workgroup y passes for padded lengths N = RS ny (RS in
// {2, 3, 4}, ny a power of two, single precision).  Inverse: with y = RS s +
// r, X[y] = sum_q (x_q e^{2 pi i q r / N}) e^{2 pi i q s / ny}, so wavefront
// r transforms the modulated kept modes (no zero slots, no combine) and
// stores the rows of its residue.  Forward: the column's residue sequences
// x[RS s + r] transformed one per wavefront, then only the kept modes
// combined, Y[q] = sum_r e^{-2 pi i q r / N} Z_r[q mod ny].
template <int RS, int NY>
__global__ void __launch_bounds__(256) k_yinv_r(YInvArgs args, Geom G, WPlan plan, int nrows, int row0) {
  static_assert(RS >= 2 && RS <= 4 && NY >= 256 && NY <= 1024, "residues and lengths");
  constexpr int N = RS * NY;
  constexpr int WL = NY + NY / 16 + 1;
  constexpr int TQ = NY / 256;
  using C = cpx<float>;
  extern __shared__ unsigned char smem[];
  C* buf = reinterpret_cast<C*>(smem);
  const C* tw = reinterpret_cast<const C*>(plan.tw);
  const int p = xcd_tile(blockIdx.x, gridDim.x);
  const YInvJob& jb = args.job[blockIdx.y];
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int half = G.ny / 2;
  const bool col = p < G.nxh && 2 * p != G.nx;
  cd v[TQ];
#pragma unroll
  for (int t = 0; t < TQ; ++t) {
    const int q = tid + 256 * t;
    const int qs = q >= half ? q - G.ny : q;
    v[t] = mk(0.0, 0.0);
    if (col && qs > -half) v[t] = jb.src[(size_t)q * G.nxh + p];
  }
#pragma unroll
  for (int t = 0; t < TQ; ++t) {
    const int q = tid + 256 * t;
    const int qs = q >= half ? q - G.ny : q;
    C w = mk(0.f, 0.f);
    if (col && qs > -half) {
      const cd x = cmul(v[t], symbol_of(G, jb, p, qs));
      w = mk((float)x.x, (float)x.y);
    }
    const C tm = tw[(qs + N) % N];
    const C md = mk(tm.x, -tm.y);  // e^{2 pi i qs / N}
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      buf[r * WL + sk(q)] = w;
      w = cmul(w, md);
    }
  }
  __syncthreads();
  if (wave >= RS || p >= G.nxh) return;
  C* b = buf + wave * WL;
  wave_fft_static<float, NY, RS, true>(b, tw, +1, lane);
  C* dst = reinterpret_cast<C*>(jb.dst);
  const int r0 = ((wave - row0) % RS + RS) % RS;
  for (int rr = r0 + RS * lane; rr < nrows; rr += RS * 64) {
    int y = row0 + rr;
    if (y >= N) y -= N * (y / N);
    dst[(size_t)rr * G.nxh + p] = b[sk((y - wave) / RS)];
  }
}

template <int RS, int NY>
__global__ void __launch_bounds__(256) k_yfwd_r(YFwdArgs A, Geom G, WPlan plan) {
  static_assert(RS >= 2 && RS <= 4 && NY >= 256 && NY <= 1024, "residues and lengths");
  constexpr int N = RS * NY;
  constexpr int WL = NY + NY / 16 + 1;
  constexpr int T = N / 256;
  constexpr int TQ = NY / 256;
  using C = cpx<float>;
  extern __shared__ unsigned char smem[];
  C* buf = reinterpret_cast<C*>(smem);
  const C* tw = reinterpret_cast<const C*>(plan.tw);
  const int p = xcd_tile(blockIdx.x, gridDim.x);
  const YFwdJob& jb = A.job[blockIdx.y];
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const bool colp = p < G.nxh;
  const C* src = reinterpret_cast<const C*>(jb.src);
  C colv[T];
  EpiOps o[TQ];
  if (colp) {
#pragma unroll
    for (int t = 0; t < T; ++t) colv[t] = src[(size_t)(tid + 256 * t) * G.nxh + p];
#pragma unroll
    for (int k = 0; k < TQ; ++k) o[k] = yfwd_epi_load(jb, A.rk, (size_t)(tid + 256 * k) * G.nxh + p);
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int y = tid + 256 * t;
      buf[(y % RS) * WL + sk(y / RS)] = colv[t];
    }
  }
  __syncthreads();
  if (wave < RS) wave_fft_static<float, NY, RS, true>(buf + wave * WL, tw, -1, lane);
  __syncthreads();
  if (!colp) return;
  const double inv = 1.0 / (double)N;
#pragma unroll
  for (int k = 0; k < TQ; ++k) {
    const int q = tid + 256 * k;
    const int qs = signed_q(q, G.ny);
    cd v = mk(0.0, 0.0);
    if (2 * p != G.nx && !(G.ny > 1 && 2 * q == G.ny)) {
      const C w1 = tw[(qs + N) % N];  // e^{-2 pi i qs / N}
      C acc = buf[sk(q)], w = w1;
#pragma unroll
      for (int r = 1; r < RS; ++r) {
        acc = acc + cmul(buf[r * WL + sk(q)], w);
        w = cmul(w, w1);
      }
      v = mk((double)acc.x * inv, (double)acc.y * inv);
    }
    yfwd_epi_store(jb, A.rk, G, p, q, qs, v, o[k]);
  }
}

// The residue forms with a runtime plan of the mode count, for padded
// lengths N = RS ny whose ny is 2/3/5-smooth (up to 64 MAXE points) and
// whose N has no compile-time transform: wavefront r runs the ny-point
// transform with the plan `pny`, whose twiddles are every RS-th entry of the
// N-point table that also gives the modulations.  Same jobs, symbols and
// epilogues as k_yinv_r / k_yfwd_r.
template <int RS, int TQ, int MAXE>
__global__ void __launch_bounds__(256) k_yinv_rr(YInvArgs args, Geom G, WPlan plan, WPlan pny, int nrows, int row0) {
  static_assert(RS >= 2 && RS <= 4, "residues");
  using C = cpx<float>;
  extern __shared__ unsigned char smem[];
  C* buf = reinterpret_cast<C*>(smem);
  const C* tw = reinterpret_cast<const C*>(plan.tw);
  const int ny = G.ny, N = RS * ny, WL = wbuf_len(ny);
  const int p = xcd_tile(blockIdx.x, gridDim.x);
  const YInvJob& jb = args.job[blockIdx.y];
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int half = ny / 2;
  const bool col = p < G.nxh && 2 * p != G.nx;
  cd v[TQ];
#pragma unroll
  for (int t = 0; t < TQ; ++t) {
    const int q = tid + 256 * t;
    const int qs = q >= half ? q - ny : q;
    v[t] = mk(0.0, 0.0);
    if (col && q < ny && qs > -half) v[t] = jb.src[(size_t)q * G.nxh + p];
  }
#pragma unroll
  for (int t = 0; t < TQ; ++t) {
    const int q = tid + 256 * t;
    if (q >= ny) continue;
    const int qs = q >= half ? q - ny : q;
    C w = mk(0.f, 0.f);
    if (col && qs > -half) {
      const cd x = cmul(v[t], symbol_of(G, jb, p, qs));
      w = mk((float)x.x, (float)x.y);
    }
    const C tm = tw[(qs + N) % N];
    const C md = mk(tm.x, -tm.y);  // e^{2 pi i qs / N}
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      buf[r * WL + sk(q)] = w;
      w = cmul(w, md);
    }
  }
  __syncthreads();
  if (wave >= RS || p >= G.nxh) return;
  C* b = buf + wave * WL;
  wave_fft<float, MAXE>(b, pny, +1, lane, RS);
  C* dst = reinterpret_cast<C*>(jb.dst);
  const int r0 = ((wave - row0) % RS + RS) % RS;
  for (int rr = r0 + RS * lane; rr < nrows; rr += RS * 64) {
    int y = row0 + rr;
    if (y >= N) y -= N * (y / N);
    dst[(size_t)rr * G.nxh + p] = b[sk((y - wave) / RS)];
  }
}

template <int RS, int TQ, int MAXE>
__global__ void __launch_bounds__(256) k_yfwd_rr(YFwdArgs A, Geom G, WPlan plan, WPlan pny) {
  static_assert(RS >= 2 && RS <= 4, "residues");
  constexpr int T = RS * TQ;  // padded points per thread, at most
  using C = cpx<float>;
  extern __shared__ unsigned char smem[];
  C* buf = reinterpret_cast<C*>(smem);
  const C* tw = reinterpret_cast<const C*>(plan.tw);
  const int ny = G.ny, N = RS * ny, WL = wbuf_len(ny);
  const int p = xcd_tile(blockIdx.x, gridDim.x);
  const YFwdJob& jb = A.job[blockIdx.y];
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const bool colp = p < G.nxh;
  const C* src = reinterpret_cast<const C*>(jb.src);
  C colv[T];
  EpiOps o[TQ];
  if (colp) {
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int y = tid + 256 * t;
      if (y < N) colv[t] = src[(size_t)y * G.nxh + p];
    }
#pragma unroll
    for (int k = 0; k < TQ; ++k) {
      const int q = tid + 256 * k;
      if (q < ny) o[k] = yfwd_epi_load(jb, A.rk, (size_t)q * G.nxh + p);
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int y = tid + 256 * t;
      if (y < N) buf[(y % RS) * WL + sk(y / RS)] = colv[t];
    }
  }
  __syncthreads();
  if (wave < RS) wave_fft<float, MAXE>(buf + wave * WL, pny, -1, lane, RS);
  __syncthreads();
  if (!colp) return;
  const double inv = 1.0 / (double)N;
#pragma unroll
  for (int k = 0; k < TQ; ++k) {
    const int q = tid + 256 * k;
    if (q >= ny) continue;
    const int qs = signed_q(q, ny);
    cd v = mk(0.0, 0.0);
    if (2 * p != G.nx && !(ny > 1 && 2 * q == ny)) {
      const C w1 = tw[(qs + N) % N];  // e^{-2 pi i qs / N}
      C acc = buf[sk(q)], w = w1;
#pragma unroll
      for (int r = 1; r < RS; ++r) {
        acc = acc + cmul(buf[r * WL + sk(q)], w);
        w = cmul(w, w1);
      }
      v = mk((double)acc.x * inv, (double)acc.y * inv);
    }
    yfwd_epi_store(jb, A.rk, G, p, q, qs, v, o[k]);
  }
}

// Fused x pass, wavefront version: block = physical row y, four wavefronts.
// Field pairs are spread over the wavefronts (each transforms its pair in
// its own LDS buffer and leaves the two real rows in LDS); after one block
// barrier every thread forms the order-M products of its points in
// registers; wavefront 0 transforms the result forward.
template <typename R, int MAXE, int NS0>
__global__ void __launch_bounds__(256) k_xpass_w(XArgs A, Geom G, WPlan plan) {
  extern __shared__ unsigned char smem[];
  using C = cpx<R>;
  const int Px = plan.n;
  const int y = blockIdx.x;
  const int hx = G.nx / 2;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int wl = wbuf_len(Px);
  C* zbuf = reinterpret_cast<C*>(smem) + (size_t)wave * wl;
  R* phys = reinterpret_cast<R*>(reinterpret_cast<C*>(smem) + 4 * (size_t)wl);  // [nin][Px]
  const int npairs = (A.nin + 1) / 2;
  for (int pi = wave; pi < npairs; pi += 4) {
    const XIn& fa = A.in[2 * pi];
    const bool hasb = 2 * pi + 1 < A.nin;
    const XIn& fb = A.in[hasb ? 2 * pi + 1 : 2 * pi];
    for (int s = lane; s < Px; s += 64) {
      C z = mk((R)0, (R)0);
      int p = -1;
      bool cj = false;
      if (s < hx) p = s;
      else if (s > Px - hx) { p = Px - s; cj = true; }
      if (p >= 0) {
        C va = load_row<R>(fa, y, p, G);
        C vb = hasb ? load_row<R>(fb, y, p, G) : mk((R)0, (R)0);
        if (cj) { va = conjg(va); vb = conjg(vb); }
        z = mk(va.x - vb.y, va.y + vb.x);
      }
      zbuf[sk(s)] = z;
    }
    wave_sync();
    wave_fft_any<R, MAXE, NS0>(zbuf, plan, +1, lane);
    for (int x = lane; x < Px; x += 64) {
      const C zx = zbuf[sk(x)];
      phys[(size_t)(2 * pi) * Px + x] = zx.x;
      if (hasb) phys[(size_t)(2 * pi + 1) * Px + x] = zx.y;
    }
    wave_sync();
  }
  __syncthreads();
  const int M = A.M;
  C* zout = reinterpret_cast<C*>(smem);  // wavefront 0's buffer
  for (int x = threadIdx.x; x < Px; x += blockDim.x) {
    R eta = (R)0, ge2 = (R)0, dot = (R)0, gp2 = (R)0, etat = (R)0, phit = (R)0;
    R W[kMaxM];
#pragma unroll
    for (int m = 0; m < kMaxM; ++m) W[m] = (R)0;
    for (int i = 0; i < A.nin; ++i) {
      const XIn& f = A.in[i];
      const R v = phys[(size_t)i * Px + x];
      switch (f.role) {
        case XR_ETA: eta = v; break;
        case XR_GRADPAIR: {
          const R b = phys[(size_t)(i + 1) * Px + x];
          ge2 += v * v;
          dot += v * b;
          gp2 += b * b;
        } break;
        case XR_G: {
          R c = (R)1;
          for (int k = 1; k <= f.pw; ++k) c *= eta / (R)k;
#pragma unroll
          for (int m = 0; m < kMaxM; ++m)
            if (m == f.wi) W[m] += c * v;
        } break;
        case XR_ETAT: etat = v; break;
        case XR_PHIT: phit = v; break;
        default: break;
      }
    }
    R o0 = (R)0, o1 = (R)0;
    if (A.stage == XS_SERIES) {
      o0 = -W[0];
    } else if (A.stage == XS_FTILDE) {
      o0 = phit;
      if (M >= 2) o0 -= W[0] * etat;
    } else {
      R wm = (R)0, wm2 = (R)0;
#pragma unroll
      for (int m = 0; m < kMaxM; ++m) {
        if (m < M) wm += W[m];
        if (m < M - 2) wm2 += W[m];
      }
      o0 = wm - W[0];
      if (M >= 3) o0 += ge2 * wm2;
      if (M >= 2) o0 -= dot;
      o1 = (R)0.5 * w2sum(W, M);
      if (M >= 2) o1 -= (R)0.5 * gp2;
      if (M >= 4) o1 += (R)0.5 * ge2 * w2sum(W, M - 2);
    }
    zout[sk(x)] = mk(o0, o1);
  }
  __syncthreads();
  if (wave != 0) return;
  wave_fft_any<R, MAXE, NS0>(zout, plan, -1, lane);
  const R sc = (R)(0.5 / (double)Px);
  C* d0 = reinterpret_cast<C*>(A.out0);
  C* d1 = reinterpret_cast<C*>(A.out1);
  for (int p = lane; p < G.nxh; p += 64) {
    C o0 = mk((R)0, (R)0), o1 = mk((R)0, (R)0);
    if (p < hx) {
      C zp = zout[sk(p)];
      C zm = conjg(zout[sk((Px - p) % Px)]);
      C sum = zp + zm, t = zp - zm;
      o0 = cscale(sum, sc);
      o1 = mk(t.y * sc, -t.x * sc);
    }
    d0[(size_t)y * G.nxh + p] = o0;
    if (d1) d1[(size_t)y * G.nxh + p] = o1;
  }
}

// Fused x pass in rounds (power-of-two rows up to 1024 points): each round,
// the four wavefronts transform one input pair each in their own LDS buffer,
// and after a block barrier every thread folds the round's rows into the
// order-M products of its points, held in registers; the inputs are taken in
// index order as in the single-pass version, so the arithmetic (and the
// result) is the same, while LDS holds only the four transform buffers and
// several rows' blocks fit on a CU.  Requires every gradient-pair input at
// an even index (its partner in the same pair).
template <int MW, typename R>
__device__ __forceinline__ R w2sum_n(const R* W, int K) {
  R s = (R)0;
#pragma unroll
  for (int m = 2; m <= MW; ++m)
#pragma unroll
    for (int l = 1; l < m; ++l)
      if (m <= K) s += W[l - 1] * W[m - l - 1];
  return s;
}

template <typename R, int MAXE, int NS0, int MW>
__global__ void __launch_bounds__(256) k_xpass_r(XArgs A, Geom G, WPlan plan) {
  // Rows of 256, 512 or 1024 points: wavefront transforms of the inputs and a
  // four-wavefront transform of the products.  Rows of 3Q points (Q = 256,
  // 512, 1024): every transform as three Q-point ones and a radix-3 combine
  // (the inputs' by their wavefront, the products' by the workgroup).
  constexpr bool B3 = NS0 % 3 == 0;
  static_assert(B3 ? (NS0 / 3 >= 256 && NS0 / 3 <= 1024 && ((NS0 / 3) & (NS0 / 3 - 1)) == 0)
                   : (NS0 >= 256 && NS0 <= 1024 && NS0 % 256 == 0),
                "rows of 256, 512 or 1024 points, or three times that");
  constexpr int PPT = NS0 / 256;           // points per thread
  constexpr int KP = NS0 / 128;            // kept modes per lane (p < Px / 2)
  constexpr int Q4 = B3 ? 64 : NS0 / 4;    // sub-transform length of the four-wavefront transform
  constexpr int Q3 = B3 ? NS0 / 3 : 64;    // sub-transform length of the three-way transforms
  // rows read a round ahead where the registers allow (not at 3Q points:
  // the per-point products already take most of them)
  constexpr bool PREF = !B3;
  extern __shared__ unsigned char smem[];
  using C = cpx<R>;
  constexpr int Px = NS0;
  const C* twc = reinterpret_cast<const C*>(plan.tw);
  // LDS slot of input element s of an input transform, and of output element
  // x of that transform
  auto ipos = [](int s) { if constexpr (B3) return b3_in<Q3>(s); else return sk(s); };
  auto fpos = [](int x) { if constexpr (B3) return b3_out<Q3>(x); else return sk(x); };
  const int y = blockIdx.x;
  const int hx = G.nx / 2;
  // wave-uniform, so the input descriptors are read with scalar loads
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int wl = B3 ? b3_len<Q3>() : wbuf_len(Px);
  C* bufs = reinterpret_cast<C*>(smem);
  C* zbuf = bufs + (size_t)wave * wl;
  R eta[PPT], ge2[PPT], dot[PPT], gp2[PPT], etat[PPT], phit[PPT], W[PPT][MW];
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    eta[j] = ge2[j] = dot[j] = gp2[j] = etat[j] = phit[j] = (R)0;
#pragma unroll
    for (int m = 0; m < MW; ++m) W[j][m] = (R)0;
  }
  // role, power of eta and order of every input, read once from the
  // arguments into LDS (visible after the first round's barrier): the fold
  // then takes them from LDS instead of a chain of dependent argument loads
  __shared__ int s_code[kMaxXIn];
  if ((int)threadIdx.x < A.nin) {
    const XIn& f = A.in[threadIdx.x];
    s_code[threadIdx.x] = f.role | (f.pw << 8) | (f.wi << 16);
  }
  const int npairs = (A.nin + 1) / 2;
  const int nrounds = (npairs + 3) / 4;
  // Rows of this wavefront's input pair, read a round ahead: the loads of
  // round rd + 1 are in flight during round rd's transform.  Mode p
  // (0 <= p < hx) goes to slot p and its conjugate image to slot Px - p; the
  // slots in between stay zero (padding).
  C va[PREF ? KP : 1], vb[PREF ? KP : 1];
  auto load_pair = [&](int pi) {
    if constexpr (!PREF) return;
    const bool hasb = 2 * pi + 1 < A.nin;
    const C* ra = reinterpret_cast<const C*>(A.in[2 * pi].src) + (size_t)y * G.nxh;
    const C* rb = reinterpret_cast<const C*>(A.in[hasb ? 2 * pi + 1 : 2 * pi].src) + (size_t)y * G.nxh;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int p = lane + 64 * k;
      va[k] = vb[k] = mk((R)0, (R)0);
      if (p < hx) {
        va[k] = ra[p];
        if (hasb) vb[k] = rb[p];
      }
    }
  };
  if (PREF && wave < npairs) load_pair(wave);
  for (int rd = 0; rd < nrounds; ++rd) {
    const int pi = 4 * rd + wave;
    if (pi < npairs) {
      const XIn fa = A.in[2 * pi];
      const bool hasb = 2 * pi + 1 < A.nin;
      const XIn fb = A.in[hasb ? 2 * pi + 1 : 2 * pi];
#pragma unroll
      for (int j = 0; j < Px / 64; ++j) {
        const int s = lane + 64 * j;
        if (s >= hx && s <= Px - hx) zbuf[ipos(s)] = mk((R)0, (R)0);
      }
      if constexpr (PREF) {
#pragma unroll
        for (int k = 0; k < KP; ++k) {
          const int p = lane + 64 * k;
          if (p < hx) {
            C a = va[k], b = vb[k];
            if (fa.dx) a = times_ikx<R>(a, p, G);
            if (hasb && fb.dx) b = times_ikx<R>(b, p, G);
            zbuf[ipos(p)] = mk(a.x - b.y, a.y + b.x);                 // a + i b
            if (p > 0) zbuf[ipos(Px - p)] = mk(a.x + b.y, b.x - a.y);  // conj(a) + i conj(b)
          }
        }
        if (pi + 4 < npairs) load_pair(pi + 4);
      } else {
        // read straight into LDS, four modes per lane at a time
        const C* ra = reinterpret_cast<const C*>(fa.src) + (size_t)y * G.nxh;
        const C* rb = reinterpret_cast<const C*>(fb.src) + (size_t)y * G.nxh;
#pragma unroll
        for (int k0 = 0; k0 < KP; k0 += 4) {
          C a4[4], b4[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int p = lane + 64 * (k0 + k);
            a4[k] = b4[k] = mk((R)0, (R)0);
            if (p < hx) {
              a4[k] = ra[p];
              if (hasb) b4[k] = rb[p];
            }
          }
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int p = lane + 64 * (k0 + k);
            if (p < hx) {
              C a = a4[k], b = b4[k];
              if (fa.dx) a = times_ikx<R>(a, p, G);
              if (hasb && fb.dx) b = times_ikx<R>(b, p, G);
              zbuf[ipos(p)] = mk(a.x - b.y, a.y + b.x);
              if (p > 0) zbuf[ipos(Px - p)] = mk(a.x + b.y, b.x - a.y);
            }
          }
        }
      }
      wave_sync();
      if constexpr (B3) wave_fft3<R, Q3>(zbuf, twc, +1, lane);
      else wave_fft_any<R, MAXE, NS0>(zbuf, plan, +1, lane);
    }
    __syncthreads();
    const int i1 = min(A.nin, 8 * (rd + 1));
    for (int i = 8 * rd; i < i1; ++i) {
      const int code = __builtin_amdgcn_readfirstlane(s_code[i]);
      const int role = code & 255, pw = (code >> 8) & 255, wi = code >> 16;
      const C* zb = bufs + (size_t)((i >> 1) - 4 * rd) * wl;
      const bool hi = i & 1;
      R c[PPT];
      if (role == XR_G) {
        // eta^pw / pw! (pw <= M <= MW); unrolled, so the divisions by 1, 2
        // and 4 become exact multiplications
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
          c[j] = (R)1;
#pragma unroll
          for (int k = 1; k <= MW; ++k)
            if (k <= pw) c[j] *= eta[j] / (R)k;
        }
      }
      // the row values at this thread's points (Px = 256 PPT), all read first
      C zv[PPT];
#pragma unroll
      for (int j = 0; j < PPT; ++j) zv[j] = zb[fpos(threadIdx.x + 256 * j)];
#pragma unroll
      for (int j = 0; j < PPT; ++j) {
        const C zx = zv[j];
        const R v = hi ? zx.y : zx.x;
        switch (role) {
          case XR_ETA: eta[j] = v; break;
          case XR_GRADPAIR: {
            const R b = zx.y;
            ge2[j] += v * v;
            dot[j] += v * b;
            gp2[j] += b * b;
          } break;
          case XR_G:
#pragma unroll
            for (int m = 0; m < MW; ++m)
              if (m == wi) W[j][m] += c[j] * v;
            break;
          case XR_ETAT: etat[j] = v; break;
          case XR_PHIT: phit[j] = v; break;
          default: break;
        }
      }
    }
    __syncthreads();
  }
  const int M = A.M;
  C* zout = bufs;  // wavefront 0's buffer
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const int x = threadIdx.x + 256 * j;
    if (x >= Px) break;
    R o0 = (R)0, o1 = (R)0;
    if (A.stage == XS_SERIES) {
      o0 = -W[j][0];
    } else if (A.stage == XS_FTILDE) {
      o0 = phit[j];
      if (M >= 2) o0 -= W[j][0] * etat[j];
    } else {
      R wm = (R)0, wm2 = (R)0;
#pragma unroll
      for (int m = 0; m < MW; ++m) {
        if (m < M) wm += W[j][m];
        if (m < M - 2) wm2 += W[j][m];
      }
      o0 = wm - W[j][0];
      if (M >= 3) o0 += ge2[j] * wm2;
      if (M >= 2) o0 -= dot[j];
      o1 = (R)0.5 * w2sum_n<MW>(W[j], M);
      if (M >= 2) o1 -= (R)0.5 * gp2[j];
      if (M >= 4) o1 += (R)0.5 * ge2[j] * w2sum_n<MW>(W[j], M - 2);
    }
    if constexpr (B3) zout[b3_in<Q3>(x)] = mk(o0, o1);
    else zout[b4_in<Q4>(x)] = mk(o0, o1);
  }
  // forward transform of the products by the workgroup
  if constexpr (B3) block3_fft<R, Q3>(zout, twc, -1);
  else block4_fft<R, NS0>(zout, twc, -1);
  auto opos = [](int k) { if constexpr (B3) return b3_out<Q3>(k); else return b4_out<Q4>(k); };
  const R sc = (R)(0.5 / (double)Px);
  C* d0 = reinterpret_cast<C*>(A.out0);
  C* d1 = reinterpret_cast<C*>(A.out1);
  for (int p = threadIdx.x; p < G.nxh; p += 256) {
    C o0 = mk((R)0, (R)0), o1 = mk((R)0, (R)0);
    if (p < hx) {
      C zp = zout[opos(p)];
      C zm = conjg(zout[opos((Px - p) % Px)]);
      C sum = zp + zm, t = zp - zm;
      o0 = cscale(sum, sc);
      o1 = mk(t.y * sc, -t.x * sc);
    }
    d0[(size_t)y * G.nxh + p] = o0;
    if (d1) d1[(size_t)y * G.nxh + p] = o1;
  }
}

// Rows of 3Q points transformed by the whole workgroup (the three
// sub-transforms on wavefronts 0-2, the radix-3 combine on every thread) in a
// single LDS buffer: an input pair (a, b) is transformed as a + i b, so that
// the real part of the result is a's row and the imaginary part b's.  The
// kept modes of the next pair are read into registers while the current pair
// is transformed (the block barriers of the transform wait on LDS operations
// only, so the loads stay in flight).
template <typename R, int Q, int NT, bool RES = false>
struct Rows3 {
  static constexpr int Px = 3 * Q;
  static constexpr int PPT = Px / NT;  // points per thread
  // kept modes per thread: p < Px / 2, or with RES (nx = Q) p < Q / 2
  static constexpr int KP = ((RES ? Q : Px) / 2 + NT - 1) / NT;
  cpx<R> va[KP], vb[KP];

  __device__ __forceinline__ void load(const XArgs& A, const Geom& G, int y, int ia, int ib) {
    const int hx = G.nx / 2;
    const cpx<R>* ra = reinterpret_cast<const cpx<R>*>(A.in[ia].src) + (size_t)y * G.nxh;
    const cpx<R>* rb = reinterpret_cast<const cpx<R>*>(A.in[ib < 0 ? ia : ib].src) + (size_t)y * G.nxh;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int p = (int)threadIdx.x + NT * k;
      va[k] = vb[k] = mk((R)0, (R)0);
      if (p < hx) {
        va[k] = ra[p];
        if (ib >= 0) vb[k] = rb[p];
      }
    }
  }

  // Writes the held pair into buf (the caller has passed a barrier since
  // buf was last read).  Without RES: the zero-padded Px-point sequence in
  // the decimated input layout of block3_fft.  With RES: the three residue
  // sequences, mode p of sub-buffer r times e^{2 pi i p r / Px} (tw holds
  // e^{-2 pi i m / Px}), so that sub-buffer r's Q-point inverse transform is
  // the row at the points x = 3 s + r.
  __device__ __forceinline__ void store(cpx<R>* buf, const cpx<R>* __restrict__ tw, const XArgs& A, const Geom& G,
                                        int ia, int ib) const {
    const int hx = G.nx / 2;
    const int dxa = A.in[ia].dx, dxb = ib >= 0 ? A.in[ib].dx : 0;
    if constexpr (RES) {
      constexpr int WL = b3_stride<Q>();
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        const int p = (int)threadIdx.x + NT * k;
        if (p < Q / 2) {
          cpx<R> a = va[k], b = vb[k];
          if (dxa) a = times_ikx<R>(a, p, G);
          if (dxb) b = times_ikx<R>(b, p, G);
          const cpx<R> zp = mk(a.x - b.y, a.y + b.x), zm = mk(a.x + b.y, b.x - a.y);
          const cpx<R> w1 = conjg(tw[p]), w2 = conjg(tw[2 * p]);
          buf[sk(p)] = zp;
          buf[WL + sk(p)] = cmul(zp, w1);
          buf[2 * WL + sk(p)] = cmul(zp, w2);
          if (p > 0) {
            buf[sk(Q - p)] = zm;
            buf[WL + sk(Q - p)] = cmul(zm, conjg(w1));
            buf[2 * WL + sk(Q - p)] = cmul(zm, conjg(w2));
          } else {
#pragma unroll
            for (int r = 0; r < 3; ++r) buf[r * WL + sk(Q / 2)] = mk((R)0, (R)0);  // the Nyquist slot
          }
        }
      }
      return;
    }
#pragma unroll
    for (int t = 0; t < PPT; ++t) {
      const int s = (int)threadIdx.x + NT * t;
      if (s >= hx && s <= Px - hx) buf[b3_in<Q>(s)] = mk((R)0, (R)0);
    }
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int p = (int)threadIdx.x + NT * k;
      if (p < hx) {
        cpx<R> a = va[k], b = vb[k];
        if (dxa) a = times_ikx<R>(a, p, G);
        if (dxb) b = times_ikx<R>(b, p, G);
        buf[b3_in<Q>(p)] = mk(a.x - b.y, a.y + b.x);                 // a + i b
        if (p > 0) buf[b3_in<Q>(Px - p)] = mk(a.x + b.y, b.x - a.y);  // conj(a) + i conj(b)
      }
    }
  }
};

// Inverse transform of the stored pair: physical point x then sits at
// b3_out(x) (block3_fft), or with RES at b3_in(x) (one residue per
// wavefront, no combine).
template <typename R, int Q, int NT, bool HT, bool RES>
__device__ __forceinline__ void rows3_inv(cpx<R>* buf, const cpx<R>* __restrict__ tw) {
  if constexpr (RES) {
    constexpr int WL = b3_stride<Q>();
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lane = threadIdx.x & 63;
    __syncthreads();
    if (wave < 3) wave_fft_static<R, Q, 3, HT>(buf + wave * WL, tw, +1, lane);
    __syncthreads();
  } else {
    block3_fft<R, Q, NT, HT>(buf, tw, +1);
  }
}

template <int Q, bool RES>
__device__ __forceinline__ int rows3_pt(int x) { return RES ? b3_in<Q>(x) : b3_out<Q>(x); }

// Forward transform of the per-point results already in buf (real part o0,
// imaginary part o1) and the kept modes of the two real rows to out0/out1.
template <typename R, int Q, int NT, bool HT = true, bool RES = false>
__device__ __forceinline__ void rows3_out(cpx<R>* buf, const cpx<R>* tw, const XArgs& A, const Geom& G, int y) {
  constexpr int Px = 3 * Q;
  constexpr int WL = b3_stride<Q>();
  const int hx = G.nx / 2;
  const R sc = (R)(0.5 / (double)Px);
  cpx<R>* d0 = reinterpret_cast<cpx<R>*>(A.out0);
  cpx<R>* d1 = reinterpret_cast<cpx<R>*>(A.out1);
  if constexpr (RES) {
    // the three residue sequences' forward transforms, then only the kept
    // modes p and Px - p (p < hx) combined: Y[k] = sum_r e^{-2 pi i k r / Px} Z_r[k mod Q]
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lane = threadIdx.x & 63;
    __syncthreads();
    if (wave < 3) wave_fft_static<R, Q, 3, HT>(buf + wave * WL, tw, -1, lane);
    __syncthreads();
    for (int p = threadIdx.x; p < G.nxh; p += NT) {
      cpx<R> o0 = mk((R)0, (R)0), o1 = mk((R)0, (R)0);
      if (p < hx) {
        const cpx<R> w1 = tw[p], w2 = tw[2 * p];
        const int q = p == 0 ? 0 : Q - p;
        const cpx<R> zp = buf[sk(p)] + cmul(buf[WL + sk(p)], w1) + cmul(buf[2 * WL + sk(p)], w2);
        const cpx<R> ym = buf[sk(q)] + cmul(buf[WL + sk(q)], conjg(w1)) + cmul(buf[2 * WL + sk(q)], conjg(w2));
        const cpx<R> zm = conjg(ym);
        const cpx<R> sum = zp + zm, t = zp - zm;
        o0 = cscale(sum, sc);
        o1 = mk(t.y * sc, -t.x * sc);
      }
      d0[(size_t)y * G.nxh + p] = o0;
      if (d1) d1[(size_t)y * G.nxh + p] = o1;
    }
    return;
  }
  block3_fft<R, Q, NT, HT>(buf, tw, -1);
  for (int p = threadIdx.x; p < G.nxh; p += NT) {
    cpx<R> o0 = mk((R)0, (R)0), o1 = mk((R)0, (R)0);
    if (p < hx) {
      cpx<R> zp = buf[b3_out<Q>(p)];
      cpx<R> zm = conjg(buf[b3_out<Q>((Px - p) % Px)]);
      cpx<R> sum = zp + zm, t = zp - zm;
      o0 = cscale(sum, sc);
      o1 = mk(t.y * sc, -t.x * sc);
    }
    d0[(size_t)y * G.nxh + p] = o0;
    if (d1) d1[(size_t)y * G.nxh + p] = o1;
  }
}

// Series stages of the x pass on rows of 3Q points: the product
// -sum_j eta^j / j! g_j of one order, or (FT) the product
// phis_t - [M >= 2] eta_t sum_j eta^j / j! g_j that the time derivative of
// the mean-level modes takes.  Per point only eta, the running sum and (FT)
// eta_t and phis_t are held; the inputs are folded in index order with the
// arithmetic of the rounds kernel.
template <typename R, int Q, int NT, bool FT, bool RES>
__global__ void __launch_bounds__(NT) k_xpass_series3(XArgs A, Geom G, WPlan plan) {
  using Rw = Rows3<R, Q, NT, RES>;
  // twiddles read ahead at 3072 points (measured faster); not with the extra
  // per-point state of FT, which leaves no registers for them
  constexpr bool HT = Q >= 1024 && !FT;
  constexpr int PPT = Rw::PPT;
  extern __shared__ unsigned char smem[];
  using C = cpx<R>;
  C* buf = reinterpret_cast<C*>(smem);
  const C* tw = reinterpret_cast<const C*>(plan.tw);
  const int y = blockIdx.x;
  const int tid = threadIdx.x;
  __shared__ int s_code[kMaxXIn];
  if (tid < A.nin) {
    const XIn& f = A.in[tid];
    s_code[tid] = f.role | (f.pw << 8);
  }
  R eta[PPT], w0[PPT], et[FT ? PPT : 1], pt[FT ? PPT : 1];
#pragma unroll
  for (int j = 0; j < PPT; ++j) eta[j] = w0[j] = (R)0;
#pragma unroll
  for (int j = 0; j < (FT ? PPT : 1); ++j) et[j] = pt[j] = (R)0;
  const int npairs = (A.nin + 1) / 2;
  Rw rows;
  rows.load(A, G, y, 0, 1 < A.nin ? 1 : -1);
  for (int pi = 0; pi < npairs; ++pi) {
    const int ib = 2 * pi + 1 < A.nin ? 2 * pi + 1 : -1;
    rows.store(buf, tw, A, G, 2 * pi, ib);
    if (pi + 1 < npairs) rows.load(A, G, y, 2 * pi + 2, 2 * pi + 3 < A.nin ? 2 * pi + 3 : -1);
    rows3_inv<R, Q, NT, HT, RES>(buf, tw);
    const int i1 = min(A.nin, 2 * pi + 2);
    for (int i = 2 * pi; i < i1; ++i) {
      const int code = s_code[i];
      const int role = code & 255, pw = (code >> 8) & 255;
      const bool hi = i & 1;
#pragma unroll
      for (int j = 0; j < PPT; ++j) {
        const C zx = buf[rows3_pt<Q, RES>(tid + NT * j)];
        const R v = hi ? zx.y : zx.x;
        if (role == XR_ETA) {
          eta[j] = v;
        } else if (role == XR_G) {
          R c = (R)1;
#pragma unroll
          for (int k = 1; k <= kMaxM; ++k)
            if (k <= pw) c *= eta[j] / (R)k;
          w0[j] += c * v;
        } else if (FT && role == XR_ETAT) {
          et[j] = v;
        } else if (FT && role == XR_PHIT) {
          pt[j] = v;
        }
      }
    }
    __syncthreads();  // the buffer is refilled by the next pair
  }
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    R o = -w0[j];
    if constexpr (FT) {
      o = pt[j];
      if (A.M >= 2) o -= w0[j] * et[j];
    }
    buf[b3_in<Q>(tid + NT * j)] = mk(o, (R)0);
  }
  rows3_out<R, Q, NT, HT, RES>(buf, tw, A, G, y);
}

// Final stage of the x pass on rows of 3Q points, in the same form.  In the
// residue layout (nx = Q: two kept modes per thread instead of six) the next
// pair is read ahead and every transform reads its twiddles ahead; in the
// decimated layout each pair's rows are read just before they are stored and
// only the lighter phases read twiddles ahead (the registers go to the
// per-point state).  The host orders the inputs as eta
// and the W terms first (A.ng of them), then the gradient pairs (each
// XR_GRADPAIR followed by its partner).  Phase one
// holds eta and W_1 .. W_M (M <= MW) per point; once the W are complete they
// are folded into the two outputs and the two multipliers of |grad eta|^2,
// so that phase two adds each gradient pair straight into the outputs:
// o0 = sum_{m>1} W_m + |grad eta|^2 sum_{m<=M-2} W_m - grad eta . grad phi,
// o1 = [W^2]_M / 2 - |grad phi|^2 / 2 + |grad eta|^2 [W^2]_{M-2} / 2
// (the order-M truncation of the rounds kernel, |grad eta|^2 and the dot
// product summed per gradient direction).
template <typename R, int Q, int MW, int NT, bool RES>
__global__ void __launch_bounds__(NT, 2) k_xpass_final3(XArgs A, Geom G, WPlan plan) {
  using Rw = Rows3<R, Q, NT, RES>;
  constexpr int PPT = Rw::PPT;
  extern __shared__ unsigned char smem[];
  using C = cpx<R>;
  C* buf = reinterpret_cast<C*>(smem);
  const C* tw = reinterpret_cast<const C*>(plan.tw);
  const int y = blockIdx.x;
  const int tid = threadIdx.x;
  const int M = A.M, ng = A.ng;
  __shared__ int s_code[kMaxXIn];
  if (tid < A.nin) {
    const XIn& f = A.in[tid];
    s_code[tid] = f.role | (f.pw << 8) | (f.wi << 16);
  }
  R o0[PPT], o1[PPT], c2[PPT], s2[PPT];
  Rw rows;
  if constexpr (RES) rows.load(A, G, y, 0, 1 < ng ? 1 : -1);
  {
    R eta[PPT], W[PPT][MW];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      eta[j] = (R)0;
#pragma unroll
      for (int m = 0; m < MW; ++m) W[j][m] = (R)0;
    }
    const int np1 = (ng + 1) / 2;
    for (int pi = 0; pi < np1; ++pi) {
      if constexpr (!RES) rows.load(A, G, y, 2 * pi, 2 * pi + 1 < ng ? 2 * pi + 1 : -1);
      rows.store(buf, tw, A, G, 2 * pi, 2 * pi + 1 < ng ? 2 * pi + 1 : -1);
      if constexpr (RES) {
        if (pi + 1 < np1) rows.load(A, G, y, 2 * pi + 2, 2 * pi + 3 < ng ? 2 * pi + 3 : -1);
        else if (ng < A.nin) rows.load(A, G, y, ng, ng + 1);
      }
      rows3_inv<R, Q, NT, RES, RES>(buf, tw);
      const int i1 = min(ng, 2 * pi + 2);
      for (int i = 2 * pi; i < i1; ++i) {
        const int code = s_code[i];
        const int role = code & 255, pw = (code >> 8) & 255, wi = code >> 16;
        const bool hi = i & 1;
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
          const C zx = buf[rows3_pt<Q, RES>(tid + NT * j)];
          const R v = hi ? zx.y : zx.x;
          if (role == XR_ETA) {
            eta[j] = v;
          } else if (role == XR_G) {
            R c = (R)1;
#pragma unroll
            for (int k = 1; k <= MW; ++k)
              if (k <= pw) c *= eta[j] / (R)k;
#pragma unroll
            for (int m = 0; m < MW; ++m)
              if (m == wi) W[j][m] += c * v;
          }
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      R wm = (R)0, wm2 = (R)0;
#pragma unroll
      for (int m = 0; m < MW; ++m) {
        if (m < M) wm += W[j][m];
        if (m < M - 2) wm2 += W[j][m];
      }
      o0[j] = wm - W[j][0];
      o1[j] = (R)0.5 * w2sum_n<MW>(W[j], M);
      c2[j] = M >= 3 ? wm2 : (R)0;
      s2[j] = M >= 4 ? (R)0.5 * w2sum_n<MW>(W[j], M - 2) : (R)0;
    }
  }
  // phase two and the output transform hold less per point: their passes
  // read the twiddles ahead of the LDS loads
  const R dm = M >= 2 ? (R)1 : (R)0;
  for (int i = ng; i < A.nin; i += 2) {
    if constexpr (!RES) rows.load(A, G, y, i, i + 1);
    rows.store(buf, tw, A, G, i, i + 1);
    if constexpr (RES)
      if (i + 2 < A.nin) rows.load(A, G, y, i + 2, i + 3);
    rows3_inv<R, Q, NT, true, RES>(buf, tw);
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const C zx = buf[rows3_pt<Q, RES>(tid + NT * j)];
      const R ge = zx.x * zx.x;
      o0[j] += ge * c2[j] - dm * (zx.x * zx.y);
      o1[j] += ge * s2[j] - dm * (R)0.5 * (zx.y * zx.y);
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < PPT; ++j) buf[b3_in<Q>(tid + NT * j)] = mk(o0[j], o1[j]);
  rows3_out<R, Q, NT, true, RES>(buf, tw, A, G, y);
}

// Physical rows <-> spectra on the mode grid (FP64, state in/out only).
__global__ void __launch_bounds__(256) k_phys_out(const cd* e_rows, const cd* p_rows, double* out_e, double* out_p,
                                                  Geom G, FftPlan plan) {
  extern __shared__ unsigned char smem[];
  const int Px = plan.n, y = blockIdx.x, hx = G.nx / 2;
  cd* za = reinterpret_cast<cd*>(smem);
  cd* zb = za + Px;
  for (int s = threadIdx.x; s < Px; s += blockDim.x) {
    cd z = mk(0.0, 0.0);
    int p = -1;
    bool cj = false;
    if (s < hx) p = s;
    else if (s > Px - hx) { p = Px - s; cj = true; }
    if (p >= 0) {
      cd va = e_rows[(size_t)y * G.nxh + p], vb = p_rows[(size_t)y * G.nxh + p];
      if (cj) { va = conjg(va); vb = conjg(vb); }
      z = mk(va.x - vb.y, va.y + vb.x);
    }
    za[s] = z;
  }
  __syncthreads();
  cd* res = block_fft<double>(za, zb, plan, 1, +1);
  for (int x = threadIdx.x; x < Px; x += blockDim.x) {
    out_e[(size_t)y * Px + x] = res[x].x;
    out_p[(size_t)y * Px + x] = res[x].y;
  }
}

__global__ void __launch_bounds__(256) k_phys_in(const double* in_e, const double* in_p, cd* e_rows, cd* p_rows,
                                                 Geom G, FftPlan plan) {
  extern __shared__ unsigned char smem[];
  const int Px = plan.n, y = blockIdx.x, hx = G.nx / 2;
  cd* za = reinterpret_cast<cd*>(smem);
  cd* zb = za + Px;
  for (int x = threadIdx.x; x < Px; x += blockDim.x)
    za[x] = mk(in_e[(size_t)y * Px + x], in_p[(size_t)y * Px + x]);
  __syncthreads();
  cd* res = block_fft<double>(za, zb, plan, 1, -1);
  const double sc = 0.5 / (double)Px;
  for (int p = threadIdx.x; p < G.nxh; p += blockDim.x) {
    cd o0 = mk(0.0, 0.0), o1 = mk(0.0, 0.0);
    if (p < hx) {
      cd zp = res[p], zm = conjg(res[(Px - p) % Px]);
      cd s = zp + zm, t = zp - zm;
      o0 = cscale(s, sc);
      o1 = mk(t.y * sc, -t.x * sc);
    }
    e_rows[(size_t)y * G.nxh + p] = o0;
    p_rows[(size_t)y * G.nxh + p] = o1;
  }
}

// Exact linear propagator over t of mode (a, b) = (eta, phis) with wavenumber k.
__device__ __forceinline__ void lin_prop(const Geom& G, double k, double t, cd& a, cd& b) {
  if (k == 0.0) {
    b = b - cscale(a, G.g * t);
    return;
  }
  const double kt = G.depth > 0.0 ? k * tanh(k * G.depth) : k;
  const double w = sqrt(G.g * kt);
  const double c = cos(w * t), s = sin(w * t);
  const cd na = cscale(a, c) + cscale(b, kt * s / w);
  const cd nb = cscale(b, c) - cscale(a, G.g * s / w);
  a = na;
  b = nb;
}

// Integrating-factor (Lawson) RK4 stage update per mode, E_t the exact
// linear propagator, k the nonlinear part at the stage input:
//   1: acc = E_h k1,        next = E_h/2 (x + h/2 k1)
//   2: acc += 2 E_h/2 k2,   next = E_h/2 x + h/2 k2
//   3: acc += 2 E_h/2 k3,   next = E_h x + h E_h/2 k3
//   4: x = E_h x + h/6 (acc + k4)
__global__ void k_ifrk4(int stage, cd* __restrict__ x0, cd* __restrict__ x1, const cd* __restrict__ k0,
                        const cd* __restrict__ k1, cd* __restrict__ a0, cd* __restrict__ a1, cd* __restrict__ s0,
                        cd* __restrict__ s1, Geom G, double hh) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)G.ny * G.nxh) return;
  const int q = (int)(i / G.nxh), p = (int)(i % G.nxh);
  const double kx = 2.0 * M_PI * (double)p / G.lx;
  const double ky = G.ny > 1 ? 2.0 * M_PI * (double)signed_q(q, G.ny) / G.ly : 0.0;
  const double k = sqrt(kx * kx + ky * ky);
  const cd ke = k0[i], kp = k1[i];
  const cd xe = x0[i], xp = x1[i];
  if (stage == 1) {
    cd ae = ke, ap = kp;
    lin_prop(G, k, hh, ae, ap);
    a0[i] = ae;
    a1[i] = ap;
    cd se = xe + cscale(ke, 0.5 * hh), sp = xp + cscale(kp, 0.5 * hh);
    lin_prop(G, k, 0.5 * hh, se, sp);
    s0[i] = se;
    s1[i] = sp;
  } else if (stage == 2 || stage == 3) {
    cd he = ke, hp = kp;
    lin_prop(G, k, 0.5 * hh, he, hp);
    a0[i] = a0[i] + cscale(he, 2.0);
    a1[i] = a1[i] + cscale(hp, 2.0);
    cd se = xe, sp = xp;
    if (stage == 2) {
      lin_prop(G, k, 0.5 * hh, se, sp);
      se = se + cscale(ke, 0.5 * hh);
      sp = sp + cscale(kp, 0.5 * hh);
    } else {
      lin_prop(G, k, hh, se, sp);
      se = se + cscale(he, hh);
      sp = sp + cscale(hp, hh);
    }
    s0[i] = se;
    s1[i] = sp;
  } else {
    cd ne = xe, np = xp;
    lin_prop(G, k, hh, ne, np);
    x0[i] = ne + cscale(a0[i] + ke, hh / 6.0);
    x1[i] = np + cscale(a1[i] + kp, hh / 6.0);
  }
}

// First RK4 stage from a right-hand side already evaluated at the state
// (the same k the stage would compute): acc = k, sout = xn + dt/2 k.
__global__ void k_rk_first(const cd* __restrict__ k0, const cd* __restrict__ k1, const cd* __restrict__ x0,
                           const cd* __restrict__ x1, cd* __restrict__ a0, cd* __restrict__ a1, cd* __restrict__ s0,
                           cd* __restrict__ s1, double dt, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const cd ka = k0[i], kb = k1[i];
  a0[i] = ka;
  a1[i] = kb;
  s0[i] = x0[i] + cscale(ka, 0.5 * dt);
  s1[i] = x1[i] + cscale(kb, 0.5 * dt);
}

__global__ void k_copy_cd(const cd* __restrict__ src, cd* __restrict__ dst, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void k_finite(const cd* a, const cd* b, size_t n, int* bad) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    if (!isfinite(a[i].x) || !isfinite(a[i].y) || !isfinite(b[i].x) || !isfinite(b[i].y)) atomicOr(bad, 1);
  }
}

// ------------------------------------------------------------------ host
int choose_tw(int Ly, size_t csize) {
  long cap = 65536 / (2L * Ly * (long)csize);
  int tw = 1;
  while (tw * 2 <= cap && tw * 2 <= 256) tw *= 2;
  return tw;
}

template <typename R>
void set_lds_limit(const void* fn, size_t bytes) {
  if (bytes > 65536) SW_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

template <typename R>
bool wave_ok(int n) {
  return n <= (sizeof(R) == 4 ? 4096 : 2048);
}

#define SW_MAXE_DISPATCH(n, LAUNCH) \
  switch (wave_maxe(n)) {           \
    case 8: LAUNCH(8); break;       \
    case 16: LAUNCH(16); break;     \
    case 32: LAUNCH(32); break;     \
    case 48: LAUNCH(48); break;     \
    default: LAUNCH(64); break;     \
  }

template <typename R>
void yinv_t(swense_hos* h, const YInvArgs& a, const FftPlan& plan, int nrows, int row0, hipStream_t st) {
  if (a.njobs == 0) return;
  if (h->prof.on) {
    // each distinct FP64 source spectrum read once, each job's rows written once
    const double spec = (double)h->G.ny * h->G.nxh * sizeof(cd);
    double b = (double)a.njobs * nrows * h->G.nxh * sizeof(cpx<R>);
    for (int j = 0; j < a.njobs; ++j) {
      bool seen = false;
      for (int i = 0; i < j; ++i) seen = seen || a.job[i].src == a.job[j].src;
      if (!seen) b += spec;
    }
    h->prof.bytes[SWENSE_K_YINV] += b;
    h->prof.tbytes[SWENSE_K_YINV] += (double)a.njobs * 2.0 * sizeof(R) * (double)h->Px * h->Py;
  }
  if constexpr (sizeof(R) == 4) {
    const int ny = h->G.ny, rs = plan.n / std::max(ny, 1);
    if ((ny == 256 || ny == 512 || ny == 1024) && rs >= 2 && rs <= 4 && rs * ny == plan.n) {
      // residue form: one wavefront per output residue
      const WPlan wp = make_wplan(plan);
      const size_t lds = (size_t)rs * (ny + ny / 16 + 1) * sizeof(cpx<R>);
      dim3 grid(h->G.nxh, a.njobs);
#define L_YIR(RS, NY) sw_launch(h, SWENSE_K_YINV, &k_yinv_r<RS, NY>, grid, dim3(256), lds, st, a, h->G, wp, nrows, row0)
#define L_YIRN(RS)                  \
  switch (ny) {                     \
    case 256: L_YIR(RS, 256); break;  \
    case 512: L_YIR(RS, 512); break;  \
    default: L_YIR(RS, 1024); break;  \
  }
      switch (rs) {
        case 2: L_YIRN(2); break;
        case 3: L_YIRN(3); break;
        default: L_YIRN(4); break;
      }
#undef L_YIRN
#undef L_YIR
      return;
    }
    if (ny >= 16 && ny <= 512 && ny % 2 == 0 && rs >= 2 && rs <= 4 && rs * ny == plan.n && !grp_len_ok(plan.n)) {
      // residue form with a runtime plan of the mode count (twiddles from the padded table)
      const WPlan wp = make_wplan(plan);
      FftPlan sub{};
      sub.n = ny;
      sub.tw = plan.tw;
      const WPlan pny = make_wplan(sub);
      const size_t lds = (size_t)rs * wbuf_len(ny) * sizeof(cpx<R>);
      dim3 grid(h->G.nxh, a.njobs);
#define L_YIRR(RS, TQ) sw_launch(h, SWENSE_K_YINV, &k_yinv_rr<RS, TQ, 8>, grid, dim3(256), lds, st, a, h->G, wp, pny, nrows, row0)
#define L_YIRRN(RS)              \
  if (ny <= 256) L_YIRR(RS, 1); \
  else L_YIRR(RS, 2);
      switch (rs) {
        case 2: L_YIRRN(2); break;
        case 3: L_YIRRN(3); break;
        default: L_YIRRN(4); break;
      }
#undef L_YIRRN
#undef L_YIRR
      return;
    }
  }
  if (grp_len_ok(plan.n) && h->G.ny > 1 && plan.n >= h->G.ny) {
    const WPlan wp = make_wplan(plan);
    const size_t lds = grp_lds_len(plan.n) * sizeof(cpx<R>);
    dim3 grid(h->G.nxh, a.njobs);
#define L_YB4(N) sw_launch(h, SWENSE_K_YINV, &k_yinv_b4<R, N>, grid, dim3(256), lds, st, a, h->G, wp, nrows, row0)
    SW_B4_DISPATCH(plan.n, L_YB4);
#undef L_YB4
    return;
  }
  if (wave_ok<R>(plan.n)) {
    const WPlan wp = make_wplan(plan);
    const size_t lds = 4ull * wbuf_len(plan.n) * sizeof(cpx<R>);
    dim3 grid((h->G.nxh + 3) / 4, a.njobs);
#define L_YINV(E, N) sw_launch(h, SWENSE_K_YINV, &k_yinv_w<R, E, N>, grid, dim3(256), lds, st, a, h->G, wp, nrows, row0)
    SW_FFT_DISPATCH(plan.n, L_YINV);
#undef L_YINV
    return;
  }
  const int TW = choose_tw(plan.n, sizeof(cpx<R>));
  const size_t lds = 2ull * TW * plan.n * sizeof(cpx<R>);
  dim3 grid((h->G.nxh + TW - 1) / TW, a.njobs);
  SW_LAUNCH(h, SWENSE_K_YINV, k_yinv<R>, grid, dim3(256), lds, st, a, h->G, plan, TW, nrows, row0);
  SW_HIP(hipGetLastError());
}

template <typename R>
void yfwd_t(swense_hos* h, const YFwdArgs& a, const FftPlan& plan, hipStream_t st) {
  if (h->prof.on) {
    // rows read once; per mode the FP64 epilogue traffic of each job
    const double modes = (double)h->G.ny * h->G.nxh, c16 = sizeof(cd);
    double b = (double)a.njobs * plan.n * h->G.nxh * sizeof(cpx<R>);
    for (int j = 0; j < a.njobs; ++j) {
      const YFwdJob& jb = a.job[j];
      double per = 0.0;
      if (jb.epi == YE_STORE) per = c16 + (jb.acc_mode == 1 ? 2 * c16 : jb.acc_mode == 2 ? c16 : 0.0);
      else if (jb.epi == YE_NL_ETA || jb.epi == YE_NL_PHI) per = c16;
      else {
        const int st4 = a.rk.stage;  // sin read; then stage-dependent state traffic
        per = c16 + (st4 == 0 ? c16 : st4 == 1 ? 3 * c16 : st4 <= 3 ? 4 * c16 : 3 * c16);
      }
      b += per * modes;
    }
    h->prof.bytes[SWENSE_K_YFWD] += b;
    h->prof.tbytes[SWENSE_K_YFWD] += (double)a.njobs * 2.0 * sizeof(R) * (double)h->Px * h->Py;
  }
  if constexpr (sizeof(R) == 4) {
    const int ny = h->G.ny, rs = plan.n / std::max(ny, 1);
    if ((ny == 256 || ny == 512 || ny == 1024) && rs >= 2 && rs <= 4 && rs * ny == plan.n) {
      // residue form: the column's residue sequences one per wavefront, kept modes combined
      const WPlan wp = make_wplan(plan);
      const size_t lds = (size_t)rs * (ny + ny / 16 + 1) * sizeof(cpx<R>);
      dim3 grid(h->G.nxh, a.njobs);
#define L_YFR(RS, NY) sw_launch(h, SWENSE_K_YFWD, &k_yfwd_r<RS, NY>, grid, dim3(256), lds, st, a, h->G, wp)
#define L_YFRN(RS)                  \
  switch (ny) {                     \
    case 256: L_YFR(RS, 256); break;  \
    case 512: L_YFR(RS, 512); break;  \
    default: L_YFR(RS, 1024); break;  \
  }
      switch (rs) {
        case 2: L_YFRN(2); break;
        case 3: L_YFRN(3); break;
        default: L_YFRN(4); break;
      }
#undef L_YFRN
#undef L_YFR
      return;
    }
    if (ny >= 16 && ny <= 512 && ny % 2 == 0 && rs >= 2 && rs <= 4 && rs * ny == plan.n && !grp_len_ok(plan.n)) {
      // residue form with a runtime plan of the mode count (twiddles from the padded table)
      const WPlan wp = make_wplan(plan);
      FftPlan sub{};
      sub.n = ny;
      sub.tw = plan.tw;
      const WPlan pny = make_wplan(sub);
      const size_t lds = (size_t)rs * wbuf_len(ny) * sizeof(cpx<R>);
      dim3 grid(h->G.nxh, a.njobs);
#define L_YFRR(RS, TQ) sw_launch(h, SWENSE_K_YFWD, &k_yfwd_rr<RS, TQ, 8>, grid, dim3(256), lds, st, a, h->G, wp, pny)
#define L_YFRRN(RS)              \
  if (ny <= 256) L_YFRR(RS, 1); \
  else L_YFRR(RS, 2);
      switch (rs) {
        case 2: L_YFRRN(2); break;
        case 3: L_YFRRN(3); break;
        default: L_YFRRN(4); break;
      }
#undef L_YFRRN
#undef L_YFRR
      return;
    }
  }
  if (grp_len_ok(plan.n) && h->G.ny <= 1024) {
    const WPlan wp = make_wplan(plan);
    const size_t lds = grp_lds_len(plan.n) * sizeof(cpx<R>);
    dim3 grid(h->G.nxh, a.njobs);
#define L_YFB4(N) sw_launch(h, SWENSE_K_YFWD, &k_yfwd_b4<R, N>, grid, dim3(256), lds, st, a, h->G, wp)
    SW_B4_DISPATCH(plan.n, L_YFB4);
#undef L_YFB4
    return;
  }
  if (wave_ok<R>(plan.n)) {
    const WPlan wp = make_wplan(plan);
    const size_t lds = 4ull * wbuf_len(plan.n) * sizeof(cpx<R>);
    dim3 grid((h->G.nxh + 3) / 4, a.njobs);
#define L_YFWD(E, N) sw_launch(h, SWENSE_K_YFWD, &k_yfwd_w<R, E, N>, grid, dim3(256), lds, st, a, h->G, wp)
    SW_FFT_DISPATCH(plan.n, L_YFWD);
#undef L_YFWD
    return;
  }
  const int TW = choose_tw(plan.n, sizeof(cpx<R>));
  const size_t lds = 2ull * TW * plan.n * sizeof(cpx<R>);
  dim3 grid((h->G.nxh + TW - 1) / TW, a.njobs);
  SW_LAUNCH(h, SWENSE_K_YFWD, k_yfwd<R>, grid, dim3(256), lds, st, a, h->G, plan, TW);
  SW_HIP(hipGetLastError());
}

template <typename R>
void xpass_t(swense_hos* h, const XArgs& a) {
  const int Px = h->plan_px.n;
  if (h->prof.on) {
    // each distinct input row set read once, each output written once
    const double rows = (double)h->Py * h->G.nxh * sizeof(cpx<R>);
    double b = ((a.out0 ? 1 : 0) + (a.out1 ? 1 : 0)) * rows;
    for (int j = 0; j < a.nin; ++j) {
      bool seen = false;
      for (int i = 0; i < j; ++i) seen = seen || a.in[i].src == a.in[j].src;
      if (!seen) b += rows;
    }
    h->prof.bytes[SWENSE_K_XPASS] += b;
    const int nout = (a.out0 ? 1 : 0) + (a.out1 ? 1 : 0);
    h->prof.tbytes[SWENSE_K_XPASS] += (double)(a.nin + nout) * 2.0 * sizeof(R) * (double)h->Px * h->Py;
  }
  // rounds version: power-of-two rows up to 1024 points, order <= 4, every
  // gradient pair at an even input index
  bool pairs_ok = true;
  for (int i = 0; i < a.nin; ++i)
    if (a.in[i].role == XR_GRADPAIR) pairs_ok = pairs_ok && (i % 2 == 0) && i + 1 < a.nin;
  if (wave_ok<R>(Px) && pairs_ok && a.M <= 4 && h->G.nx <= Px && (Px == 256 || Px == 512 || Px == 1024)) {
    const size_t lds = 4ull * wbuf_len(Px) * sizeof(cpx<R>);
    const WPlan wp = make_wplan(h->plan_px);
    switch (Px) {
      case 256: sw_launch(h, SWENSE_K_XPASS, &k_xpass_r<R, 8, 256, 4>, dim3(h->Py), dim3(256), lds, h->st, a, h->G, wp); break;
      case 512: sw_launch(h, SWENSE_K_XPASS, &k_xpass_r<R, 8, 512, 4>, dim3(h->Py), dim3(256), lds, h->st, a, h->G, wp); break;
      default: sw_launch(h, SWENSE_K_XPASS, &k_xpass_r<R, 16, 1024, 4>, dim3(h->Py), dim3(256), lds, h->st, a, h->G, wp); break;
    }
    return;
  }
  // FP32 rows of 768, 1536 and 3072 points (three-way transforms): series
  // stages on the workgroup-transform kernel, the others in rounds (order <= 5)
  if constexpr (sizeof(R) == 4) {
    const bool ft = a.stage == XS_FTILDE;
    bool series_ok = (a.stage == XS_SERIES || ft) && h->G.nx <= Px && (Px == 768 || Px == 1536 || Px == 3072);
    for (int i = 0; i < a.nin && series_ok; ++i)
      series_ok = a.in[i].role == XR_ETA || (a.in[i].role == XR_G && a.in[i].wi == 0 && a.in[i].pw <= kMaxM) ||
                  (ft && (a.in[i].role == XR_ETAT || a.in[i].role == XR_PHIT));
    bool final_ok = a.stage == XS_FINAL && pairs_ok && a.M <= 5 && h->G.nx <= Px && Px == 3072;
    for (int i = 0; i < a.nin && final_ok; ++i)
      final_ok = a.in[i].role == XR_ETA || a.in[i].role == XR_G || a.in[i].role == XR_GRADPAIR ||
                 (a.in[i].role == XR_NONE && i > 0 && a.in[i - 1].role == XR_GRADPAIR);
    if (final_ok) {
      // eta and the W terms first (their order kept), then the gradient pairs
      XArgs b = a;
      b.nin = 0;
      for (int i = 0; i < a.nin; ++i)
        if (a.in[i].role == XR_ETA || a.in[i].role == XR_G) b.in[b.nin++] = a.in[i];
      b.ng = b.nin;
      for (int i = 0; i < a.nin; ++i)
        if (a.in[i].role == XR_GRADPAIR) {
          b.in[b.nin++] = a.in[i];
          b.in[b.nin++] = a.in[i + 1];
        }
      SW_REQUIRE(b.nin == a.nin && b.ng >= 1 && b.in[0].role == XR_ETA, "final-stage inputs out of order");
      const WPlan wp = make_wplan(h->plan_px);
      // residue form when the row is three times the mode count
      if (h->G.nx == 1024)
        sw_launch(h, SWENSE_K_XPASS, &k_xpass_final3<R, 1024, 5, 256, true>, dim3(h->Py), dim3(256),
                  b3_len<1024>() * sizeof(cpx<R>), h->st, b, h->G, wp);
      else
        sw_launch(h, SWENSE_K_XPASS, &k_xpass_final3<R, 1024, 5, 256, false>, dim3(h->Py), dim3(256),
                  b3_len<1024>() * sizeof(cpx<R>), h->st, b, h->G, wp);
      return;
    }
    if (series_ok) {
      const WPlan wp = make_wplan(h->plan_px);
#define L_S3R(Q, FT, RES) sw_launch(h, SWENSE_K_XPASS, &k_xpass_series3<R, Q, 256, FT, RES>, dim3(h->Py), dim3(256), \
                                   b3_len<Q>() * sizeof(cpx<R>), h->st, a, h->G, wp)
#define L_S3(Q, FT) \
  if (h->G.nx == Q) L_S3R(Q, FT, true); else L_S3R(Q, FT, false)
      switch (Px) {
        case 768: if (ft) L_S3(256, true); else L_S3(256, false); break;
        case 1536: if (ft) L_S3(512, true); else L_S3(512, false); break;
        default: if (ft) L_S3(1024, true); else L_S3(1024, false); break;
      }
#undef L_S3
#undef L_S3R
      return;
    }
    if (pairs_ok && a.M <= 5 && h->G.nx <= Px && (Px == 768 || Px == 1536 || Px == 3072)) {
      const WPlan wp = make_wplan(h->plan_px);
      const size_t wl = Px == 768 ? b3_len<256>() : (Px == 1536 ? b3_len<512>() : b3_len<1024>());
      const size_t lds = 4ull * wl * sizeof(cpx<R>);
      switch (Px) {
        case 768: sw_launch(h, SWENSE_K_XPASS, &k_xpass_r<R, 16, 768, 5>, dim3(h->Py), dim3(256), lds, h->st, a, h->G, wp); break;
        case 1536: sw_launch(h, SWENSE_K_XPASS, &k_xpass_r<R, 32, 1536, 5>, dim3(h->Py), dim3(256), lds, h->st, a, h->G, wp); break;
        default: sw_launch(h, SWENSE_K_XPASS, &k_xpass_r<R, 48, 3072, 5>, dim3(h->Py), dim3(256), lds, h->st, a, h->G, wp); break;
      }
      return;
    }
  }
  {
    const size_t lds = 4ull * wbuf_len(Px) * sizeof(cpx<R>) + (size_t)a.nin * Px * sizeof(R);
    if (wave_ok<R>(Px) && lds <= 160 * 1024) {
      const WPlan wp = make_wplan(h->plan_px);
#define L_XP(E, N) sw_launch(h, SWENSE_K_XPASS, &k_xpass_w<R, E, N>, dim3(h->Py), dim3(256), lds, h->st, a, h->G, wp)
      SW_FFT_DISPATCH(Px, L_XP);
#undef L_XP
      return;
    }
  }
  const size_t lds = 2ull * Px * sizeof(cpx<R>) + (size_t)a.nslots * Px * sizeof(R);
  SW_REQUIRE(lds <= 160 * 1024, "x pass needs more LDS than a workgroup has (reduce nx or order)");
  set_lds_limit<R>(reinterpret_cast<const void*>(&k_xpass<R>), lds);
  SW_LAUNCH(h, SWENSE_K_XPASS, k_xpass<R>, dim3(h->Py), dim3(256), lds, h->st, a, h->G, h->plan_px);
  SW_HIP(hipGetLastError());
}

void add_job(YInvArgs& a, const cd* src, void* dst, int sym, int jpow = 0) {
  SW_REQUIRE(a.njobs < kMaxYJobs, "too many y jobs");
  YInvJob& j = a.job[a.njobs++];
  std::memset(&j, 0, sizeof(j));
  j.src = src;
  j.dst = dst;
  j.sym = sym;
  j.jpow = jpow;
}

void add_in(XArgs& a, const void* src, int dx, int role, int slot = 0, int pw = 0, int wi = 0) {
  SW_REQUIRE(a.nin < kMaxXIn, "too many x inputs");
  XIn& f = a.in[a.nin++];
  f.src = src;
  f.dx = dx;
  f.role = role;
  f.slot = slot;
  f.pw = pw;
  f.wi = wi;
}

// Order-M Dirichlet series: given g(1, j) = F^-1(Dz^j base) already in the
// g buffers for j <= jmax(1), produce modes m = 2..M into `modes` and the
// g(m, j) they need; jmax(m) = M - m + extra (extra = 1 when W is needed).
template <typename R>
void series_t(swense_hos* h, cd** modes, cd* accum, int extra) {
  const int M = h->d.order_m;
  for (int m = 1; m < M; ++m) {
    XArgs xa;
    std::memset(&xa, 0, sizeof(xa));
    xa.stage = XS_SERIES;
    xa.M = M;
    xa.nslots = 2;
    xa.s_eta = 0;
    xa.s_w[0] = 1;
    add_in(xa, h->e_, 0, XR_ETA);
    for (int j = 1; j <= m; ++j) add_in(xa, h->gbuf[m + 1 - j][j], 0, XR_G, 1, j);
    xa.out0 = h->q_;
    xa.out1 = nullptr;
    xpass_t<R>(h, xa);
    YFwdArgs fa;
    std::memset(&fa, 0, sizeof(fa));
    fa.njobs = 1;
    fa.job[0].src = h->q_;
    fa.job[0].dst = modes[m + 1];
    fa.job[0].acc = accum;
    fa.job[0].acc_mode = accum ? 1 : 0;
    fa.job[0].epi = YE_STORE;
    yfwd_t<R>(h, fa, h->plan_py, h->st);
    YInvArgs ya;
    std::memset(&ya, 0, sizeof(ya));
    for (int j = 1; j <= M - (m + 1) + extra; ++j) add_job(ya, modes[m + 1], h->gbuf[m + 1][j], SYM_DZ, j);
    yinv_t<R>(h, ya, h->plan_py, h->Py, 0, h->st);
  }
}

template <typename R>
void rhs_t(swense_hos* h, const cd* se, const cd* sp, const RkArgs& rk, bool want_modes, bool nl_only = false) {
  const int M = h->d.order_m;
  const bool three = h->G.ny > 1;
  YInvArgs ya;
  std::memset(&ya, 0, sizeof(ya));
  add_job(ya, se, h->e_, SYM_ONE);
  if (three) add_job(ya, se, h->ey_, SYM_IKY);
  add_job(ya, sp, h->ph_, SYM_ONE);
  if (three) add_job(ya, sp, h->py_, SYM_IKY);
  for (int j = 1; j <= M; ++j) add_job(ya, sp, h->gbuf[1][j], SYM_DZ, j);
  yinv_t<R>(h, ya, h->plan_py, h->Py, 0, h->st);
  if (want_modes) {
    SW_LAUNCH(h, SWENSE_K_AUX, k_copy_cd, dim3((h->nc + 255) / 256), dim3(256), 0, h->st, sp, h->amod, h->nc);
    SW_HIP(hipGetLastError());
  }
  series_t<R>(h, h->phim, want_modes ? h->amod : nullptr, 1);
  // final products
  XArgs xa;
  std::memset(&xa, 0, sizeof(xa));
  xa.stage = XS_FINAL;
  xa.M = M;
  xa.s_eta = 0;
  xa.s_ge2 = 1;
  xa.s_dot = 2;
  xa.s_gp2 = 3;
  for (int m = 0; m < M; ++m) xa.s_w[m] = 4 + m;
  xa.nslots = 4 + M;
  add_in(xa, h->e_, 0, XR_ETA);
  add_in(xa, h->gbuf[1][1], 0, XR_G, xa.s_w[0], 0, 0);
  add_in(xa, h->e_, 1, XR_GRADPAIR);
  add_in(xa, h->ph_, 1, XR_NONE);
  if (three) {
    add_in(xa, h->ey_, 0, XR_GRADPAIR);
    add_in(xa, h->py_, 0, XR_NONE);
  }
  for (int m = 1; m <= M; ++m)
    for (int j = 1; m + j <= M + 1; ++j) {
      if (m == 1 && j == 1) continue;
      add_in(xa, h->gbuf[m][j], 0, XR_G, xa.s_w[m + j - 2], j - 1, m + j - 2);
    }
  xa.out0 = h->r0_;
  xa.out1 = h->r1_;
  xpass_t<R>(h, xa);
  YFwdArgs fa;
  std::memset(&fa, 0, sizeof(fa));
  fa.njobs = 2;
  fa.job[0].src = h->r0_;
  fa.job[0].epi = nl_only ? YE_NL_ETA : YE_RHS_ETA;
  fa.job[1].src = h->r1_;
  fa.job[1].epi = nl_only ? YE_NL_PHI : YE_RHS_PHI;
  fa.rk = rk;
  yfwd_t<R>(h, fa, h->plan_py, h->st);
}

template <typename R>
void step_t(swense_hos* h, int nsteps) {
  if (nsteps <= 0) return;
  // The first stage reuses the right-hand side of the current state when the
  // mean-level modes have just evaluated it (the usual CFD coupling: step,
  // then interpolate).  Under graph capture the owner of the graph decides
  // (graph_reuse_k): it holds only when every replay ends with the modes of
  // its new state and the first replay is primed (hos_prime_rhs).
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  SW_HIP(hipStreamIsCapturing(h->st, &cap));
  const bool reuse_k = cap == hipStreamCaptureStatusNone ? h->kk_version == h->version : h->graph_reuse_k;
  for (int n = 0; n < nsteps; ++n) {
    const cd* sin_e[4] = {h->xn[0], h->sa[0], h->sb[0], h->sa[0]};
    const cd* sin_p[4] = {h->xn[1], h->sa[1], h->sb[1], h->sa[1]};
    cd* sout_e[4] = {h->sa[0], h->sb[0], h->sa[0], nullptr};
    cd* sout_p[4] = {h->sa[1], h->sb[1], h->sa[1], nullptr};
    for (int s = 0; s < 4; ++s) {
      RkArgs rk;
      std::memset(&rk, 0, sizeof(rk));
      rk.stage = s + 1;
      rk.dt = h->d.dt;
      rk.xn[0] = h->xn[0];
      rk.xn[1] = h->xn[1];
      rk.sin[0] = sin_e[s];
      rk.sin[1] = sin_p[s];
      rk.sout[0] = sout_e[s];
      rk.sout[1] = sout_p[s];
      rk.acc[0] = h->acc[0];
      rk.acc[1] = h->acc[1];
      if (s == 0 && n == 0 && reuse_k) {
        SW_LAUNCH(h, SWENSE_K_AUX, k_rk_first, dim3((h->nc + 255) / 256), dim3(256), 0, h->st, h->kk[0], h->kk[1],
                  h->xn[0], h->xn[1], h->acc[0], h->acc[1], sout_e[0], sout_p[0], h->d.dt, h->nc);
        SW_HIP(hipGetLastError());
        continue;
      }
      rhs_t<R>(h, sin_e[s], sin_p[s], rk, false);
    }
    h->t += h->d.dt;
  }
  h->version++;
}

template <typename R>
void step_exp_t(swense_hos* h, double tau, int nsub) {
  const double hh = tau / nsub;
  for (int n = 0; n < nsub; ++n) {
    for (int s = 1; s <= 4; ++s) {
      const cd* se = s == 1 ? h->xn[0] : h->sa[0];
      const cd* sp = s == 1 ? h->xn[1] : h->sa[1];
      RkArgs rk;
      std::memset(&rk, 0, sizeof(rk));
      rk.kout[0] = h->sb[0];
      rk.kout[1] = h->sb[1];
      rhs_t<R>(h, se, sp, rk, false, true);
      SW_LAUNCH(h, SWENSE_K_AUX, k_ifrk4, dim3((h->nc + 255) / 256), dim3(256), 0, h->st, s, h->xn[0], h->xn[1],
                h->sb[0], h->sb[1], h->acc[0], h->acc[1], h->sa[0], h->sa[1], h->G, hh);
      SW_HIP(hipGetLastError());
    }
    h->t += hh;
  }
  h->version++;
}

template <typename R>
void rhs_only_t(swense_hos* h, bool want_modes) {
  RkArgs rk;
  std::memset(&rk, 0, sizeof(rk));
  rk.stage = 0;
  rk.sin[0] = h->xn[0];
  rk.sin[1] = h->xn[1];
  rk.kout[0] = h->kk[0];
  rk.kout[1] = h->kk[1];
  rhs_t<R>(h, h->xn[0], h->xn[1], rk, want_modes);
  h->kk_version = h->version;
}

// a6: A = sum phi^(m) (from the series), eta_t (the right-hand side) and A_t
// from the series on f = phis_t - [M>=2] W_M eta_t.
template <typename R>
void modes_t(swense_hos* h) {
  const int M = h->d.order_m;
  rhs_only_t<R>(h, true);
  YInvArgs ya;
  std::memset(&ya, 0, sizeof(ya));
  add_job(ya, h->kk[0], h->et_, SYM_ONE);
  add_job(ya, h->kk[1], h->pt_, SYM_ONE);
  yinv_t<R>(h, ya, h->plan_py, h->Py, 0, h->st);
  XArgs xa;
  std::memset(&xa, 0, sizeof(xa));
  xa.stage = XS_FTILDE;
  xa.M = M;
  xa.s_eta = 0;
  xa.s_w[0] = 1;
  xa.s_etat = 2;
  xa.s_phit = 3;
  xa.nslots = 4;
  add_in(xa, h->e_, 0, XR_ETA);
  if (M >= 2)
    for (int m = 1; m <= M; ++m)
      for (int j = 1; m + j <= M + 1; ++j) add_in(xa, h->gbuf[m][j], 0, XR_G, 1, j - 1);
  add_in(xa, h->et_, 0, XR_ETAT);
  add_in(xa, h->pt_, 0, XR_PHIT);
  xa.out0 = h->q_;
  xpass_t<R>(h, xa);
  YFwdArgs fa;
  std::memset(&fa, 0, sizeof(fa));
  fa.njobs = 1;
  fa.job[0].src = h->q_;
  fa.job[0].dst = h->bm[1];
  fa.job[0].acc = h->atmod;
  fa.job[0].acc_mode = 2;
  fa.job[0].epi = YE_STORE;
  yfwd_t<R>(h, fa, h->plan_py, h->st);
  std::memset(&ya, 0, sizeof(ya));
  for (int j = 1; j <= M - 1; ++j) add_job(ya, h->bm[1], h->gbuf[1][j], SYM_DZ, j);
  yinv_t<R>(h, ya, h->plan_py, h->Py, 0, h->st);
  series_t<R>(h, h->bm, h->atmod, 0);
  h->modes_version = h->version;
}

void set_state_phys(swense_hos* h, const double* eta, const double* phis) {
  const size_t np = (size_t)h->G.nx * h->G.ny;
  SW_HIP(hipMemcpyAsync(h->phys, eta, np * sizeof(double), hipMemcpyHostToDevice, h->st));
  SW_HIP(hipMemcpyAsync(h->phys + np, phis, np * sizeof(double), hipMemcpyHostToDevice, h->st));
  hos_phys_to_spec(h, h->xn[0], h->xn[1], false);
}

void get_state_phys(swense_hos* h, double* eta, double* phis) {
  const size_t np = (size_t)h->G.nx * h->G.ny;
  hos_spec_to_phys(h, h->xn[0], h->xn[1]);
  if (eta) SW_HIP(hipMemcpyAsync(eta, h->phys, np * sizeof(double), hipMemcpyDeviceToHost, h->st));
  if (phis) SW_HIP(hipMemcpyAsync(phis, h->phys + np, np * sizeof(double), hipMemcpyDeviceToHost, h->st));
  SW_HIP(hipStreamSynchronize(h->st));
}

void check_desc(const swense_hos_desc* d) {
  SW_REQUIRE(d != nullptr, "null descriptor");
  SW_REQUIRE(d->dim == 2 || d->dim == 3, "dim must be 2 or 3");
  SW_REQUIRE(d->nx >= 4 && d->nx % 2 == 0 && is_235_smooth(d->nx), "nx must be even, >= 4 and 2/3/5-smooth");
  if (d->dim == 2) SW_REQUIRE(d->ny == 1, "ny must be 1 in 2D");
  else SW_REQUIRE(d->ny >= 4 && d->ny % 2 == 0 && is_235_smooth(d->ny), "ny must be even, >= 4 and 2/3/5-smooth");
  SW_REQUIRE(d->order_m >= 1 && d->order_m <= kMaxM, "order_m must be in [1, 8]");
  SW_REQUIRE(d->lx > 0 && d->ly > 0 && d->g > 0 && d->rho > 0, "lengths, g and rho must be positive");
  SW_REQUIRE(d->precision == 0 || d->precision == 1, "precision must be 0 or 1");
  SW_REQUIRE(d->dealias >= 0 && d->dealias <= 2, "dealias must be 0, 1 or 2");
}

// Product-grid length: the mode count (dealias 0), the smallest even
// 2/3/5-smooth length >= (M + 1) n / 2 (1), or the smallest 2^k or 3 2^k
// length >= (M + 1) n / 2 (2: the lengths with compile-time transforms; any
// length past the bound gives the same truncated products).
int padded_len(int n, int M, int dealias) {
  if (n == 1) return 1;
  if (!dealias) return n;
  int v = ((M + 1) * n + 1) / 2;
  v += v & 1;
  if (dealias == 2) {
    long long best = 0;
    for (long long b : {2ll, 6ll}) {
      long long c = b;
      while (c < v) c *= 2;
      if (best == 0 || c < best) best = c;
    }
    return (int)best;
  }
  while (!is_235_smooth(v)) v += 2;
  return v;
}

size_t up256(size_t b) { return (b + 255) & ~size_t(255); }

// Bytes of the handle's pool: FP64 spectral buffers, transform-precision
// intermediates, physical staging, a state-check flag.
size_t pool_bytes(const swense_hos_desc* d) {
  const int M = d->order_m;
  const size_t ny = d->dim == 2 ? 1 : d->ny, nxh = d->nx / 2 + 1;
  const size_t nc = ny * nxh, ni = (size_t)padded_len(d->ny, M, d->dealias) * nxh;
  const size_t isz = d->precision == 1 ? sizeof(cd) : sizeof(cf);
  const size_t ncd = 2 * 5 + (size_t)(M + 1) * 2 + 2;  // xn sa sb acc kk, phim bm, amod atmod
  size_t ngb = 0;
  for (int m = 1; m <= M; ++m) ngb += M + 2 - m;
  const size_t nint = 4 + ngb + 5;
  const size_t nphys = (size_t)d->nx * ny;
  return up256(ncd * nc * sizeof(cd) + nint * ni * isz + 2 * nphys * sizeof(double) + 2 * nc * sizeof(cd) + 1024 + 256);
}

// Whole workspace of a handle: pool, twiddle tables of the product and mode
// grids, the surface copy of the concurrent interpolation, the snapshot and
// the spectra interpolated in time.
size_t workspace_bytes(const swense_hos_desc* d) {
  const size_t ny = d->dim == 2 ? 1 : d->ny, nc = ny * (d->nx / 2 + 1);
  const bool fp64 = d->precision == 1;
  const int px = padded_len(d->nx, d->order_m, d->dealias), py = padded_len(d->dim == 2 ? 1 : d->ny, d->order_m, d->dealias);
  return pool_bytes(d) + TwiddleCache::table_bytes(px, fp64) + TwiddleCache::table_bytes(py, fp64) +
         TwiddleCache::table_bytes(d->nx, true) + TwiddleCache::table_bytes(d->dim == 2 ? 1 : d->ny, true) +
         up256(nc * sizeof(cd)) + 2 * up256(4 * nc * sizeof(cd));
}

void allocate(swense_hos* h, void* ws) {
  const int M = h->d.order_m;
  h->nc = (size_t)h->G.ny * h->G.nxh;
  h->ni = (size_t)h->Py * h->G.nxh;
  const size_t bytes = pool_bytes(&h->d);
  if (ws) h->pool = ws;
  else SW_HIP(hipMalloc(&h->pool, bytes));
  SW_HIP(hipMemsetAsync(h->pool, 0, bytes, h->st));
  h->flag = reinterpret_cast<int*>(reinterpret_cast<char*>(h->pool) + bytes - 256);
  char* p = reinterpret_cast<char*>(h->pool);
  auto take_cd = [&]() {
    cd* r = reinterpret_cast<cd*>(p);
    p += h->nc * sizeof(cd);
    return r;
  };
  auto take_i = [&]() {
    void* r = p;
    p += h->ni * h->isz();
    return r;
  };
  for (int w = 0; w < 2; ++w) {
    h->xn[w] = take_cd();
    h->sa[w] = take_cd();
    h->sb[w] = take_cd();
    h->acc[w] = take_cd();
    h->kk[w] = take_cd();
  }
  for (int m = 0; m <= M; ++m) {
    h->phim[m] = take_cd();
    h->bm[m] = take_cd();
  }
  h->amod = take_cd();
  h->atmod = take_cd();
  h->e_ = take_i();
  h->ey_ = take_i();
  h->ph_ = take_i();
  h->py_ = take_i();
  for (int m = 1; m <= M; ++m)
    for (int j = 1; j <= M + 1 - m; ++j) h->gbuf[m][j] = take_i();
  h->q_ = take_i();
  h->r0_ = take_i();
  h->r1_ = take_i();
  h->et_ = take_i();
  h->pt_ = take_i();
  p = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(p) + 255) & ~uintptr_t(255));
  h->phys = reinterpret_cast<double*>(p);
}

void load_state(swense_hos* h, const double* eta, const double* phis, int layout) {
  SW_REQUIRE(eta && phis, "null state arrays");
  if (layout == SWENSE_SPECTRAL) {
    // enforce the kept-mode convention: zero Nyquist row/column
    std::vector<cd> e(h->nc), ph(h->nc);
    std::memcpy(e.data(), eta, h->nc * sizeof(cd));
    std::memcpy(ph.data(), phis, h->nc * sizeof(cd));
    for (int q = 0; q < h->G.ny; ++q)
      for (int pp = 0; pp < h->G.nxh; ++pp) {
        bool nyq = (2 * pp == h->G.nx) || (h->G.ny > 1 && 2 * q == h->G.ny);
        if (nyq) {
          e[(size_t)q * h->G.nxh + pp] = mk(0.0, 0.0);
          ph[(size_t)q * h->G.nxh + pp] = mk(0.0, 0.0);
        }
      }
    SW_HIP(hipMemcpyAsync(h->xn[0], e.data(), h->nc * sizeof(cd), hipMemcpyHostToDevice, h->st));
    SW_HIP(hipMemcpyAsync(h->xn[1], ph.data(), h->nc * sizeof(cd), hipMemcpyHostToDevice, h->st));
    SW_HIP(hipStreamSynchronize(h->st));
  } else {
    SW_REQUIRE(layout == SWENSE_PHYSICAL, "layout must be SWENSE_PHYSICAL or SWENSE_SPECTRAL");
    set_state_phys(h, eta, phis);
    SW_HIP(hipStreamSynchronize(h->st));
  }
  h->version++;
}

}  // namespace

void set_error(swense_hos* h, const SwenseError& e) { h->err = e.msg; }

void hos_phys_to_spec(swense_hos* h, cd* e, cd* p, bool add) {
  const int nx = h->G.nx, ny = h->G.ny;
  const size_t np = (size_t)nx * ny;
  cd* rows_e = reinterpret_cast<cd*>(h->phys + 2 * np);
  cd* rows_p = rows_e + (size_t)ny * h->G.nxh;
  const size_t lds = 2ull * nx * sizeof(cd);
  SW_LAUNCH(h, SWENSE_K_AUX, k_phys_in, dim3(ny), dim3(256), lds, h->st, h->phys, h->phys + np, rows_e, rows_p, h->G,
            h->plan_nx);
  SW_HIP(hipGetLastError());
  YFwdArgs fa;
  std::memset(&fa, 0, sizeof(fa));
  fa.njobs = 2;
  if (add) {
    // the transformed fields are added into (e, p); the RK stage buffers (free
    // between steps) take the plain result
    cd* tmp_e = reinterpret_cast<cd*>(h->sa[0]);
    cd* tmp_p = reinterpret_cast<cd*>(h->sa[1]);
    fa.job[0] = YFwdJob{rows_e, tmp_e, e, 1, YE_STORE};
    fa.job[1] = YFwdJob{rows_p, tmp_p, p, 1, YE_STORE};
  } else {
    fa.job[0] = YFwdJob{rows_e, e, nullptr, 0, YE_STORE};
    fa.job[1] = YFwdJob{rows_p, p, nullptr, 0, YE_STORE};
  }
  yfwd_t<double>(h, fa, h->plan_ny, h->st);
  h->version++;
}

void hos_spec_to_phys(swense_hos* h, const cd* e, const cd* p) {
  const int nx = h->G.nx, ny = h->G.ny;
  const size_t np = (size_t)nx * ny;
  cd* rows_e = reinterpret_cast<cd*>(h->phys + 2 * np);
  cd* rows_p = rows_e + (size_t)ny * h->G.nxh;
  YInvArgs ya;
  std::memset(&ya, 0, sizeof(ya));
  add_job(ya, const_cast<cd*>(e), rows_e, SYM_ONE);
  add_job(ya, const_cast<cd*>(p), rows_p, SYM_ONE);
  yinv_t<double>(h, ya, h->plan_ny, ny, 0, h->st);
  const size_t lds = 2ull * nx * sizeof(cd);
  SW_LAUNCH(h, SWENSE_K_AUX, k_phys_out, dim3(ny), dim3(256), lds, h->st, rows_e, rows_p, h->phys, h->phys + np, h->G,
            h->plan_nx);
  SW_HIP(hipGetLastError());
}

void hos_step(swense_hos* h, int nsteps) {
  if (h->fp64) step_t<double>(h, nsteps);
  else step_t<float>(h, nsteps);
}

void hos_step_exp(swense_hos* h, double tau, int nsub) {
  SW_REQUIRE(nsub >= 1 && tau >= 0.0, "nsub >= 1 and tau >= 0");
  if (h->fp64) step_exp_t<double>(h, tau, nsub);
  else step_exp_t<float>(h, tau, nsub);
}

void hos_prime_rhs(swense_hos* h) {
  if (h->kk_version == h->version) return;
  h->modes_version = -1;
  launch_modes(h);
}

double hos_energy(swense_hos* h) {
  launch_modes(h);
  std::vector<cd> e(h->nc), ph(h->nc), et(h->nc);
  SW_HIP(hipMemcpyAsync(e.data(), h->xn[0], h->nc * sizeof(cd), hipMemcpyDeviceToHost, h->st));
  SW_HIP(hipMemcpyAsync(ph.data(), h->xn[1], h->nc * sizeof(cd), hipMemcpyDeviceToHost, h->st));
  SW_HIP(hipMemcpyAsync(et.data(), h->kk[0], h->nc * sizeof(cd), hipMemcpyDeviceToHost, h->st));
  SW_HIP(hipStreamSynchronize(h->st));
  // Parseval on the half spectrum: p = 0 column once, p > 0 twice.
  double s1 = 0.0, s2 = 0.0;
  for (int q = 0; q < h->G.ny; ++q)
    for (int p = 0; p < h->G.nxh; ++p) {
      const size_t i = (size_t)q * h->G.nxh + p;
      const double w = p == 0 ? 1.0 : 2.0;
      s1 += w * (ph[i].x * et[i].x + ph[i].y * et[i].y);
      s2 += w * (e[i].x * e[i].x + e[i].y * e[i].y);
    }
  const double area = h->G.lx * h->G.ly;
  return 0.5 * area * s1 + 0.5 * h->G.g * area * s2;
}

void launch_yinv(swense_hos* h, const YInvArgs& a, const FftPlan& plan, int nrows, int row0, hipStream_t st) {
  if (h->fp64) yinv_t<double>(h, a, plan, nrows, row0, st);
  else yinv_t<float>(h, a, plan, nrows, row0, st);
}

void launch_modes(swense_hos* h) {
  if (h->modes_version == h->version) return;
  if (h->fp64) modes_t<double>(h);
  else modes_t<float>(h);
}

// ------------------------------------------------------------------ C ABI
extern "C" {

const char* swense_version(void) { return "swense-gfx950 0.1"; }

const char* swense_last_error(const swense_hos* h) {
  if (!h) return "no handle";
  return h->err.c_str();
}

}  // extern "C"

namespace {
int hos_init_impl(const swense_hos_desc* d, const double* eta0, const double* phis0, int layout, void* stream,
                  void* ws, swense_hos** out);
}  // namespace

extern "C" {

int swense_hos_workspace_bytes(const swense_hos_desc* d, size_t* bytes) {
  if (!bytes) return SWENSE_EINVAL;
  *bytes = 0;
  try {
    check_desc(d);
    *bytes = workspace_bytes(d);
    return SWENSE_OK;
  } catch (const SwenseError& e) {
    return e.code;
  }
}

int swense_hos_init_ws(const swense_hos_desc* d, const double* eta0, const double* phis0, int layout, void* stream,
                       void* ws, size_t ws_bytes, swense_hos** out) {
  if (!out) return SWENSE_EINVAL;
  *out = nullptr;
  try {
    check_desc(d);
  } catch (const SwenseError& e) {
    return e.code;
  }
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255)) return SWENSE_EINVAL;
  if (ws_bytes < workspace_bytes(d)) return SWENSE_ENOMEM;
  return hos_init_impl(d, eta0, phis0, layout, stream, ws, out);
}

int swense_hos_init(const swense_hos_desc* d, const double* eta0, const double* phis0, int layout, void* stream,
                    swense_hos** out) {
  if (!out) return SWENSE_EINVAL;
  return hos_init_impl(d, eta0, phis0, layout, stream, nullptr, out);
}

}  // extern "C"

namespace {
int hos_init_impl(const swense_hos_desc* d, const double* eta0, const double* phis0, int layout, void* stream,
                  void* ws, swense_hos** out) {
  *out = nullptr;
  swense_hos* h = nullptr;
  try {
    check_desc(d);
    h = new swense_hos();
    if (ws) {
      // the caller's workspace: pool first, then the tables and buffers
      char* base = reinterpret_cast<char*>(ws);
      const size_t pb = pool_bytes(d), nc = (size_t)(d->dim == 2 ? 1 : d->ny) * (d->nx / 2 + 1);
      const size_t tail = workspace_bytes(d) - pb - up256(nc * sizeof(cd)) - 2 * up256(4 * nc * sizeof(cd));
      h->own_mem = false;
      h->tw.arena = base + pb;
      h->tw.arena_left = tail;
      char* q = base + pb + tail;
      h->eta_snap = reinterpret_cast<cd*>(q);
      h->snapm = reinterpret_cast<cd*>(q + up256(nc * sizeof(cd)));
      h->herm = reinterpret_cast<cd*>(q + up256(nc * sizeof(cd)) + up256(4 * nc * sizeof(cd)));
    }
    h->d = *d;
    h->st = reinterpret_cast<hipStream_t>(stream);
    h->fp64 = d->precision == 1;
    h->G = Geom{d->nx, d->ny, d->nx / 2 + 1, d->lx, d->dim == 2 ? 1.0 : d->ly, d->depth, d->g, d->rho};
    h->Px = padded_len(d->nx, d->order_m, d->dealias);
    h->Py = padded_len(d->ny, d->order_m, d->dealias);
    h->t = d->t0;
    SW_HIP(hipGetDevice(&h->device));
    noalloc_scratch_setup(h->device);  // with the handle's device current
    h->plan_px = h->tw.get(h->Px, h->fp64);
    h->plan_py = h->tw.get(h->Py, h->fp64);
    h->plan_nx = h->tw.get(d->nx, true);
    h->plan_ny = h->tw.get(d->ny, true);
    h->tw.arena = nullptr;  // later tables (evaluation grids) are the library's
    h->tw.arena_left = 0;
    allocate(h, ws);
    load_state(h, eta0, phis0, layout);
    *out = h;
    return SWENSE_OK;
  } catch (const SwenseError& e) {
    if (h) {
      swense_hos_destroy(h);
    }
    return e.code;
  } catch (...) {
    if (h) swense_hos_destroy(h);
    return SWENSE_EHIP;
  }
}
}  // namespace

extern "C" {

int swense_hos_set_state(swense_hos* h, const double* eta, const double* phis, int layout, double t) {
  if (!h) return SWENSE_EINVAL;
  return guarded(h, [&] {
    load_state(h, eta, phis, layout);
    h->t = t;
    return SWENSE_OK;
  });
}

int swense_hos_tune_padding(const swense_hos_desc* d, int nsteps, void* stream, int* dealias, double* ms) {
  if (!d || !dealias || nsteps < 1) return SWENSE_EINVAL;
  try {
    check_desc(d);
    SW_REQUIRE(d->dealias != 0, "padding is tuned for dealiased products only");
    const int ny = d->dim == 2 ? 1 : d->ny;
    int px[2], py[2];
    for (int k = 0; k < 2; ++k) {
      px[k] = padded_len(d->nx, d->order_m, 1 + k);
      py[k] = padded_len(ny, d->order_m, 1 + k);
    }
    double t[2] = {-1.0, -1.0};
    *dealias = 1;
    if (px[0] != px[1] || py[0] != py[1]) {
      // a zero state costs what any state does: the step is data-independent work
      const size_t nc = (size_t)ny * (d->nx / 2 + 1);
      std::vector<double> zero(2 * nc, 0.0);
      for (int k = 0; k < 2; ++k) {
        swense_hos_desc e = *d;
        e.dealias = 1 + k;
        swense_hos* h = nullptr;
        const int rc = hos_init_impl(&e, zero.data(), zero.data(), SWENSE_SPECTRAL, stream, nullptr, &h);
        if (rc != SWENSE_OK) return rc;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        float el = 0.f;
        bool ok = true;
        try {
          hos_step(h, 1);  // plans and tables
          SW_HIP(hipEventCreate(&e0));
          SW_HIP(hipEventCreate(&e1));
          SW_HIP(hipEventRecord(e0, h->st));
          hos_step(h, nsteps);
          SW_HIP(hipEventRecord(e1, h->st));
          SW_HIP(hipEventSynchronize(e1));
          SW_HIP(hipEventElapsedTime(&el, e0, e1));
        } catch (...) {
          ok = false;
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        swense_hos_destroy(h);
        if (!ok) return SWENSE_EHIP;
        t[k] = (double)el / nsteps;
      }
      *dealias = t[1] < t[0] ? 2 : 1;
    }
    if (ms) {
      ms[0] = t[0];
      ms[1] = t[1];
    }
    return SWENSE_OK;
  } catch (const SwenseError& e) {
    return e.code;
  } catch (...) {
    return SWENSE_EHIP;
  }
}

int swense_hos_step(swense_hos* h, int nsteps) {
  if (!h) return SWENSE_EINVAL;
  return guarded(h, [&] {
    SW_REQUIRE(nsteps >= 0, "nsteps must be >= 0");
    hos_step(h, nsteps);
    return SWENSE_OK;
  });
}

int swense_hos_step_exp(swense_hos* h, double tau, int nsub) {
  if (!h) return SWENSE_EINVAL;
  return guarded(h, [&] {
    hos_step_exp(h, tau, nsub);
    return SWENSE_OK;
  });
}

int swense_hos_get_state(swense_hos* h, double* eta, double* phis, double* t, int layout) {
  if (!h) return SWENSE_EINVAL;
  return guarded(h, [&] {
    int* bad = h->flag;
    SW_HIP(hipMemsetAsync(bad, 0, sizeof(int), h->st));
    SW_LAUNCH(h, SWENSE_K_AUX, k_finite, dim3((h->nc + 255) / 256), dim3(256), 0, h->st, h->xn[0], h->xn[1], h->nc, bad);
    int hb = 0;
    SW_HIP(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, h->st));
    SW_HIP(hipStreamSynchronize(h->st));
    if (layout == SWENSE_SPECTRAL) {
      if (eta) SW_HIP(hipMemcpyAsync(eta, h->xn[0], h->nc * sizeof(cd), hipMemcpyDeviceToHost, h->st));
      if (phis) SW_HIP(hipMemcpyAsync(phis, h->xn[1], h->nc * sizeof(cd), hipMemcpyDeviceToHost, h->st));
      SW_HIP(hipStreamSynchronize(h->st));
    } else {
      SW_REQUIRE(layout == SWENSE_PHYSICAL, "layout must be SWENSE_PHYSICAL or SWENSE_SPECTRAL");
      get_state_phys(h, eta, phis);
    }
    if (t) *t = h->t;
    if (hb) throw SwenseError{SWENSE_EUNSTABLE, "state holds non-finite values"};
    return SWENSE_OK;
  });
}

int swense_hos_rhs(swense_hos* h, double* eta_t, double* phis_t) {
  if (!h) return SWENSE_EINVAL;
  return guarded(h, [&] {
    if (h->fp64) rhs_only_t<double>(h, false);
    else rhs_only_t<float>(h, false);
    if (eta_t) SW_HIP(hipMemcpyAsync(eta_t, h->kk[0], h->nc * sizeof(cd), hipMemcpyDeviceToHost, h->st));
    if (phis_t) SW_HIP(hipMemcpyAsync(phis_t, h->kk[1], h->nc * sizeof(cd), hipMemcpyDeviceToHost, h->st));
    SW_HIP(hipStreamSynchronize(h->st));
    return SWENSE_OK;
  });
}

int swense_hos_modes(swense_hos* h, double* a_hat, double* a_t_hat, double* eta_t_hat) {
  if (!h) return SWENSE_EINVAL;
  return guarded(h, [&] {
    launch_modes(h);
    if (a_hat) SW_HIP(hipMemcpyAsync(a_hat, h->amod, h->nc * sizeof(cd), hipMemcpyDeviceToHost, h->st));
    if (a_t_hat) SW_HIP(hipMemcpyAsync(a_t_hat, h->atmod, h->nc * sizeof(cd), hipMemcpyDeviceToHost, h->st));
    if (eta_t_hat) SW_HIP(hipMemcpyAsync(eta_t_hat, h->kk[0], h->nc * sizeof(cd), hipMemcpyDeviceToHost, h->st));
    SW_HIP(hipStreamSynchronize(h->st));
    return SWENSE_OK;
  });
}

int swense_hos_energy(swense_hos* h, double* energy) {
  if (!h || !energy) return SWENSE_EINVAL;
  return guarded(h, [&] {
    *energy = hos_energy(h);
    return SWENSE_OK;
  });
}

int swense_profile_enable(swense_hos* h, int enable) {
  if (!h) return SWENSE_EINVAL;
  return guarded(h, [&] {
    SW_HIP(hipStreamSynchronize(h->st));
    h->prof.recs.clear();
    h->prof.used = 0;
    for (int k = 0; k < SWENSE_K_COUNT; ++k) {
      h->prof.total_ms[k] = 0.0;
      h->prof.count[k] = 0;
      h->prof.bytes[k] = 0.0;
      h->prof.tbytes[k] = 0.0;
    }
    h->prof.on = enable != 0;
    return SWENSE_OK;
  });
}

int swense_profile_read(swense_hos* h, int kernel, double* total_ms, long long* count) {
  if (!h || kernel < 0 || kernel >= SWENSE_K_COUNT) return SWENSE_EINVAL;
  return guarded(h, [&] {
    SW_HIP(hipStreamSynchronize(h->st));
    // fold the pending records into the totals and recycle their events
    for (const ProfRec& r : h->prof.recs) {
      float ms = 0.f;
      SW_HIP(hipEventElapsedTime(&ms, r.a, r.b));
      h->prof.total_ms[r.kid] += ms;
      h->prof.count[r.kid] += 1;
    }
    h->prof.recs.clear();
    h->prof.used = 0;
    if (total_ms) *total_ms = h->prof.total_ms[kernel];
    if (count) *count = h->prof.count[kernel];
    return SWENSE_OK;
  });
}

int swense_profile_bytes(swense_hos* h, int kernel, double* bytes) {
  if (!h || !bytes || kernel < 0 || kernel >= SWENSE_K_COUNT) return SWENSE_EINVAL;
  *bytes = h->prof.bytes[kernel];
  return SWENSE_OK;
}

int swense_profile_transform_bytes(swense_hos* h, int kernel, double* bytes) {
  if (!h || !bytes || kernel < 0 || kernel >= SWENSE_K_COUNT) return SWENSE_EINVAL;
  *bytes = h->prof.tbytes[kernel];
  return SWENSE_OK;
}

void swense_hos_destroy(swense_hos* h) {
  if (!h) return;
  if (h->aux) (void)hipStreamSynchronize(h->aux);
  h->prof.release();
  eval_release(h);
  if (h->own_mem) {
    if (h->eta_snap) (void)hipFree(h->eta_snap);
    if (h->snapm) (void)hipFree(h->snapm);
    if (h->herm) (void)hipFree(h->herm);
  }
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  if (h->ev_join) (void)hipEventDestroy(h->ev_join);
  if (h->aux) (void)hipStreamDestroy(h->aux);
  if (h->pool && h->own_mem) (void)hipFree(h->pool);
  h->tw.release();
  delete h;
}

}  // extern "C"
