// Spectral neural operator surrogate on gfx950: BF16 MFMA GEMMs with FP32
// accumulation for every channel contraction (lift, 1x1 convolutions,
// per-mode complex mixing, projection, and their transposes in the backward
// pass), FP32 wavefront FFTs for the truncated spectral transforms, FP32
// element-wise kernels, and an Adam optimiser on FP32 master weights that
// re-quantises the BF16 copy used by the GEMMs after every step.
//
// Network (per sample, grid n x n, C channels):
//   v0 = W0 x + b0 (x: in_channels input fields);  for l = 1..L: z = W_l v + b_l + K_l(v), v = gelu(z);
//   y = Q2 gelu(Q1 v + c1) + c2.
//   K_l(v): rfft2(v)/n^2 on the retained modes S = {p < P, |q| <= Q}, per-mode
//   complex mixing by R_l (C x C), Hermitian projection of the p = 0 column,
//   inverse real transform sum_S c_p Re(y e^{ik.x}).
// BF16 rounding (round to nearest even) happens at every GEMM input.
#include <algorithm>
#include <cmath>
#include <string>
#include <cstring>
#include <vector>

#include "internal.h"
#include "swense_surrogate.h"
#include "wfft.h"

typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ unsigned short f2bf(float f) {
  unsigned int b = __float_as_uint(f);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (unsigned short)(b >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

__device__ __forceinline__ float gelu_f(float z) {
  const float k = 0.7978845608028654f;
  return 0.5f * z * (1.f + tanhf(k * (z + 0.044715f * z * z * z)));
}
__device__ __forceinline__ float gelu_g(float z) {
  const float k = 0.7978845608028654f;
  const float t = tanhf(k * (z + 0.044715f * z * z * z));
  return 0.5f * (1.f + t) + 0.5f * z * (1.f - t * t) * k * (1.f + 3.f * 0.044715f * z * z);
}

// ------------------------------------------------------------------ GEMM
// C[b](m, n) = alpha sum_k A[b](m, k) B[b](k, n) + beta C[b](m, n) + bias[m]
// Operands FP32 or BF16 with arbitrary strides; batch index b = b1 nb2 + b2
// with separate strides for the two levels (split-K and per-sample batches).
// Complex mode: A holds interleaved complex rows (real K' = 2K), B holds a
// complex K x N matrix expanded on load to the real 2K x 2N block form
// [[Re, Im], [-Im, Re]], C receives interleaved complex; conjugation flags
// apply before the expansion.
struct GemmArgs {
  int M, N, K;        // real sizes (complex mode: K, N are the real 2K, 2N)
  int nb1, nb2;
  const void* A;
  long long sAb1, sAb2, sAm, sAk;
  int a_bf16, a_conj;  // a_conj: complex A (interleaved): negate odd k
  const void* B;
  long long sBb1, sBb2, sBk, sBn;  // complex mode: strides of the complex matrix
  int b_bf16, b_cplx, b_conj;
  float* C;
  long long sCb1, sCb2, sCm, sCn;
  float alpha, beta;
  const float* bias;
  // optional epilogue: + add (same layout as C), pre-activation copy to zout, gelu
  const float* add;
  float* zout;
  int act;
  // load modes chosen on the host from strides and alignment:
  // a_mode 0 scalar, 1 FP32 x4 along k, 2 BF16 x4 along k, 3 BF16 x4 along m;
  // b_mode 0 scalar, 1 FP32 x4 along k, 2 FP32 x4 along n, 3 complex BF16 pairs
  int a_mode, b_mode;
};

constexpr int TM = 64, TN = 64, TK = 32;

__device__ __forceinline__ float ld(const void* p, long long i, int bf) {
  return bf ? bf2f(reinterpret_cast<const unsigned short*>(p)[i]) : reinterpret_cast<const float*>(p)[i];
}

__device__ __forceinline__ float4 ld4(const void* p, long long i) {
  return *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(p) + i);
}

__device__ __forceinline__ uint2 pack4(float a, float b, float c, float d) {
  return uint2{(unsigned)f2bf(a) | ((unsigned)f2bf(b) << 16), (unsigned)f2bf(c) | ((unsigned)f2bf(d) << 16)};
}

// Scalar-mode element e of a tile: (row, k) of A or (col, k) of B.
__device__ __forceinline__ void a_elem(const GemmArgs& g, int e, int& m, int& k) {
  if (g.sAk == 1) { m = e / TK; k = e - m * TK; }
  else { k = e / TM; m = e - k * TM; }
}
__device__ __forceinline__ void b_elem(const GemmArgs& g, int e, int& n, int& k) {
  if (!g.b_cplx && g.sBn == 1) { k = e / TN; n = e - k * TN; }
  else { n = e / TK; k = e - n * TK; }
}

// Global -> registers for the tile at k0 (8 values of A and of B per thread).
template <int AM, int BM>
__device__ __forceinline__ void gemm_load(const GemmArgs& g, long long aoff, long long boff, int m0, int n0, int k0,
                                          int tid, float ra[8], float rb[8]) {
  if constexpr (AM == 1) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int gm = m0 + (tid >> 3) + 32 * j, gk = k0 + (tid & 7) * 4;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (gm < g.M && gk < g.K) v = ld4(g.A, aoff + gm * g.sAm + gk);
      ra[4 * j] = v.x; ra[4 * j + 1] = v.y; ra[4 * j + 2] = v.z; ra[4 * j + 3] = v.w;
    }
  } else if constexpr (AM == 2 || AM == 3) {
    // raw BF16 bits, four consecutive along k (AM 2) or m (AM 3)
    const unsigned short* A = reinterpret_cast<const unsigned short*>(g.A);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int e = tid + 256 * j;
      int gm, gk;
      if constexpr (AM == 2) { gm = m0 + (e >> 3); gk = k0 + (e & 7) * 4; }
      else { gk = k0 + (e >> 4); gm = m0 + (e & 15) * 4; }
      uint2 v = uint2{0u, 0u};
      if (gm < g.M && gk < g.K) v = *reinterpret_cast<const uint2*>(A + aoff + gm * g.sAm + gk * g.sAk);
      ra[2 * j] = __uint_as_float(v.x);
      ra[2 * j + 1] = __uint_as_float(v.y);
    }
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      int m, k;
      a_elem(g, tid + 256 * j, m, k);
      const int gm = m0 + m, gk = k0 + k;
      float v = 0.f;
      if (gm < g.M && gk < g.K) {
        v = ld(g.A, aoff + gm * g.sAm + gk * g.sAk, g.a_bf16);
        if (g.a_conj && (gk & 1)) v = -v;
      }
      ra[j] = v;
    }
  }
  if constexpr (BM == 1) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int gn = n0 + (tid >> 3) + 32 * j, gk = k0 + (tid & 7) * 4;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (gn < g.N && gk < g.K) v = ld4(g.B, boff + gn * g.sBn + gk);
      rb[4 * j] = v.x; rb[4 * j + 1] = v.y; rb[4 * j + 2] = v.z; rb[4 * j + 3] = v.w;
    }
  } else if constexpr (BM == 2) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int gk = k0 + (tid >> 4) + 16 * j, gn = n0 + (tid & 15) * 4;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (gn < g.N && gk < g.K) v = ld4(g.B, boff + gk * g.sBk + gn);
      rb[4 * j] = v.x; rb[4 * j + 1] = v.y; rb[4 * j + 2] = v.z; rb[4 * j + 3] = v.w;
    }
  } else if constexpr (BM == 3) {
    // one complex BF16 element (re, im) per load, expanded to its 2 x 2 real block on store
    const unsigned* Bc = reinterpret_cast<const unsigned*>(g.B);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int e = tid + 256 * j;
      int kc, nc;
      if (g.sBn == 1) { nc = e & 31; kc = e >> 5; }
      else { kc = e & 15; nc = e >> 4; }
      const int gk = k0 + 2 * kc, gn = n0 + 2 * nc;
      unsigned v = 0u;
      if (gk < g.K && gn < g.N) v = Bc[boff + (long long)(gk >> 1) * g.sBk + (long long)(gn >> 1) * g.sBn];
      if (g.b_conj) v ^= 0x80000000u;
      rb[j] = __uint_as_float(v);
    }
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      int n, k;
      b_elem(g, tid + 256 * j, n, k);
      const int gn = n0 + n, gk = k0 + k;
      float v = 0.f;
      if (gn < g.N && gk < g.K) {
        if (g.b_cplx) {
          // real block form of a complex matrix: (gk, gn) -> complex (gk/2, gn/2)
          const long long base = boff + (long long)(gk >> 1) * g.sBk + (long long)(gn >> 1) * g.sBn;
          const float re = ld(g.B, 2 * base, g.b_bf16);
          float im = ld(g.B, 2 * base + 1, g.b_bf16);
          if (g.b_conj) im = -im;
          const int rk = gk & 1, rn = gn & 1;
          v = (rk == rn) ? re : (rk == 0 ? im : -im);
        } else {
          v = ld(g.B, boff + gk * g.sBk + gn * g.sBn, g.b_bf16);
        }
      }
      rb[j] = v;
    }
  }
}

// Registers -> LDS tiles, rounded to BF16.
template <int AM, int BM>
__device__ __forceinline__ void gemm_store(const GemmArgs& g, int tid, const float ra[8], const float rb[8],
                                           unsigned short (*As)[TK + 4], unsigned short (*Bs)[TK + 4]) {
  if constexpr (AM == 1) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int m = (tid >> 3) + 32 * j, k = (tid & 7) * 4;
      *reinterpret_cast<uint2*>(&As[m][k]) = pack4(ra[4 * j], ra[4 * j + 1], ra[4 * j + 2], ra[4 * j + 3]);
    }
  } else if constexpr (AM == 2) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int e = tid + 256 * j;
      *reinterpret_cast<uint2*>(&As[e >> 3][(e & 7) * 4]) = uint2{__float_as_uint(ra[2 * j]), __float_as_uint(ra[2 * j + 1])};
    }
  } else if constexpr (AM == 3) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int e = tid + 256 * j;
      const int k = e >> 4, m = (e & 15) * 4;
      const unsigned lo = __float_as_uint(ra[2 * j]), hi = __float_as_uint(ra[2 * j + 1]);
      As[m][k] = (unsigned short)(lo & 0xFFFFu);
      As[m + 1][k] = (unsigned short)(lo >> 16);
      As[m + 2][k] = (unsigned short)(hi & 0xFFFFu);
      As[m + 3][k] = (unsigned short)(hi >> 16);
    }
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      int m, k;
      a_elem(g, tid + 256 * j, m, k);
      As[m][k] = f2bf(ra[j]);
    }
  }
  if constexpr (BM == 1) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = (tid >> 3) + 32 * j, k = (tid & 7) * 4;
      *reinterpret_cast<uint2*>(&Bs[n][k]) = pack4(rb[4 * j], rb[4 * j + 1], rb[4 * j + 2], rb[4 * j + 3]);
    }
  } else if constexpr (BM == 2) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int k = (tid >> 4) + 16 * j, n = (tid & 15) * 4;
#pragma unroll
      for (int i = 0; i < 4; ++i) Bs[n + i][k] = f2bf(rb[4 * j + i]);
    }
  } else if constexpr (BM == 3) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int e = tid + 256 * j;
      int kc, nc;
      if (g.sBn == 1) { nc = e & 31; kc = e >> 5; }
      else { kc = e & 15; nc = e >> 4; }
      // [[re, im], [-im, re]] in (k, n): row n = 2nc holds (re, -im), row 2nc + 1 holds (im, re)
      const unsigned v = __float_as_uint(rb[j]);
      const unsigned re = v & 0xFFFFu, im = v >> 16, nim = im ^ 0x8000u;
      *reinterpret_cast<unsigned*>(&Bs[2 * nc][2 * kc]) = re | (nim << 16);
      *reinterpret_cast<unsigned*>(&Bs[2 * nc + 1][2 * kc]) = im | (re << 16);
    }
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      int n, k;
      b_elem(g, tid + 256 * j, n, k);
      Bs[n][k] = f2bf(rb[j]);
    }
  }
}

// One 64 x 64 output tile per block (4 waves, 32 x 32 each as 2 x 2 MFMA
// 16x16x32 tiles, one instruction per tile and K tile); the next K tile is
// fetched into registers while the current one is multiplied.  Lane l holds
// row (or column) l % 16 and the eight k = 8 (l / 16) .. + 7 of A and of B
// alike, so the contraction covers every k once.  AM, BM: load modes (see
// GemmArgs).
template <int AM, int BM>
__global__ void __launch_bounds__(256) k_gemm_bf16(GemmArgs g) {
  __shared__ __align__(16) unsigned short As[TM][TK + 4];  // [m][k]
  __shared__ __align__(16) unsigned short Bs[TN][TK + 4];  // [n][k]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int tiles_n = (g.N + TN - 1) / TN;
  const int m0 = (blockIdx.x / tiles_n) * TM, n0 = (blockIdx.x % tiles_n) * TN;
  const int b = blockIdx.y;
  const int b1 = b / g.nb2, b2 = b - b1 * g.nb2;
  const long long aoff = b1 * g.sAb1 + b2 * g.sAb2;
  const long long boff = b1 * g.sBb1 + b2 * g.sBb2;
  const long long coff = b1 * g.sCb1 + b2 * g.sCb2;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  float ra[8], rb[8];
  gemm_load<AM, BM>(g, aoff, boff, m0, n0, 0, tid, ra, rb);
  for (int k0 = 0; k0 < g.K; k0 += TK) {
    gemm_store<AM, BM>(g, tid, ra, rb, As, Bs);
    __syncthreads();
    if (k0 + TK < g.K) gemm_load<AM, BM>(g, aoff, boff, m0, n0, k0 + TK, tid, ra, rb);
    {
      static_assert(TK == 32, "one 16x16x32 MFMA per K tile");
      const int kq = 8 * (lane >> 4);
      v8bf af[2], bfr[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        // two 8-byte LDS reads each (the padded rows keep 8-byte alignment)
        const v4s* pa = reinterpret_cast<const v4s*>(&As[wm + 16 * i + (lane & 15)][kq]);
        const v4s* pb = reinterpret_cast<const v4s*>(&Bs[wn + 16 * i + (lane & 15)][kq]);
        const v4s a0 = pa[0], a1 = pa[1], b0 = pb[0], b1 = pb[1];
        af[i] = __builtin_bit_cast(v8bf, v8s{a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]});
        bfr[i] = __builtin_bit_cast(v8bf, v8s{b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3]});
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int gn = n0 + wn + 16 * j + (lane & 15);
        if (gm < g.M && gn < g.N) {
          float* cp = g.C + coff + gm * g.sCm + gn * g.sCn;
          float v = g.alpha * acc[i][j][r];
          if (g.beta != 0.f) v += g.beta * *cp;
          if (g.bias) v += g.bias[gm];
          const long long ci = coff + gm * g.sCm + gn * g.sCn;
          if (g.add) v += g.add[ci];
          if (g.zout) g.zout[ci] = v;
          if (g.act) v = gelu_f(v);
          *cp = v;
        }
      }
}

// first level of a split-K sum: out2[grp][i] = sum of part[c][i] over the
// parts c of group grp (blockIdx.y), groups of ceil(nparts / gridDim.y)
__global__ void k_reduce_stage(const float* __restrict__ part, int nparts, long long n, float* __restrict__ out2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int per = (nparts + gridDim.y - 1) / gridDim.y;
  const int c0 = blockIdx.y * per, c1 = min(nparts, c0 + per);
  float s = 0.f;
  for (int c = c0; c < c1; ++c) s += part[(long long)c * n + i];
  out2[(long long)blockIdx.y * n + i] = s;
}

// per-channel sums, first level: part[split][c] = sum of channel c of g
// [B][chans][plane] over the split-th slice of the (sample, point) range
__global__ void __launch_bounds__(256) k_rowsum_stage(const float* __restrict__ g, float* __restrict__ part, int B,
                                                      int chans, long long plane) {
  const int c = blockIdx.x, split = blockIdx.y, nsplit = gridDim.y;
  const long long total = (long long)B * plane, len = (total + nsplit - 1) / nsplit;
  const long long u0 = split * len, u1 = min(total, u0 + len);
  float s = 0.f;
  for (long long u = u0 + threadIdx.x; u < u1; u += blockDim.x) {
    const long long b = u / plane, pt = u - b * plane;
    s += g[(b * chans + c) * plane + pt];
  }
  __shared__ float red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(long long)split * chans + c] = red[0];
}

// sum over split-K partials: out[i] = beta out[i] + sum_c part[c][i]
__global__ void k_reduce_parts(const float* __restrict__ part, int nparts, long long n, float* out, float beta) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int c = 0; c < nparts; ++c) s += part[(long long)c * n + i];
  out[i] = (beta != 0.f ? beta * out[i] : 0.f) + s;
}

// ------------------------------------------------------------------ spectral transforms
// Forward: v [B][C][n][n] -> U [B][S][C] complex, S = (qi, p) retained modes
// in q-major order (q = 0..Q, -Q..-1), p < P.  x pass: one wavefront per
// (b, channel pair, row): real transform of two channels packed as one
// complex sequence, keep p < P; y pass: one wavefront per (b, c, p).
struct FnoDims {
  int n, C, P, Q, B;
};

__device__ __forceinline__ int nq_of(const FnoDims& d) { return 2 * d.Q + 1; }

template <int N>
__global__ void __launch_bounds__(256) k_fno_fx(const float* __restrict__ v, cf* __restrict__ xi, FnoDims d,
                                                WPlan plan) {
  extern __shared__ unsigned char smem[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rows_per_block = 4;
  const int ncp = d.C / 2;
  const int job = blockIdx.x * rows_per_block + wave;  // (b, cpair, row)
  const int row = job % N;
  const int cp = (job / N) % ncp;
  const int b = job / (N * ncp);
  if (b >= d.B) return;
  cf* buf = reinterpret_cast<cf*>(smem) + (size_t)wave * wbuf_len(N);
  const float* a = v + (((size_t)b * d.C + 2 * cp) * N + row) * N;
  const float* c = a + (size_t)N * N;
  for (int x = lane; x < N; x += 64) buf[sk(x)] = mk(a[x], c[x]);
  wave_sync();
  wave_fft_any<float, N / 64 < 8 ? 8 : N / 64, N, true>(buf, plan, -1, lane);
  const float sc = 0.5f;
  for (int p = lane; p < d.P; p += 64) {
    const cf zp = buf[sk(p)], zm = conjg(buf[sk((N - p) % N)]);
    const cf s = zp + zm, t = zp - zm;
    const cf o0 = cscale(s, sc), o1 = mk(t.y * sc, -t.x * sc);
    xi[(((size_t)b * d.C + 2 * cp) * N + row) * d.P + p] = o0;
    xi[(((size_t)b * d.C + 2 * cp + 1) * N + row) * d.P + p] = o1;
  }
}

// y pass forward: U[b][s][c] = scale * (cp_flag ? c_p : 1) * F_y(xi[b][c][:, p])[q]
template <int N>
__global__ void __launch_bounds__(256) k_fno_fy(const cf* __restrict__ xi, cf* __restrict__ U, FnoDims d, WPlan plan,
                                                float scale, int cp_flag) {
  extern __shared__ unsigned char smem[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int job = blockIdx.x * 4 + wave;  // (b, c, p)
  const int p = job % d.P, c = (job / d.P) % d.C, b = job / (d.P * d.C);
  if (b >= d.B) return;
  cf* buf = reinterpret_cast<cf*>(smem) + (size_t)wave * wbuf_len(N);
  const cf* src = xi + ((size_t)b * d.C + c) * N * d.P + p;
  for (int y = lane; y < N; y += 64) buf[sk(y)] = src[(size_t)y * d.P];
  wave_sync();
  wave_fft_any<float, N / 64 < 8 ? 8 : N / 64, N, true>(buf, plan, -1, lane);
  const float s = scale * ((cp_flag && p > 0) ? 2.f : 1.f);
  const int nq = nq_of(d);
  for (int a = lane; a < nq; a += 64) {
    const int q = a <= d.Q ? a : a - nq;  // retained order 0..Q, -Q..-1
    const int slot = (q + N) % N;
    U[((size_t)b * nq * d.P + (size_t)a * d.P + p) * d.C + c] = cscale(buf[sk(slot)], s);
  }
}

// Hermitian projection of the p = 0 column of Y [B][S][C] (in place) with an
// optional division by c_p of the p > 0 modes first.
__global__ void k_fno_herm(cf* Y, FnoDims d, int div_cp) {
  const int nq = nq_of(d);
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)d.B * d.C * nq * d.P) return;
  // element (b, a, p, c)
  const int c = (int)(i % d.C);
  const int p = (int)((i / d.C) % d.P);
  const int a = (int)((i / ((long long)d.C * d.P)) % nq);
  const int b = (int)(i / ((long long)d.C * d.P * nq));
  cf* e = Y + (((size_t)b * nq + a) * d.P + p) * d.C + c;
  if (p > 0) {
    if (div_cp) *e = cscale(*e, 0.5f);
    return;
  }
  if (a == 0) {
    e->y = 0.f;
    return;
  }
  if (a > d.Q) return;  // the -q partner is written by the +q thread
  const int am = nq - a;  // position of -q
  cf* f = Y + (((size_t)b * nq + am) * d.P + 0) * d.C + c;
  const cf x = *e, y = *f;
  const cf avg = mk(0.5f * (x.x + y.x), 0.5f * (x.y - y.y));
  *e = avg;
  *f = conjg(avg);
}

// y pass inverse: xi[b][c][row][p] = F_y^-1 of the retained q values of Y[b][:, p][c].
// hmode 1 reads Y through the Hermitian projection of its p = 0 column (the
// +q and -q entries averaged as k_fno_herm does, q = 0 made real); hmode 2
// also halves the p > 0 modes (the projection with the division by c_p).
template <int N>
__global__ void __launch_bounds__(256) k_fno_iy(const cf* __restrict__ Y, cf* __restrict__ xi, FnoDims d,
                                                WPlan plan, int hmode) {
  extern __shared__ unsigned char smem[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int job = blockIdx.x * 4 + wave;
  const int p = job % d.P, c = (job / d.P) % d.C, b = job / (d.P * d.C);
  if (b >= d.B) return;
  cf* buf = reinterpret_cast<cf*>(smem) + (size_t)wave * wbuf_len(N);
  const int nq = nq_of(d);
  for (int y = lane; y < N; y += 64) buf[sk(y)] = mk(0.f, 0.f);
  wave_sync();
  for (int a = lane; a < nq; a += 64) {
    const int q = a <= d.Q ? a : a - nq;
    cf v = Y[((size_t)b * nq * d.P + (size_t)a * d.P + p) * d.C + c];
    if (hmode && p == 0) {
      if (a == 0) {
        v.y = 0.f;
      } else {
        // 0.5 (Y(q) + conj Y(-q)) at +q, its conjugate at -q
        const cf w = Y[((size_t)b * nq * d.P + (size_t)(nq - a) * d.P) * d.C + c];
        v = a <= d.Q ? mk(0.5f * (v.x + w.x), 0.5f * (v.y - w.y)) : mk(0.5f * (w.x + v.x), -(0.5f * (w.y - v.y)));
      }
    } else if (hmode == 2) {
      v = cscale(v, 0.5f);
    }
    buf[sk((q + N) % N)] = v;
  }
  wave_sync();
  wave_fft_any<float, N / 64 < 8 ? 8 : N / 64, N, true>(buf, plan, +1, lane);
  cf* dst = xi + ((size_t)b * d.C + c) * N * d.P + p;
  for (int y = lane; y < N; y += 64) dst[(size_t)y * d.P] = buf[sk(y)];
}

// x pass inverse: out[b][c][row][x] = scale * sum_p c_p Re(xi[..][p] e^{i p x})
// (two channels per complex transform); beta: out = beta out + that.
template <int N>
__global__ void __launch_bounds__(256) k_fno_ix(const cf* __restrict__ xi, float* __restrict__ out, FnoDims d,
                                                WPlan plan, float scale, float beta, const float* __restrict__ zact,
                                                float* __restrict__ gout) {
  extern __shared__ unsigned char smem[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ncp = d.C / 2;
  const int job = blockIdx.x * 4 + wave;
  const int row = job % N, cp = (job / N) % ncp, b = job / (N * ncp);
  if (b >= d.B) return;
  cf* buf = reinterpret_cast<cf*>(smem) + (size_t)wave * wbuf_len(N);
  const cf* ra = xi + (((size_t)b * d.C + 2 * cp) * N + row) * d.P;
  const cf* rb = xi + (((size_t)b * d.C + 2 * cp + 1) * N + row) * d.P;
  for (int s = lane; s < N; s += 64) {
    cf z = mk(0.f, 0.f);
    int p = -1;
    bool cj = false;
    if (s < d.P) p = s;
    else if (s > N - d.P) { p = N - s; cj = true; }
    if (p >= 0) {
      cf va = ra[p], vb = rb[p];
      if (cj) { va = conjg(va); vb = conjg(vb); }
      if (p == 0) { va.y = 0.f; vb.y = 0.f; }  // the p = 0 column transforms to real values
      z = mk(va.x - vb.y, va.y + vb.x);
    }
    buf[sk(s)] = z;
  }
  wave_sync();
  wave_fft_any<float, N / 64 < 8 ? 8 : N / 64, N, true>(buf, plan, +1, lane);
  float* oa = out + (((size_t)b * d.C + 2 * cp) * N + row) * N;
  float* ob = oa + (size_t)N * N;
  if (zact) {
    // the backward's next step fused: gout = out * gelu'(zact), out not stored
    const size_t o0 = (((size_t)b * d.C + 2 * cp) * N + row) * N;
    const float* za = zact + o0;
    const float* zb = za + (size_t)N * N;
    float* ga = gout + o0;
    float* gb = ga + (size_t)N * N;
    for (int x = lane; x < N; x += 64) {
      const cf z = buf[sk(x)];
      const float va = (beta != 0.f ? beta * oa[x] : 0.f) + scale * z.x;
      const float vb = (beta != 0.f ? beta * ob[x] : 0.f) + scale * z.y;
      ga[x] = va * gelu_g(za[x]);
      gb[x] = vb * gelu_g(zb[x]);
    }
    return;
  }
  for (int x = lane; x < N; x += 64) {
    const cf z = buf[sk(x)];
    oa[x] = (beta != 0.f ? beta * oa[x] : 0.f) + scale * z.x;
    ob[x] = (beta != 0.f ? beta * ob[x] : 0.f) + scale * z.y;
  }
}

// Spectral mixing at small batch, Y[b][s][o] = sum_i U[b][s][i] R[s][i][o]
// for b < B <= BB: a weight-bandwidth-bound product (each mode's C x C
// complex BF16 block is read once and used B times), so it runs on the vector
// ALUs with one wavefront per mode instead of a mostly empty MFMA tile.  Lane
// (o4, ig) holds four consecutive outputs o and the rows i = ig (mod G),
// G = 256 / C; its 16-byte weight loads of a row group are contiguous across
// the wavefront.  Operands are the GEMM's: U rounded to BF16, products exact
// in FP32, sums in FP32 (per lane over its rows, then across the G lanes of
// an output quad).
template <int C, int BB>
__global__ void __launch_bounds__(256) k_mix_small(const cf* __restrict__ U, const unsigned* __restrict__ R,
                                                   cf* __restrict__ Y, int B, int S) {
  constexpr int Q4 = C / 4, G = 64 / Q4, ROWS = C / G;
  __shared__ float2 su[4][C][BB];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int s = blockIdx.x * 4 + wave;
  if (s >= S) return;
  for (int e = lane; e < BB * C; e += 64) {
    const int b = e / C, i = e - b * C;
    cf u = mk(0.f, 0.f);
    if (b < B) u = U[((size_t)b * S + s) * C + i];
    su[wave][i][b] = make_float2(bf2f(f2bf(u.x)), bf2f(f2bf(u.y)));
  }
  wave_sync();
  const int o4 = lane % Q4, ig = lane / Q4;
  const uint4* w = reinterpret_cast<const uint4*>(R + (size_t)s * C * C) + o4;
  float2 acc[BB][4];
#pragma unroll
  for (int b = 0; b < BB; ++b)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[b][j] = make_float2(0.f, 0.f);
  constexpr int CH = ROWS < 16 ? ROWS : 16;
#pragma unroll 1
  for (int t0 = 0; t0 < ROWS; t0 += CH) {
    uint4 r[CH];
#pragma unroll
    for (int t = 0; t < CH; ++t) r[t] = w[(size_t)(ig + G * (t0 + t)) * Q4];
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      const int i = ig + G * (t0 + t);
      const unsigned rv[4] = {r[t].x, r[t].y, r[t].z, r[t].w};
#pragma unroll
      for (int b = 0; b < BB; ++b) {
        const float2 u = su[wave][i][b];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float re = __uint_as_float(rv[j] << 16), im = __uint_as_float(rv[j] & 0xFFFF0000u);
          acc[b][j].x = fmaf(u.x, re, fmaf(-u.y, im, acc[b][j].x));
          acc[b][j].y = fmaf(u.x, im, fmaf(u.y, re, acc[b][j].y));
        }
      }
    }
  }
#pragma unroll
  for (int m = Q4; m < 64; m <<= 1)
#pragma unroll
    for (int b = 0; b < BB; ++b)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        acc[b][j].x += __shfl_xor(acc[b][j].x, m);
        acc[b][j].y += __shfl_xor(acc[b][j].y, m);
      }
#pragma unroll
  for (int b = 0; b < BB; ++b)
    if (b % G == ig && b < B) {
      float4* dst = reinterpret_cast<float4*>(Y + ((size_t)b * S + s) * C + 4 * o4);
      dst[0] = make_float4(acc[b][0].x, acc[b][0].y, acc[b][1].x, acc[b][1].y);
      dst[1] = make_float4(acc[b][2].x, acc[b][2].y, acc[b][3].x, acc[b][3].y);
    }
}

// One Fourier layer's output row, fused: for sample b, grid row y and half h
// of the output channels, the inverse x transforms of the row's retained
// modes for those channels (the spectral branch, channel pairs as one
// complex sequence, k_fno_ix's arithmetic) land in LDS while the layer
// input's row values the 1x1 convolution needs are read into registers as
// BF16; the convolution runs on 16x16x32 BF16 MFMA with k_gemm_bf16's
// operands and K order, and the epilogue adds the bias and the spectral
// branch, keeps the pre-activation (zout, when non-null) and applies GELU.
// Results equal the unfused kernels' bit for bit; the spectral branch never
// goes through HBM.  512 threads: wavefront w transforms channel pairs
// 16 h + w and 16 h + w + 8 and computes x tiles 2w, 2w + 1 (16 points
// each) of the half's 32 output channels.
constexpr int kRowC = 64;
template <int N>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) k_fno_row(const cf* __restrict__ xi, const float* __restrict__ vin,
                                                 const unsigned short* __restrict__ W, const float* __restrict__ bias,
                                                 float* __restrict__ vout, float* __restrict__ zout,
                                                 cf* __restrict__ xn, FnoDims d, WPlan plan) {
  static_assert(N == 256, "one row of 256 points, 16 x tiles over 8 wavefronts");
  constexpr int C = kRowC, TP = N + 16, HC = C / 2;
  extern __shared__ unsigned char smem[];
  float* ts = reinterpret_cast<float*>(smem);                  // [half's channel][x], pitch TP
  cf* fb = reinterpret_cast<cf*>(ts + (size_t)HC * TP);        // per-wavefront transform buffers
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int h = blockIdx.x & 1, row = blockIdx.x >> 1;
  const int b = row / N, y = row - b * N;
  const size_t plane = (size_t)N * N;
  const int kq = 8 * (lane >> 4);
  cf* buf = fb + (size_t)wave * wbuf_len(N);
#pragma unroll 1
  for (int cp = HC / 2 * h + wave; cp < HC / 2 * (h + 1); cp += 8) {
    const cf* ra = xi + (((size_t)b * C + 2 * cp) * N + y) * d.P;
    const cf* rb = xi + (((size_t)b * C + 2 * cp + 1) * N + y) * d.P;
    for (int s2 = lane; s2 < N; s2 += 64) {
      cf z = mk(0.f, 0.f);
      int p = -1;
      bool cj = false;
      if (s2 < d.P) p = s2;
      else if (s2 > N - d.P) { p = N - s2; cj = true; }
      if (p >= 0) {
        cf va = ra[p], vb = rb[p];
        if (cj) { va = conjg(va); vb = conjg(vb); }
        if (p == 0) { va.y = 0.f; vb.y = 0.f; }
        z = mk(va.x - vb.y, va.y + vb.x);
      }
      buf[sk(s2)] = z;
    }
    wave_sync();
    wave_fft_any<float, 8, N, true>(buf, plan, +1, lane);
    const int c0 = 2 * cp - HC * h;
    for (int x = lane; x < N; x += 64) {
      const cf z = buf[sk(x)];
      ts[c0 * TP + x] = 0.f + 1.f * z.x;
      ts[(c0 + 1) * TP + x] = 0.f + 1.f * z.y;
    }
    wave_sync();
  }
  // the convolution's B operands (input channels k0 + kq .. + 7 at this
  // lane's x of each tile), read once the transforms are done (held
  // across them they would cost the registers of a second workgroup per CU)
  float vr[2][2][8];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int x = 16 * (2 * wave + j) + (lane & 15);
#pragma unroll
    for (int kc = 0; kc < 2; ++kc)
#pragma unroll
      for (int u = 0; u < 8; ++u) vr[j][kc][u] = vin[((size_t)b * C + 32 * kc + kq + u) * plane + (size_t)y * N + x];
  }
  __syncthreads();
  v4f acc[2][2];
#pragma unroll
  for (int ot = 0; ot < 2; ++ot)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[ot][j] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kc = 0; kc < 2; ++kc) {
    v8bf af[2], bfr[2];
#pragma unroll
    for (int ot = 0; ot < 2; ++ot)
      af[ot] = __builtin_bit_cast(
          v8bf, *reinterpret_cast<const v8s*>(W + (size_t)(HC * h + 16 * ot + (lane & 15)) * C + 32 * kc + kq));
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      v8s t;
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] = (short)f2bf(vr[j][kc][u]);
      bfr[j] = __builtin_bit_cast(v8bf, t);
    }
#pragma unroll
    for (int ot = 0; ot < 2; ++ot)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[ot][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[ot], bfr[j], acc[ot][j], 0, 0, 0);
  }
#pragma unroll
  for (int ot = 0; ot < 2; ++ot)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ol = 16 * ot + 4 * (lane >> 4) + r, o = HC * h + ol;
        const int x = 16 * (2 * wave + j) + (lane & 15);
        float v = 1.f * acc[ot][j][r];
        v += bias[o];
        v += ts[ol * TP + x];
        const size_t ci = ((size_t)b * C + o) * plane + (size_t)y * N + x;
        if (zout) zout[ci] = v;
        const float g = gelu_f(v);
        vout[ci] = g;
        if (xn) ts[ol * TP + x] = g;  // this lane's own slot, read just above
      }
  if (!xn) return;
  // the next layer's forward x transforms of the half's rows (k_fno_fx's
  // arithmetic): channel pairs as one complex sequence, kept modes unpacked
  __syncthreads();
#pragma unroll 1
  for (int lp = wave; lp < HC / 2; lp += 8) {
    for (int x = lane; x < N; x += 64) buf[sk(x)] = mk(ts[(2 * lp) * TP + x], ts[(2 * lp + 1) * TP + x]);
    wave_sync();
    wave_fft_any<float, 8, N, true>(buf, plan, -1, lane);
    const float sc = 0.5f;
    const int c = HC * h + 2 * lp;
    for (int p = lane; p < d.P; p += 64) {
      const cf zp = buf[sk(p)], zm = conjg(buf[sk((N - p) % N)]);
      const cf s2 = zp + zm, t = zp - zm;
      xn[(((size_t)b * C + c) * N + y) * d.P + p] = cscale(s2, sc);
      xn[(((size_t)b * C + c + 1) * N + y) * d.P + p] = mk(t.y * sc, -t.x * sc);
    }
    wave_sync();
  }
}

// Spectral weight gradient: gR[s][i][o] = sum_b conj(U[b][s][i]) gY[b][s][o]
// with both factors rounded to BF16.  A handful of samples per mode makes
// this an outer-product sum bound by the store of gR, so it runs on plain
// FP32 FMAs, one block per mode, the factors staged in LDS.
__global__ void __launch_bounds__(256) k_mix_dw(const cf* __restrict__ U, const cf* __restrict__ gY,
                                                float* __restrict__ gR, int B, int S, int C) {
  extern __shared__ unsigned char smem[];
  cf* su = reinterpret_cast<cf*>(smem);
  cf* sy = su + (size_t)B * C;
  const int s = blockIdx.x;
  for (int e = threadIdx.x; e < B * C; e += blockDim.x) {
    const int b = e / C, c = e - b * C;
    const cf u = U[((size_t)b * S + s) * C + c], y = gY[((size_t)b * S + s) * C + c];
    su[e] = mk(bf2f(f2bf(u.x)), bf2f(f2bf(u.y)));
    sy[e] = mk(bf2f(f2bf(y.x)), bf2f(f2bf(y.y)));
  }
  __syncthreads();
  float2* out = reinterpret_cast<float2*>(gR) + (size_t)s * C * C;
  for (int e = threadIdx.x; e < C * C; e += blockDim.x) {
    const int i = e / C, o = e - i * C;
    float re = 0.f, im = 0.f;
    for (int b = 0; b < B; ++b) {
      const cf u = su[b * C + i], y = sy[b * C + o];
      re += u.x * y.x + u.y * y.y;
      im += u.x * y.y - u.y * y.x;
    }
    out[e] = make_float2(re, im);
  }
}

// ------------------------------------------------------------------ element-wise
__global__ void k_fno_gelu_back(const float* gv, const float* z, float* gz, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) gz[i] = gv[i] * gelu_g(z[i]);
}

// relative L2 per (b, channel): sums of d^2 and t^2 per plane
__global__ void __launch_bounds__(256) k_fno_loss_sums(const float* y, const float* t, float* sums, long long plane) {
  const int bc = blockIdx.x;
  const float* py = y + (size_t)bc * plane;
  const float* pt = t + (size_t)bc * plane;
  float dd = 0.f, tt = 0.f;
  for (long long i = threadIdx.x; i < plane; i += blockDim.x) {
    const float d = py[i] - pt[i];
    dd += d * d;
    tt += pt[i] * pt[i];
  }
  __shared__ float r1[256], r2[256];
  r1[threadIdx.x] = dd;
  r2[threadIdx.x] = tt;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      r1[threadIdx.x] += r1[threadIdx.x + w];
      r2[threadIdx.x] += r2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    sums[2 * bc] = r1[0];
    sums[2 * bc + 1] = r2[0];
  }
}

__global__ void k_fno_loss_grad(const float* y, const float* t, const float* sums, float* gy, long long plane,
                                long long n, float inv_count) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int bc = (int)(i / plane);
  gy[i] = 2.f * (y[i] - t[i]) / sums[2 * bc + 1] * inv_count;
}

// Adam on FP32 masters; the BF16 copy read by the GEMMs is refreshed.
__global__ void k_adam(float* w, unsigned short* wb, const float* g, float* m, float* v, long long n, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  wb[i] = f2bf(wi);
}

__global__ void k_to_bf16(const float* w, unsigned short* wb, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) wb[i] = f2bf(w[i]);
}

}  // namespace

// ------------------------------------------------------------------ host
struct swense_fno {
  swense_fno_desc d{};
  hipStream_t st = nullptr;
  std::string err;
  TwiddleCache tw;
  WPlan plan{};
  size_t nparam = 0;
  // parameter offsets (floats) in the packed vector
  size_t oW0, ob0, oQ1, oc1, oQ2, oc2;
  std::vector<size_t> oW, ob, oR;
  float* w = nullptr;            // FP32 master
  unsigned short* wb = nullptr;  // BF16 copy
  float* g = nullptr;            // gradients
  float* am = nullptr;           // Adam moments
  float* av = nullptr;
  long long adam_t = 0;
  // activations for up to max_batch samples
  int maxb = 0;
  float* act = nullptr;  // v_0 .. v_L, z_1 .. z_L, zq, h  (each [B][C or H][n][n])
  float* tmp = nullptr;  // scratch [B][H][n][n] x 2
  cf* xi = nullptr;      // [B][C][n][P]
  cf* xi2 = nullptr;     // the same, the fused rows' forward modes of the next layer
  cf* U = nullptr;       // per layer [B][S][C]
  cf* Y = nullptr;       // [B][S][C]
  float* part = nullptr;     // split-K partials
  float* part2 = nullptr;    // first-level sums of the partials
  float* rowpart = nullptr;  // per-channel partial sums
  size_t npart = 0;
  float* sums = nullptr;
  int last_batch = 0;
  bool fuse_rows = false;  // layers through k_fno_row (64 channels, 256-point rows, aligned weights)
  float* trace = nullptr;  // caller's buffer for the backward's intermediate gradients (checking)
  void* mem = nullptr;
};

namespace {

size_t count_params(const swense_fno_desc& d) {
  const size_t C = d.channels, H = d.hidden, S = (size_t)(2 * d.q_modes + 1) * d.p_modes;
  return C * d.in_channels + C + (size_t)d.layers * (C * C + C + S * C * C * 2) + H * C + H + 2 * H + 2;
}

void layout(swense_fno* f) {
  const auto& d = f->d;
  const size_t C = d.channels, H = d.hidden, S = (size_t)(2 * d.q_modes + 1) * d.p_modes;
  size_t o = 0;
  f->oW0 = o; o += C * d.in_channels;
  f->ob0 = o; o += C;
  for (int l = 0; l < d.layers; ++l) {
    f->oW.push_back(o); o += C * C;
    f->ob.push_back(o); o += C;
    f->oR.push_back(o); o += S * C * C * 2;
  }
  f->oQ1 = o; o += H * C;
  f->oc1 = o; o += H;
  f->oQ2 = o; o += 2 * H;
  f->oc2 = o; o += 2;
  f->nparam = o;
}

bool aligned(const void* p, int bytes) { return (reinterpret_cast<uintptr_t>(p) & (bytes - 1)) == 0; }

void launch_gemm(hipStream_t st, GemmArgs g) {
  // vector load modes where the contiguous dimension and every offset allow
  // 16-byte (FP32) or 8-byte (BF16) loads
  const bool a_off4 = g.sAb1 % 4 == 0 && g.sAb2 % 4 == 0;
  g.a_mode = 0;
  if (!g.a_conj && a_off4) {
    if (!g.a_bf16 && aligned(g.A, 16) && g.sAk == 1 && g.K % 4 == 0 && g.sAm % 4 == 0) g.a_mode = 1;
    else if (g.a_bf16 && aligned(g.A, 8) && g.sAk == 1 && g.K % 4 == 0 && g.sAm % 4 == 0) g.a_mode = 2;
    else if (g.a_bf16 && aligned(g.A, 8) && g.sAm == 1 && g.M % 4 == 0 && g.sAk % 4 == 0) g.a_mode = 3;
  }
  const bool b_off4 = g.sBb1 % 4 == 0 && g.sBb2 % 4 == 0;
  g.b_mode = 0;
  if (g.b_cplx) {
    if (g.b_bf16 && aligned(g.B, 4) && (g.sBk == 1 || g.sBn == 1)) g.b_mode = 3;
  } else if (!g.b_bf16 && b_off4 && aligned(g.B, 16)) {
    if (g.sBk == 1 && g.K % 4 == 0 && g.sBn % 4 == 0) g.b_mode = 1;
    else if (g.sBn == 1 && g.N % 4 == 0 && g.sBk % 4 == 0) g.b_mode = 2;
  }
  const int tiles = ((g.M + TM - 1) / TM) * ((g.N + TN - 1) / TN);
  SW_REQUIRE(g.nb1 * g.nb2 <= 65535, "GEMM batch count above the grid limit");
  const dim3 grid(tiles, g.nb1 * g.nb2);
#define SW_GEMM_CASE(a, b) \
  case 4 * a + b: hipLaunchKernelGGL((k_gemm_bf16<a, b>), grid, dim3(256), 0, st, g); break;
  switch (4 * g.a_mode + g.b_mode) {
    SW_GEMM_CASE(0, 0) SW_GEMM_CASE(0, 1) SW_GEMM_CASE(0, 2) SW_GEMM_CASE(0, 3)
    SW_GEMM_CASE(1, 0) SW_GEMM_CASE(1, 1) SW_GEMM_CASE(1, 2) SW_GEMM_CASE(1, 3)
    SW_GEMM_CASE(2, 0) SW_GEMM_CASE(2, 1) SW_GEMM_CASE(2, 2) SW_GEMM_CASE(2, 3)
    SW_GEMM_CASE(3, 0) SW_GEMM_CASE(3, 1) SW_GEMM_CASE(3, 2) SW_GEMM_CASE(3, 3)
    default: throw SwenseError{SWENSE_EINVAL, "GEMM load mode"};
  }
#undef SW_GEMM_CASE
  SW_HIP(hipGetLastError());
}

// Split of the point range of a weight-gradient reduction: about 1024 parts
// (several blocks per CU in flight), each a power-of-two chunk of >= 256
// points within one sample.
int wgrad_chunk(long long plane, int B) {
  long long c = 256;
  while (c < plane && (long long)B * plane / c > 1024) c *= 2;
  return (int)c;
}

constexpr int kReduceGroups = 64;

// gW = sum over the nparts partial products in f->part (deterministic two-level sum)
void reduce_parts(swense_fno* f, int nparts, long long n, float* gW) {
  const int groups = std::min(kReduceGroups, nparts);
  hipLaunchKernelGGL(k_reduce_stage, dim3((unsigned)((n + 255) / 256), groups), dim3(256), 0, f->st, f->part, nparts,
                     n, f->part2);
  SW_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_reduce_parts, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, f->st, f->part2, groups, n, gW,
                     0.f);
  SW_HIP(hipGetLastError());
}

GemmArgs gemm0() {
  GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  g.nb1 = g.nb2 = 1;
  g.alpha = 1.f;
  return g;
}

// out[b][o][pt] = sum_i W[o][i] in[b][i][pt] (+ bias), W BF16 [o][i]; with
// add/zout/act the epilogue also adds `add`, keeps the pre-activation in zout
// and applies gelu
void conv1x1(swense_fno* f, const unsigned short* W, int cout, int cin, const float* in, float* out, int B,
             const float* bias, const float* add = nullptr, float* zout = nullptr, int act = 0) {
  const long long plane = (long long)f->d.n * f->d.n;
  GemmArgs g = gemm0();
  g.M = cout;
  g.N = (int)plane;
  g.K = cin;
  g.nb1 = B;
  g.A = W;
  g.sAm = cin;
  g.sAk = 1;
  g.a_bf16 = 1;
  g.B = in;
  g.sBb1 = (long long)cin * plane;
  g.sBk = plane;
  g.sBn = 1;
  g.C = out;
  g.sCb1 = (long long)cout * plane;
  g.sCm = plane;
  g.sCn = 1;
  g.bias = bias;
  g.add = add;
  g.zout = zout;
  g.act = act;
  launch_gemm(f->st, g);
}

// in-grad of a 1x1 convolution: gin[b][i][pt] = sum_o W[o][i] gout[b][o][pt]
void conv1x1_dx(swense_fno* f, const unsigned short* W, int cout, int cin, const float* gout, float* gin, int B,
                float beta) {
  const long long plane = (long long)f->d.n * f->d.n;
  GemmArgs g = gemm0();
  g.M = cin;
  g.N = (int)plane;
  g.K = cout;
  g.nb1 = B;
  g.A = W;
  g.sAm = 1;
  g.sAk = cin;
  g.a_bf16 = 1;
  g.B = gout;
  g.sBb1 = (long long)cout * plane;
  g.sBk = plane;
  g.sBn = 1;
  g.C = gin;
  g.sCb1 = (long long)cin * plane;
  g.sCm = plane;
  g.sCn = 1;
  g.beta = beta;
  launch_gemm(f->st, g);
}

// weight grad: gW[o][i] = sum_{b,pt} gout[b][o][pt] in[b][i][pt], split over
// (sample, point chunk) and reduced
void conv1x1_dw(swense_fno* f, const float* gout, const float* in, int cout, int cin, int B, float* gW) {
  const long long plane = (long long)f->d.n * f->d.n;
  const int chunk = wgrad_chunk(plane, B);
  const int nch = (int)(plane / chunk);
  GemmArgs g = gemm0();
  g.M = cout;
  g.N = cin;
  g.K = chunk;
  g.nb1 = B;
  g.nb2 = nch;
  g.A = gout;
  g.sAb1 = (long long)cout * plane;
  g.sAb2 = chunk;
  g.sAm = plane;
  g.sAk = 1;
  g.B = in;
  g.sBb1 = (long long)cin * plane;
  g.sBb2 = chunk;
  g.sBk = 1;
  g.sBn = plane;
  g.C = f->part;
  g.sCb1 = (long long)nch * cout * cin;
  g.sCb2 = (long long)cout * cin;
  g.sCm = cin;
  g.sCn = 1;
  SW_REQUIRE(plane % chunk == 0 && (long long)B * nch * cout * cin <= (long long)f->npart, "split-K sizes");
  launch_gemm(f->st, g);
  reduce_parts(f, B * nch, (long long)cout * cin, gW);
}

template <int N>
void spec_fwd_n(swense_fno* f, const float* v, cf* U, int B, float scale, int cp_flag) {
  const FnoDims dd{N, f->d.channels, f->d.p_modes, f->d.q_modes, B};
  const size_t lds = 4ull * wbuf_len(N) * sizeof(cf);
  const int jx = B * (f->d.channels / 2) * N;
  hipLaunchKernelGGL(k_fno_fx<N>, dim3((jx + 3) / 4), dim3(256), lds, f->st, v, f->xi, dd, f->plan);
  SW_HIP(hipGetLastError());
  const int jy = B * f->d.channels * f->d.p_modes;
  hipLaunchKernelGGL(k_fno_fy<N>, dim3((jy + 3) / 4), dim3(256), lds, f->st, f->xi, U, dd, f->plan, scale, cp_flag);
  SW_HIP(hipGetLastError());
}

template <int N>
void spec_inv_n(swense_fno* f, const cf* Y, float* out, int B, float scale, float beta, int hmode,
                const float* zact, float* gout) {
  const FnoDims dd{N, f->d.channels, f->d.p_modes, f->d.q_modes, B};
  const size_t lds = 4ull * wbuf_len(N) * sizeof(cf);
  const int jy = B * f->d.channels * f->d.p_modes;
  hipLaunchKernelGGL(k_fno_iy<N>, dim3((jy + 3) / 4), dim3(256), lds, f->st, Y, f->xi, dd, f->plan, hmode);
  SW_HIP(hipGetLastError());
  const int jx = B * (f->d.channels / 2) * N;
  hipLaunchKernelGGL(k_fno_ix<N>, dim3((jx + 3) / 4), dim3(256), lds, f->st, f->xi, out, dd, f->plan, scale, beta,
                     zact, gout);
  SW_HIP(hipGetLastError());
}

void spec_fwd(swense_fno* f, const float* v, cf* U, int B, float scale, int cp_flag) {
  switch (f->d.n) {
    case 64: spec_fwd_n<64>(f, v, U, B, scale, cp_flag); break;
    case 128: spec_fwd_n<128>(f, v, U, B, scale, cp_flag); break;
    case 256: spec_fwd_n<256>(f, v, U, B, scale, cp_flag); break;
    case 512: spec_fwd_n<512>(f, v, U, B, scale, cp_flag); break;
    default: spec_fwd_n<1024>(f, v, U, B, scale, cp_flag); break;
  }
}

// out = beta out + scale * inverse transform of Y; hmode as k_fno_iy (the
// Hermitian projection applied on the way in, Y itself untouched)
// zact, gout (both or neither): instead of storing out, store out * gelu'(zact)
// into gout (the backward's step through the previous layer's activation)
void spec_inv(swense_fno* f, const cf* Y, float* out, int B, float scale, float beta, int hmode,
              const float* zact = nullptr, float* gout = nullptr) {
  switch (f->d.n) {
    case 64: spec_inv_n<64>(f, Y, out, B, scale, beta, hmode, zact, gout); break;
    case 128: spec_inv_n<128>(f, Y, out, B, scale, beta, hmode, zact, gout); break;
    case 256: spec_inv_n<256>(f, Y, out, B, scale, beta, hmode, zact, gout); break;
    case 512: spec_inv_n<512>(f, Y, out, B, scale, beta, hmode, zact, gout); break;
    default: spec_inv_n<1024>(f, Y, out, B, scale, beta, hmode, zact, gout); break;
  }
}

void herm(swense_fno* f, cf* Y, int B, int div_cp) {
  const FnoDims dd{f->d.n, f->d.channels, f->d.p_modes, f->d.q_modes, B};
  const long long n = (long long)B * f->d.channels * (2 * f->d.q_modes + 1) * f->d.p_modes;
  hipLaunchKernelGGL(k_fno_herm, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, f->st, Y, dd, div_cp);
  SW_HIP(hipGetLastError());
}

template <int C>
bool mix_small_c(swense_fno* f, const cf* U, const unsigned short* R, cf* Y, int B, int S) {
  const dim3 grid((S + 3) / 4);
  const unsigned* r = reinterpret_cast<const unsigned*>(R);
  if (B <= 1) hipLaunchKernelGGL((k_mix_small<C, 1>), grid, dim3(256), 0, f->st, U, r, Y, B, S);
  else if (B <= 2) hipLaunchKernelGGL((k_mix_small<C, 2>), grid, dim3(256), 0, f->st, U, r, Y, B, S);
  else if (B <= 4) hipLaunchKernelGGL((k_mix_small<C, 4>), grid, dim3(256), 0, f->st, U, r, Y, B, S);
  else hipLaunchKernelGGL((k_mix_small<C, 8>), grid, dim3(256), 0, f->st, U, r, Y, B, S);
  SW_HIP(hipGetLastError());
  return true;
}

// Y[b][s][o] = sum_i U[b][s][i] R[s][i][o] (complex), per mode s
void mix(swense_fno* f, const cf* U, const unsigned short* R, cf* Y, int B) {
  const int C = f->d.channels, S = (2 * f->d.q_modes + 1) * f->d.p_modes;
  if (B <= 8 && aligned(R, 16) && aligned(Y, 16)) {
    if (C == 32 && mix_small_c<32>(f, U, R, Y, B, S)) return;
    if (C == 64 && mix_small_c<64>(f, U, R, Y, B, S)) return;
    if (C == 128 && mix_small_c<128>(f, U, R, Y, B, S)) return;
  }
  GemmArgs g = gemm0();
  g.M = B;
  g.N = 2 * C;
  g.K = 2 * C;
  g.nb1 = S;
  g.A = U;
  g.sAb1 = 2LL * C;     // floats
  g.sAm = 2LL * S * C;  // next sample
  g.sAk = 1;
  g.B = R;
  g.b_bf16 = 1;
  g.b_cplx = 1;
  g.sBb1 = (long long)C * C;  // complex elements
  g.sBk = C;
  g.sBn = 1;
  g.C = reinterpret_cast<float*>(Y);
  g.sCb1 = 2LL * C;
  g.sCm = 2LL * S * C;
  g.sCn = 1;
  launch_gemm(f->st, g);
}

// gU[b][s][i] = sum_o gY[b][s][o] conj(R[s][i][o])
void mix_dx(swense_fno* f, const cf* gY, const unsigned short* R, cf* gU, int B) {
  const int C = f->d.channels, S = (2 * f->d.q_modes + 1) * f->d.p_modes;
  GemmArgs g = gemm0();
  g.M = B;
  g.N = 2 * C;
  g.K = 2 * C;
  g.nb1 = S;
  g.A = gY;
  g.sAb1 = 2LL * C;
  g.sAm = 2LL * S * C;
  g.sAk = 1;
  g.B = R;
  g.b_bf16 = 1;
  g.b_cplx = 1;
  g.b_conj = 1;
  g.sBb1 = (long long)C * C;
  g.sBk = 1;  // element (k = o, n = i) -> R[i][o]
  g.sBn = C;
  g.C = reinterpret_cast<float*>(gU);
  g.sCb1 = 2LL * C;
  g.sCm = 2LL * S * C;
  g.sCn = 1;
  launch_gemm(f->st, g);
}

// gR[s][i][o] = sum_b conj(U[b][s][i]) gY[b][s][o]
void mix_dw(swense_fno* f, const cf* U, const cf* gY, float* gR, int B) {
  const int C = f->d.channels, S = (2 * f->d.q_modes + 1) * f->d.p_modes;
  const size_t lds = 2ull * B * C * sizeof(cf);
  hipLaunchKernelGGL(k_mix_dw, dim3(S), dim3(256), lds, f->st, U, gY, gR, B, S, C);
  SW_HIP(hipGetLastError());
}

void check_fno_desc(const swense_fno_desc* d) {
  SW_REQUIRE(d != nullptr, "null descriptor");
  SW_REQUIRE(d->n == 64 || d->n == 128 || d->n == 256 || d->n == 512 || d->n == 1024,
             "n must be 64, 128, 256, 512 or 1024");
  SW_REQUIRE(d->channels >= 2 && d->channels % 2 == 0 && d->channels <= 256, "channels must be even, <= 256");
  SW_REQUIRE(d->layers >= 1 && d->layers <= 32, "layers in [1, 32]");
  SW_REQUIRE(d->p_modes >= 1 && d->p_modes < d->n / 2, "p_modes in [1, n/2)");
  SW_REQUIRE(d->q_modes >= 0 && 2 * d->q_modes + 1 <= d->n / 2, "2 q_modes + 1 <= n/2");
  SW_REQUIRE(d->hidden >= 1 && d->max_batch >= 1, "hidden and max_batch must be positive");
  SW_REQUIRE(d->in_channels >= 1 && d->in_channels <= 16, "in_channels in [1, 16]");
  SW_REQUIRE(2ull * d->max_batch * d->channels * sizeof(cf) <= 64 * 1024, "max_batch x channels too large");
}

void allocate_fno(swense_fno* f) {
  const auto& d = f->d;
  const size_t plane = (size_t)d.n * d.n, B = d.max_batch, C = d.channels, H = d.hidden;
  const size_t S = (size_t)(2 * d.q_modes + 1) * d.p_modes;
  const size_t nact = (size_t)(2 * d.layers + 1) * B * C * plane + 2 * B * H * plane + 4 * B * plane;
  const size_t ntmp = 2 * B * std::max(H, C) * plane;
  const size_t nxi = B * C * d.n * d.p_modes;
  const size_t nU = (size_t)d.layers * B * S * C;
  const size_t nY = 2 * B * S * C;
  // split-K partials: at most max(1024, B plane / 256) parts of the largest
  // weight matrix (H x C, C x C, 2 x H or C x in_channels)
  const size_t maxmn = std::max({C * C, H * C, 2 * H, C * (size_t)d.in_channels});
  const size_t nparts = std::max<size_t>(1024, B * plane / 256);
  const size_t npart = nparts * maxmn;
  const size_t npart2 = (size_t)kReduceGroups * maxmn;
  const size_t nrow = 64 * std::max(C, H);
  f->npart = npart;
  // the fused layer rows write the next layer's forward x modes beside the
  // current inverse ones
  const size_t nxi2 = (C == kRowC && d.n == 256) ? nxi : 0;
  size_t bytes = f->nparam * (4 + 2 + 4 + 4 + 4) + nact * 4 + ntmp * 4 + (nxi + nxi2) * 8 + nU * 8 + nY * 8 +
                 npart * 4 + npart2 * 4 + nrow * 4 + 3 * 256 + 2 * B * 2 * 4 + 17 * 256;
  SW_HIP(hipMalloc(&f->mem, bytes));
  SW_HIP(hipMemset(f->mem, 0, bytes));
  char* p = reinterpret_cast<char*>(f->mem);
  auto take = [&](size_t b) {
    void* r = p;
    p += (b + 255) & ~size_t(255);
    return r;
  };
  f->w = reinterpret_cast<float*>(take(f->nparam * 4));
  f->wb = reinterpret_cast<unsigned short*>(take(f->nparam * 2));
  f->g = reinterpret_cast<float*>(take(f->nparam * 4));
  f->am = reinterpret_cast<float*>(take(f->nparam * 4));
  f->av = reinterpret_cast<float*>(take(f->nparam * 4));
  f->act = reinterpret_cast<float*>(take(nact * 4));
  f->tmp = reinterpret_cast<float*>(take(ntmp * 4));
  f->xi = reinterpret_cast<cf*>(take(nxi * 8));
  f->xi2 = nxi2 ? reinterpret_cast<cf*>(take(nxi2 * 8)) : nullptr;
  f->U = reinterpret_cast<cf*>(take(nU * 8));
  f->Y = reinterpret_cast<cf*>(take(nY * 8));
  f->part = reinterpret_cast<float*>(take(npart * 4));
  f->part2 = reinterpret_cast<float*>(take(npart2 * 4));
  f->rowpart = reinterpret_cast<float*>(take(nrow * 4));
  f->sums = reinterpret_cast<float*>(take(2 * B * 2 * 4));
  SW_REQUIRE(p <= reinterpret_cast<char*>(f->mem) + bytes, "internal carve overflow");
}

// activation slots: v_l (l = 0..L) then z_l (l = 1..L), then zq, h
float* v_of(swense_fno* f, int l) {
  return f->act + (size_t)l * (size_t)f->d.max_batch * f->d.channels * f->d.n * f->d.n;
}
float* z_of(swense_fno* f, int l) {
  return f->act + (size_t)(f->d.layers + l) * (size_t)f->d.max_batch * f->d.channels * f->d.n * f->d.n;
}
float* zq_of(swense_fno* f) {
  return f->act + (size_t)(2 * f->d.layers + 1) * (size_t)f->d.max_batch * f->d.channels * f->d.n * f->d.n;
}
float* h_of(swense_fno* f) { return zq_of(f) + (size_t)f->d.max_batch * f->d.hidden * f->d.n * f->d.n; }

// dynamic LDS of k_fno_row<256>: the spectral branch's row for half the
// channels, eight transform buffers
constexpr size_t kRowLds = (size_t)(kRowC / 2) * (256 + 16) * 4 + 8ull * (256 + 16 + 1) * sizeof(cf);

// One layer's spectral inverse and 1x1 convolution fused per row (k_fno_row)
// when its shapes fit: 64 channels, 256 points per row, 16-byte aligned
// weights.  Returns false when the unfused kernels must run.
bool layer_row(swense_fno* f, const unsigned short* W, const float* in, float* out, int B, const float* bias,
               float* zout, cf* xn) {
  const auto& d = f->d;
  if (d.channels != kRowC || d.n != 256 || !aligned(W, 16) || !aligned(f->xi, 8)) return false;
  const FnoDims dd{256, d.channels, d.p_modes, d.q_modes, B};
  hipLaunchKernelGGL(k_fno_row<256>, dim3((unsigned)(B * 256 * 2)), dim3(512), kRowLds, f->st, f->xi, in, W, bias, out, zout,
                     xn, dd, f->plan);
  SW_HIP(hipGetLastError());
  return true;
}

// keep: store the pre-activations a backward pass needs (an inference call
// skips those writes and leaves no forward for a backward to follow)
void forward_impl(swense_fno* f, const float* x, float* y, int B, bool keep = true) {
  const auto& d = f->d;
  const int C = d.channels, H = d.hidden;
  float* tS = f->tmp + (size_t)d.max_batch * std::max(H, C) * d.n * d.n;
  conv1x1(f, f->wb + f->oW0, C, d.in_channels, x, v_of(f, 0), B, f->w + f->ob0);
  for (int l = 1; l <= d.layers; ++l) {
    const float* v = v_of(f, l - 1);
    cf* U = f->U + (size_t)(l - 1) * d.max_batch * (2 * d.q_modes + 1) * d.p_modes * C;
    if (f->fuse_rows && l > 1) {
      // the x modes of this layer's input came with the previous layer's rows
      const FnoDims dd{d.n, C, d.p_modes, d.q_modes, B};
      const size_t lds = 4ull * wbuf_len(d.n) * sizeof(cf);
      hipLaunchKernelGGL(k_fno_fy<256>, dim3((B * C * d.p_modes + 3) / 4), dim3(256), lds, f->st, f->xi2, U, dd,
                         f->plan, 1.f / ((float)d.n * d.n), 0);
      SW_HIP(hipGetLastError());
    } else {
      spec_fwd(f, v, U, B, 1.f / ((float)d.n * d.n), 0);
    }
    mix(f, U, f->wb + f->oR[l - 1], f->Y, B);
    if (f->fuse_rows) {
      // the y inverse into xi, then the fused x inverse + 1x1 convolution per row
      const FnoDims dd{d.n, C, d.p_modes, d.q_modes, B};
      const size_t lds = 4ull * wbuf_len(d.n) * sizeof(cf);
      hipLaunchKernelGGL(k_fno_iy<256>, dim3((B * C * d.p_modes + 3) / 4), dim3(256), lds, f->st, f->Y, f->xi, dd,
                         f->plan, 1);
      SW_HIP(hipGetLastError());
      if (layer_row(f, f->wb + f->oW[l - 1], v, v_of(f, l), B, f->w + f->ob[l - 1], keep ? z_of(f, l) : nullptr,
                    l < d.layers ? f->xi2 : nullptr))
        continue;
      throw SwenseError{SWENSE_EHIP, "fused layer rows unavailable"};
    }
    spec_inv(f, f->Y, tS, B, 1.f, 0.f, 1);
    conv1x1(f, f->wb + f->oW[l - 1], C, C, v, v_of(f, l), B, f->w + f->ob[l - 1], tS, keep ? z_of(f, l) : nullptr, 1);
  }
  conv1x1(f, f->wb + f->oQ1, H, C, v_of(f, d.layers), h_of(f), B, f->w + f->oc1, nullptr, keep ? zq_of(f) : nullptr, 1);
  conv1x1(f, f->wb + f->oQ2, 2, H, h_of(f), y, B, f->w + f->oc2);
  f->last_batch = keep ? B : 0;
}

void bias_grad(swense_fno* f, const float* g, float* gb, int B, int chans) {
  constexpr int nsplit = 64;
  hipLaunchKernelGGL(k_rowsum_stage, dim3(chans, nsplit), dim3(256), 0, f->st, g, f->rowpart, B, chans,
                     (long long)f->d.n * f->d.n);
  SW_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_reduce_parts, dim3((unsigned)((chans + 255) / 256)), dim3(256), 0, f->st, f->rowpart, nsplit,
                     (long long)chans, gb, 0.f);
  SW_HIP(hipGetLastError());
}

void gelu_back(swense_fno* f, const float* gv, const float* z, float* gz, long long n) {
  hipLaunchKernelGGL(k_fno_gelu_back, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, f->st, gv, z, gz, n);
  SW_HIP(hipGetLastError());
}

// gradients of the loss w.r.t. every parameter (into f->g) given gy; the
// input gradient goes to gx when non-null
void backward_impl(swense_fno* f, const float* x, const float* gy, float* gx, int B) {
  const auto& d = f->d;
  const int C = d.channels, H = d.hidden;
  const long long plane = (long long)d.n * d.n;
  float* gh = f->tmp;  // [B][H] then reused
  float* gv = f->tmp + (size_t)d.max_batch * std::max(H, C) * plane;
  const int S = (2 * d.q_modes + 1) * d.p_modes;
  // projection
  conv1x1_dw(f, gy, h_of(f), 2, H, B, f->g + f->oQ2);
  bias_grad(f, gy, f->g + f->oc2, B, 2);
  conv1x1_dx(f, f->wb + f->oQ2, 2, H, gy, gh, B, 0.f);
  gelu_back(f, gh, zq_of(f), gh, (long long)B * H * plane);
  const size_t cplane = (size_t)B * C * plane;  // one traced [B][C][n][n] block
  auto trace = [&](const float* src, size_t slot, size_t count) {
    if (f->trace)
      SW_HIP(hipMemcpyAsync(f->trace + slot * (size_t)d.max_batch * C * plane, src, count * sizeof(float),
                            hipMemcpyDeviceToDevice, f->st));
  };
  trace(gh, (size_t)d.layers + 1, (size_t)B * H * plane);
  conv1x1_dw(f, gh, v_of(f, d.layers), H, C, B, f->g + f->oQ1);
  bias_grad(f, gh, f->g + f->oc1, B, H);
  conv1x1_dx(f, f->wb + f->oQ1, H, C, gh, gv, B, 0.f);
  float* gz = gh;  // reuse
  cf* gY = f->Y;
  cf* gU = f->Y + (size_t)d.max_batch * S * C;
  for (int l = d.layers; l >= 1; --l) {
    // below the top layer, gz came with the previous iteration's inverse x pass
    if (l == d.layers) gelu_back(f, gv, z_of(f, l), gz, (long long)B * C * plane);
    trace(gz, (size_t)l - 1, cplane);
    const float* u = v_of(f, l - 1);
    conv1x1_dw(f, gz, u, C, C, B, f->g + f->oW[l - 1]);
    bias_grad(f, gz, f->g + f->ob[l - 1], B, C);
    // spectral branch
    spec_fwd(f, gz, gY, B, 1.f, 1);  // c_p n^2 rfft2(gz)/n^2
    herm(f, gY, B, 0);
    const cf* U = f->U + (size_t)(l - 1) * d.max_batch * S * C;
    mix_dw(f, U, gY, f->g + f->oR[l - 1], B);
    mix_dx(f, gY, f->wb + f->oR[l - 1], gU, B);
    // gv = W^T gz + (1/n^2) Re sum P(gU / c_p) e^{ik.x}
    conv1x1_dx(f, f->wb + f->oW[l - 1], C, C, gz, gv, B, 0.f);
    if (l > 1)  // gz of layer l - 1 = gv * gelu'(z_{l-1}), gz's uses above done
      spec_inv(f, gU, gv, B, 1.f / ((float)plane), 1.f, 2, z_of(f, l - 1), gz);
    else
      spec_inv(f, gU, gv, B, 1.f / ((float)plane), 1.f, 2);
  }
  trace(gv, (size_t)d.layers, cplane);
  conv1x1_dw(f, gv, x, C, d.in_channels, B, f->g + f->oW0);
  bias_grad(f, gv, f->g + f->ob0, B, C);
  if (gx) conv1x1_dx(f, f->wb + f->oW0, C, d.in_channels, gv, gx, B, 0.f);
}

float loss_impl(swense_fno* f, const float* y, const float* t, float* gy, int B) {
  const long long plane = (long long)f->d.n * f->d.n;
  hipLaunchKernelGGL(k_fno_loss_sums, dim3(B * 2), dim3(256), 0, f->st, y, t, f->sums, plane);
  SW_HIP(hipGetLastError());
  const long long n = (long long)B * 2 * plane;
  hipLaunchKernelGGL(k_fno_loss_grad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, f->st, y, t, f->sums, gy,
                     plane, n, 1.f / (2.f * B));
  SW_HIP(hipGetLastError());
  std::vector<float> s(4 * B);
  SW_HIP(hipMemcpyAsync(s.data(), f->sums, 4 * B * sizeof(float), hipMemcpyDeviceToHost, f->st));
  SW_HIP(hipStreamSynchronize(f->st));
  double L = 0.0;
  for (int i = 0; i < 2 * B; ++i) L += s[2 * i] / s[2 * i + 1];
  return (float)(L / (2.0 * B));
}

template <typename F>
int guarded_f(swense_fno* f, F&& fn) {
  try {
    return fn();
  } catch (const SwenseError& e) {
    if (f) f->err = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    if (f) f->err = e.what();
    return SWENSE_EHIP;
  }
}

}  // namespace

hipStream_t fno_stream(const swense_fno* f) { return f->st; }
swense_fno_desc fno_desc_of(const swense_fno* f) { return f->d; }

// The network's output only, for callers inside the library that never
// take a gradient (the surrogate's calls).
__attribute__((visibility("hidden"))) int fno_forward_infer(swense_fno* f, const float* x, float* y, int batch) {
  if (!f || !x || !y) return SWENSE_EINVAL;
  return guarded_f(f, [&] {
    SW_REQUIRE(batch >= 1 && batch <= f->d.max_batch, "batch outside [1, max_batch]");
    forward_impl(f, x, y, batch, false);
    return (int)SWENSE_OK;
  });
}

extern "C" {

size_t swense_fno_param_count(const swense_fno_desc* d) { return d ? count_params(*d) : 0; }

int swense_fno_create(const swense_fno_desc* d, const float* params, void* stream, swense_fno** out) {
  if (!out) return SWENSE_EINVAL;
  *out = nullptr;
  swense_fno* f = new swense_fno();
  int rc = guarded_f(f, [&] {
    check_fno_desc(d);
    SW_REQUIRE(params != nullptr, "null parameters");
    f->d = *d;
    f->st = reinterpret_cast<hipStream_t>(stream);
    layout(f);
    SW_REQUIRE(f->nparam == count_params(*d), "internal layout mismatch");
    f->plan = make_wplan(f->tw.get(d->n, false));
    allocate_fno(f);
    f->fuse_rows = d->channels == kRowC && d->n == 256 && aligned(f->xi, 8) && f->xi2 != nullptr;
    for (int l = 0; l < d->layers; ++l) f->fuse_rows = f->fuse_rows && aligned(f->wb + f->oW[l], 16);
    if (f->fuse_rows)
      SW_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fno_row<256>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)kRowLds));
    SW_HIP(hipMemcpy(f->w, params, f->nparam * 4, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((f->nparam + 255) / 256)), dim3(256), 0, f->st, f->w, f->wb,
                       (long long)f->nparam);
    SW_HIP(hipGetLastError());
    SW_HIP(hipStreamSynchronize(f->st));
    return (int)SWENSE_OK;
  });
  if (rc != SWENSE_OK) {
    swense_fno_destroy(f);
    return rc;
  }
  *out = f;
  return SWENSE_OK;
}

int swense_fno_forward(swense_fno* f, const float* x, float* y, int batch) {
  if (!f || !x || !y) return SWENSE_EINVAL;
  return guarded_f(f, [&] {
    SW_REQUIRE(batch >= 1 && batch <= f->d.max_batch, "batch outside [1, max_batch]");
    forward_impl(f, x, y, batch);
    return (int)SWENSE_OK;
  });
}

int swense_fno_backward(swense_fno* f, const float* x, const float* gy, float* gx, int batch) {
  if (!f || !x || !gy) return SWENSE_EINVAL;
  return guarded_f(f, [&] {
    SW_REQUIRE(batch == f->last_batch, "backward must follow a forward of the same batch");
    backward_impl(f, x, gy, gx, batch);
    return (int)SWENSE_OK;
  });
}

int swense_fno_loss(swense_fno* f, const float* y, const float* t, float* gy, int batch, float* loss) {
  if (!f || !y || !t || !gy) return SWENSE_EINVAL;
  return guarded_f(f, [&] {
    SW_REQUIRE(batch >= 1 && batch <= f->d.max_batch, "batch outside [1, max_batch]");
    const float L = loss_impl(f, y, t, gy, batch);
    if (loss) *loss = L;
    return (int)SWENSE_OK;
  });
}

int swense_fno_train_step(swense_fno* f, const float* x, const float* t, int batch, float lr, float* loss) {
  if (!f || !x || !t) return SWENSE_EINVAL;
  return guarded_f(f, [&] {
    SW_REQUIRE(batch >= 1 && batch <= f->d.max_batch, "batch outside [1, max_batch]");
    const long long plane = (long long)f->d.n * f->d.n;
    float* y = h_of(f) + (size_t)f->d.max_batch * f->d.hidden * plane;
    float* gy = y + (size_t)f->d.max_batch * 2 * plane;
    forward_impl(f, x, y, batch);
    const float L = loss_impl(f, y, t, gy, batch);
    backward_impl(f, x, gy, nullptr, batch);
    f->adam_t++;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)f->adam_t), c2 = 1.f - std::pow(b2, (float)f->adam_t);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((f->nparam + 255) / 256)), dim3(256), 0, f->st, f->w, f->wb, f->g,
                       f->am, f->av, (long long)f->nparam, lr, b1, b2, 1e-8f, c1, c2);
    SW_HIP(hipGetLastError());
    if (loss) *loss = L;
    return (int)SWENSE_OK;
  });
}

int swense_fno_get(swense_fno* f, int what, float* host) {
  if (!f || !host) return SWENSE_EINVAL;
  return guarded_f(f, [&] {
    SW_REQUIRE(what >= 0 && what <= 3, "what must be 0..3");
    const float* src = what == 0 ? f->w : what == 1 ? f->g : what == 2 ? f->am : f->av;
    SW_HIP(hipStreamSynchronize(f->st));
    SW_HIP(hipMemcpy(host, src, f->nparam * 4, hipMemcpyDeviceToHost));
    return (int)SWENSE_OK;
  });
}

int swense_fno_get_activations(swense_fno* f, float* host) {
  if (!f || !host) return SWENSE_EINVAL;
  return guarded_f(f, [&] {
    SW_REQUIRE(f->last_batch >= 1, "no forward pass yet");
    const size_t B = f->last_batch, plane = (size_t)f->d.n * f->d.n;
    const size_t cblk = B * f->d.channels * plane, hblk = B * f->d.hidden * plane;
    SW_HIP(hipStreamSynchronize(f->st));
    float* o = host;
    for (int l = 0; l <= f->d.layers; ++l, o += cblk) SW_HIP(hipMemcpy(o, v_of(f, l), cblk * 4, hipMemcpyDeviceToHost));
    for (int l = 1; l <= f->d.layers; ++l, o += cblk) SW_HIP(hipMemcpy(o, z_of(f, l), cblk * 4, hipMemcpyDeviceToHost));
    SW_HIP(hipMemcpy(o, zq_of(f), hblk * 4, hipMemcpyDeviceToHost));
    SW_HIP(hipMemcpy(o + hblk, h_of(f), hblk * 4, hipMemcpyDeviceToHost));
    return (int)SWENSE_OK;
  });
}

int swense_fno_set_trace(swense_fno* f, float* trace) {
  if (!f) return SWENSE_EINVAL;
  f->trace = trace;
  return SWENSE_OK;
}

int swense_fno_set(swense_fno* f, int what, const float* host) {
  if (!f || !host) return SWENSE_EINVAL;
  return guarded_f(f, [&] {
    SW_REQUIRE(what == 0 || what == 2 || what == 3, "what must be 0, 2 or 3");
    SW_HIP(hipStreamSynchronize(f->st));
    float* dst = what == 0 ? f->w : (what == 2 ? f->am : f->av);
    SW_HIP(hipMemcpy(dst, host, f->nparam * 4, hipMemcpyHostToDevice));
    if (what == 0) {
      hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((f->nparam + 255) / 256)), dim3(256), 0, f->st, f->w, f->wb,
                         (long long)f->nparam);
      SW_HIP(hipGetLastError());
      SW_HIP(hipStreamSynchronize(f->st));
    }
    return (int)SWENSE_OK;
  });
}

int swense_gemm_bf16(int M, int N, int K, const float* A, const float* B, float* C, void* stream) {
  if (!A || !B || !C || M < 1 || N < 1 || K < 1) return SWENSE_EINVAL;
  try {
    GemmArgs g = gemm0();
    g.M = M;
    g.N = N;
    g.K = K;
    g.A = A;
    g.sAm = K;
    g.sAk = 1;
    g.B = B;
    g.sBk = N;
    g.sBn = 1;
    g.C = C;
    g.sCm = N;
    g.sCn = 1;
    launch_gemm(reinterpret_cast<hipStream_t>(stream), g);
  } catch (const SwenseError& e) {
    return e.code;
  }
  return SWENSE_OK;
}

const char* swense_fno_last_error(const swense_fno* f) { return f ? f->err.c_str() : "no handle"; }

void swense_fno_destroy(swense_fno* f) {
  if (!f) return;
  if (f->mem) (void)hipFree(f->mem);
  f->tw.release();
  delete f;
}

}  // extern "C"
