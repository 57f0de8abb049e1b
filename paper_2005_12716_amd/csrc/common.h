// Shared definitions of the gfx950 incident-wave library: complex type,
// error plumbing, FFT plans and the LDS-resident mixed-radix Stockham FFT
// used by every spectral <-> physical transform of the hot path.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "swense.h"

// ---------------------------------------------------------------- complex
template <typename R>
struct cpx {
  R x, y;
};
using cf = cpx<float>;
using cd = cpx<double>;

template <typename R>
__host__ __device__ __forceinline__ cpx<R> mk(R a, R b) {
  cpx<R> c;
  c.x = a;
  c.y = b;
  return c;
}
template <typename R>
__host__ __device__ __forceinline__ cpx<R> operator+(cpx<R> a, cpx<R> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename R>
__host__ __device__ __forceinline__ cpx<R> operator-(cpx<R> a, cpx<R> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename R>
__host__ __device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename R>
__host__ __device__ __forceinline__ cpx<R> cscale(cpx<R> a, R s) { return mk(a.x * s, a.y * s); }
template <typename R>
__host__ __device__ __forceinline__ cpx<R> conjg(cpx<R> a) { return mk(a.x, -a.y); }
// multiply by sign * i
template <typename R>
__host__ __device__ __forceinline__ cpx<R> mul_si(cpx<R> a, int sign) {
  return sign > 0 ? mk(-a.y, a.x) : mk(a.y, -a.x);
}

// ---------------------------------------------------------------- errors
struct SwenseError {
  int code;
  std::string msg;
};

#define SW_HIP(call)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      throw SwenseError{SWENSE_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)};     \
  } while (0)

#define SW_REQUIRE(cond, msg)                                        \
  do {                                                               \
    if (!(cond)) throw SwenseError{SWENSE_EINVAL, std::string(msg)}; \
  } while (0)

// ---------------------------------------------------------------- FFT plan
// A length n = product of radices (8, 4, 2, 3, 5) and a device table of
// exp(-2 pi i m / n), m < n, computed in FP64 and rounded to the transform's
// precision.  Plans are small and passed to kernels by value.
constexpr int kMaxRad = 16;

struct FftPlan {
  int n;
  int nrad;
  int rad[kMaxRad];
  const void* tw;
};

inline bool is_235_smooth(int n) {
  if (n < 1) return false;
  for (int f : {2, 3, 5})
    while (n % f == 0) n /= f;
  return n == 1;
}

inline std::vector<int> factor_radices(int n) {
  std::vector<int> r;
  while (n % 8 == 0) { r.push_back(8); n /= 8; }
  while (n % 4 == 0) { r.push_back(4); n /= 4; }
  while (n % 2 == 0) { r.push_back(2); n /= 2; }
  while (n % 3 == 0) { r.push_back(3); n /= 3; }
  while (n % 5 == 0) { r.push_back(5); n /= 5; }
  return r;
}

// Twiddle-table cache owned by a handle (device memory, freed with it).
struct TwiddleCache {
  std::map<std::pair<int, int>, void*> tables;  // (n, bytes per complex)
  // caller-owned memory tables may be carved from (not freed by release)
  char* arena = nullptr;
  size_t arena_left = 0;
  std::vector<void*> borrowed;
  static size_t table_bytes(int n, bool fp64) { return ((size_t)n * (fp64 ? sizeof(cd) : sizeof(cf)) + 255) & ~size_t(255); }
  // The table exp(-2 pi i m / n), m < n, written to caller memory `dst`
  // (synchronous copy), and its plan.
  static FftPlan fill(int n, bool fp64, void* dst) {
    FftPlan p{};
    p.n = n;
    auto rs = factor_radices(n);
    SW_REQUIRE((int)rs.size() <= kMaxRad, "transform length has too many factors");
    p.nrad = (int)rs.size();
    for (int i = 0; i < p.nrad; ++i) p.rad[i] = rs[i];
    if (fp64) {
      std::vector<cd> h(n);
      for (int m = 0; m < n; ++m) h[m] = mk(std::cos(-2.0 * M_PI * m / n), std::sin(-2.0 * M_PI * m / n));
      SW_HIP(hipMemcpy(dst, h.data(), (size_t)n * sizeof(cd), hipMemcpyHostToDevice));
    } else {
      std::vector<cf> h(n);
      for (int m = 0; m < n; ++m)
        h[m] = mk((float)std::cos(-2.0 * M_PI * m / n), (float)std::sin(-2.0 * M_PI * m / n));
      SW_HIP(hipMemcpy(dst, h.data(), (size_t)n * sizeof(cf), hipMemcpyHostToDevice));
    }
    p.tw = dst;
    return p;
  }
  static FftPlan plan_with(int n, void* tw) {
    FftPlan p{};
    p.n = n;
    auto rs = factor_radices(n);
    p.nrad = (int)rs.size();
    for (int i = 0; i < p.nrad; ++i) p.rad[i] = rs[i];
    p.tw = tw;
    return p;
  }
  FftPlan get(int n, bool fp64) {
    FftPlan p{};
    p.n = n;
    auto rs = factor_radices(n);
    SW_REQUIRE((int)rs.size() <= kMaxRad, "transform length has too many factors");
    p.nrad = (int)rs.size();
    for (int i = 0; i < p.nrad; ++i) p.rad[i] = rs[i];
    auto key = std::make_pair(n, fp64 ? 16 : 8);
    auto it = tables.find(key);
    if (it == tables.end()) {
      void* d = nullptr;
      size_t bytes = (size_t)n * (fp64 ? sizeof(cd) : sizeof(cf));
      if (arena && table_bytes(n, fp64) <= arena_left) {
        d = arena;
        arena += table_bytes(n, fp64);
        arena_left -= table_bytes(n, fp64);
        borrowed.push_back(d);
      } else {
        SW_HIP(hipMalloc(&d, bytes));
      }
      if (fp64) {
        std::vector<cd> h(n);
        for (int m = 0; m < n; ++m) {
          double a = -2.0 * M_PI * (double)m / (double)n;
          h[m] = mk(std::cos(a), std::sin(a));
        }
        SW_HIP(hipMemcpy(d, h.data(), bytes, hipMemcpyHostToDevice));
      } else {
        std::vector<cf> h(n);
        for (int m = 0; m < n; ++m) {
          double a = -2.0 * M_PI * (double)m / (double)n;
          h[m] = mk((float)std::cos(a), (float)std::sin(a));
        }
        SW_HIP(hipMemcpy(d, h.data(), bytes, hipMemcpyHostToDevice));
      }
      it = tables.emplace(key, d).first;
    }
    p.tw = it->second;
    return p;
  }
  bool has(int n, bool fp64) const { return tables.count(std::make_pair(n, fp64 ? 16 : 8)) != 0; }
  void release() {
    for (auto& kv : tables) {
      bool b = false;
      for (void* q : borrowed) b = b || q == kv.second;
      if (!b) (void)hipFree(kv.second);
    }
    tables.clear();
    borrowed.clear();
  }
};

// ---------------------------------------------------------------- radix DFTs
// y[m] = sum_r x[r] exp(sign * 2 pi i r m / R), in place.
template <typename R>
__device__ __forceinline__ void dft2(cpx<R>* v) {
  cpx<R> a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}

template <typename R>
__device__ __forceinline__ void dft3(cpx<R>* v, int sign) {
  const R c = (R)-0.5;
  const R s = (R)0.86602540378443864676;
  cpx<R> s12 = v[1] + v[2];
  cpx<R> d12 = v[1] - v[2];
  cpx<R> t = v[0] + cscale(s12, c);
  cpx<R> u = mul_si(cscale(d12, s), sign);
  v[0] = v[0] + s12;
  v[1] = t + u;
  v[2] = t - u;
}

template <typename R>
__device__ __forceinline__ void dft4(cpx<R>* v, int sign) {
  cpx<R> a = v[0] + v[2], b = v[0] - v[2];
  cpx<R> c = v[1] + v[3], d = mul_si(v[1] - v[3], sign);
  v[0] = a + c;
  v[2] = a - c;
  v[1] = b + d;
  v[3] = b - d;
}

template <typename R>
__device__ __forceinline__ void dft5(cpx<R>* v, int sign) {
  const R c1 = (R)0.30901699437494742410;   // cos(2 pi / 5)
  const R c2 = (R)-0.80901699437494742410;  // cos(4 pi / 5)
  const R s1 = (R)0.95105651629515357212;   // sin(2 pi / 5)
  const R s2 = (R)0.58778525229247312917;   // sin(4 pi / 5)
  cpx<R> a14 = v[1] + v[4], d14 = v[1] - v[4];
  cpx<R> a23 = v[2] + v[3], d23 = v[2] - v[3];
  cpx<R> t1 = v[0] + cscale(a14, c1) + cscale(a23, c2);
  cpx<R> t2 = v[0] + cscale(a14, c2) + cscale(a23, c1);
  cpx<R> u1 = mul_si(cscale(d14, s1) + cscale(d23, s2), sign);
  cpx<R> u2 = mul_si(cscale(d14, s2) - cscale(d23, s1), sign);
  v[0] = v[0] + a14 + a23;
  v[1] = t1 + u1;
  v[4] = t1 - u1;
  v[2] = t2 + u2;
  v[3] = t2 - u2;
}

template <typename R>
__device__ __forceinline__ void dft8(cpx<R>* v, int sign) {
  cpx<R> e[4] = {v[0], v[2], v[4], v[6]};
  cpx<R> o[4] = {v[1], v[3], v[5], v[7]};
  dft4(e, sign);
  dft4(o, sign);
  const R h = (R)0.70710678118654752440;
  // w^m = exp(sign i pi m / 4)
  cpx<R> o1 = cmul(o[1], mk(h, sign * h));
  cpx<R> o2 = mul_si(o[2], sign);
  cpx<R> o3 = cmul(o[3], mk(-h, sign * h));
  v[0] = e[0] + o[0];
  v[4] = e[0] - o[0];
  v[1] = e[1] + o1;
  v[5] = e[1] - o1;
  v[2] = e[2] + o2;
  v[6] = e[2] - o2;
  v[3] = e[3] + o3;
  v[7] = e[3] - o3;
}

// One Stockham (self-sorting) radix-RAD pass over nseq sequences of length n,
// each at src + s * n, writing to dst.  Ns = product of the radices of the
// previous passes.  Butterfly j reads x[j + r n/RAD], twiddles by
// exp(sign 2 pi i (j mod Ns) r / (Ns RAD)), and writes positions
// (j div Ns) Ns RAD + (j mod Ns) + r Ns.
template <typename R, int RAD>
__device__ __forceinline__ void stockham_pass(const cpx<R>* __restrict__ src, cpx<R>* __restrict__ dst, int n,
                                              int Ns, int nseq, const cpx<R>* __restrict__ tw, int sign,
                                              int tid, int nthr) {
  const int nb = n / RAD;
  const int total = nb * nseq;
  const int twstep = n / (Ns * RAD);
  for (int t = tid; t < total; t += nthr) {
    const int s = t / nb;
    const int j = t - s * nb;
    const int k = j % Ns;
    const cpx<R>* in = src + (size_t)s * n;
    cpx<R> v[RAD];
#pragma unroll
    for (int r = 0; r < RAD; ++r) {
      cpx<R> x = in[j + r * nb];
      if (r > 0 && k > 0) {
        cpx<R> w = tw[k * r * twstep];
        if (sign > 0) w.y = -w.y;
        x = cmul(x, w);
      }
      v[r] = x;
    }
    if (RAD == 2) dft2(v);
    else if (RAD == 3) dft3(v, sign);
    else if (RAD == 4) dft4(v, sign);
    else if (RAD == 5) dft5(v, sign);
    else if (RAD == 8) dft8(v, sign);
    cpx<R>* out = dst + (size_t)s * n + (j / Ns) * Ns * RAD + k;
#pragma unroll
    for (int r = 0; r < RAD; ++r) out[r * Ns] = v[r];
  }
}

// Full transform of nseq contiguous sequences of length plan.n held in LDS
// buffer a (b is scratch of the same size).  Returns the buffer that holds
// the result.  Unnormalised; sign -1 forward, +1 inverse.  Must be called by
// every thread of the block (it synchronises between passes).
template <typename R>
__device__ cpx<R>* block_fft(cpx<R>* a, cpx<R>* b, const FftPlan& plan, int nseq, int sign) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  const cpx<R>* tw = (const cpx<R>*)plan.tw;
  cpx<R>* src = a;
  cpx<R>* dst = b;
  int Ns = 1;
  for (int p = 0; p < plan.nrad; ++p) {
    const int rad = plan.rad[p];
    switch (rad) {
      case 8: stockham_pass<R, 8>(src, dst, plan.n, Ns, nseq, tw, sign, tid, nthr); break;
      case 4: stockham_pass<R, 4>(src, dst, plan.n, Ns, nseq, tw, sign, tid, nthr); break;
      case 2: stockham_pass<R, 2>(src, dst, plan.n, Ns, nseq, tw, sign, tid, nthr); break;
      case 3: stockham_pass<R, 3>(src, dst, plan.n, Ns, nseq, tw, sign, tid, nthr); break;
      default: stockham_pass<R, 5>(src, dst, plan.n, Ns, nseq, tw, sign, tid, nthr); break;
    }
    __syncthreads();
    Ns *= rad;
    cpx<R>* t = src;
    src = dst;
    dst = t;
  }
  return const_cast<cpx<R>*>(src);
}

// ---------------------------------------------------------------- geometry
// Mode grid and physical constants as seen by the kernels.
struct Geom {
  int nx, ny, nxh;
  double lx, ly;
  double depth;  // <= 0: infinite
  double g, rho;
};

__host__ __device__ __forceinline__ int signed_q(int q, int ny) { return (ny > 1 && q >= ny / 2) ? q - ny : q; }

// Vertical factors C = cosh k(z+h)/cosh kh and S = sinh k(z+h)/cosh kh in the
// overflow-safe form (e^{kz} +- e^{-k(z+2h)}) / (1 + e^{-2kh}); e^{kz} in deep water.
__device__ __forceinline__ void vfactors(double k, double z, double depth, double& C, double& S) {
  if (!(depth > 0.0)) {
    C = S = exp(k * z);
    return;
  }
  double a = exp(k * z);
  double b = exp(-k * (z + 2.0 * depth));
  double d = 1.0 + exp(-2.0 * k * depth);
  C = (a + b) / d;
  S = (a - b) / d;
}
