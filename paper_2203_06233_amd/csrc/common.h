// Shared definitions of the gfx950 STAP kernels: problem dimensions, complex
// helpers, MFMA vector types and compile-time twiddle tables.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "stap.h"

namespace stap {

// The thread index as the solve code reads it.  By default threadIdx.x is
// passed through an empty volatile asm statement: the dozens of per-lane
// offsets derived from it are then recomputed where they are used instead
// of being computed once and kept live in registers across the whole kernel
// (or, in a persistent kernel, across every system it takes), which the
// register allocator otherwise pays for with spills.  Where keeping them
// live measures faster (the 8-wave one-cube fused kernels, the one-wave
// solve), the translation unit defines STAP_TID_DIRECT before any include.
__device__ __forceinline__ int lane_tid() {
#ifdef STAP_TID_DIRECT
  return (int)threadIdx.x;
#else
  int t;
  asm volatile("" : "=v"(t) : "0"((int)threadIdx.x));
  return t;
#endif
}


constexpr int kMaxDof = 192;
constexpr int kMaxSteer = 64;
constexpr int kMaxTdof = 4;
constexpr int kMinPulse = 32;
constexpr int kMaxPulse = 512;
constexpr int kMaxCfarRef = 64;    // CA-CFAR reference cells per side
constexpr int kMaxCfarGuard = 64;  // CA-CFAR guard cells per side

// Problem dimensions as the kernels see them (all derived on the host).
struct Dims {
  int C, P, R, T, B, S;
  int D;   // T*C, degrees of freedom
  int N;   // R/B, range cells per training block
  int L;   // P-T+1, sub-CPI (window) length
  float eps;
  int prec, refine;
  long long sc, sp;  // cube strides of channel and pulse (elements)
  int train;         // stap_training
  int guard;         // guard cells per side (STAP_TRAIN_EXCLUDE)
  int tap_rel;       // 1: each tap's DFT referenced to its own first pulse
  int steer_bin;     // 1: steering vectors given per Doppler bin, [P][S][D]
  int sub;           // array elements summed into each channel C (>= 1)
};

// The N range cells that train block b, as two runs: cells a0 .. a0+nl-1 and
// a1 .. a1+(N-nl)-1.  Block mode: the block itself.  Exclude mode: the block
// and G guard cells per side are skipped; the nearest remaining cells are
// taken, floor(N/2) on the left and the rest on the right, shifted to the
// other side where the cube ends (the host has checked that N cells exist).
struct CellMap {
  int a0, nl, a1;
  __host__ __device__ int cell(int c) const { return c < nl ? a0 + c : a1 + (c - nl); }
};
__host__ __device__ inline CellMap train_cells(const Dims& d, int b) {
  if (!d.train) return CellMap{b * d.N, d.N, 0};
  const int lo = b * d.N - d.guard, hi = b * d.N + d.N + d.guard;
  const int left = lo > 0 ? lo : 0, right = d.R - hi > 0 ? d.R - hi : 0;
  const int want_left = d.N / 2 < left ? d.N / 2 : left;
  const int nr = d.N - want_left < right ? d.N - want_left : right;
  const int nl = d.N - nr;
  return CellMap{lo - nl, nl, hi};
}

// Steering set of system sys (bin sys / B): the shared V[S][D] or the bin's
// slice of V[P][S][D].
__host__ __device__ inline long long steer_offset(const Dims& d, long long sys) {
  return d.steer_bin ? (sys / d.B) * (long long)d.S * d.D : 0;
}

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));

struct cf {
  float re, im;
};

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// Streaming stores for outputs that are written once and read back by a
// later kernel (not by this one).
__device__ __forceinline__ void store_stream(float2* p, float2 v) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  const f2v x = {v.x, v.y};
  __builtin_nontemporal_store(x, reinterpret_cast<f2v*>(p));
}
__device__ __forceinline__ void store_stream(float* p, float v) { __builtin_nontemporal_store(v, p); }
// A read of data that is used once (streamed past the caches' retention).
__device__ __forceinline__ float2 load_stream(const float2* p) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  const f2v x = __builtin_nontemporal_load(reinterpret_cast<const f2v*>(p));
  return make_float2(x.x, x.y);
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// ---------------------------------------------------------------------------
// Compile-time twiddles exp(-2 pi i j / 64), j = 0..63, evaluated in double by
// the compiler (Taylor series after reduction to [-pi, pi]) and rounded once
// to float.  In-register FFTs of size M <= 64 read W_M^j = W_64^(j*64/M).
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double taylor_sin(double x) {
  double term = x, sum = x;
  for (int n = 1; n < 30; ++n) {
    term *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int n = 1; n < 30; ++n) {
    term *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
    sum += term;
  }
  return sum;
}
struct Tw64 {
  float c[64];
  float s[64];
};
constexpr Tw64 make_tw64() {
  Tw64 t{};
  for (int j = 0; j < 64; ++j) {
    int jj = j > 32 ? j - 64 : j;  // angle in [-pi, pi]
    double a = 2.0 * kPi * jj / 64.0;
    t.c[j] = (float)taylor_cos(a);
    t.s[j] = (float)taylor_sin(a);
  }
  return t;
}

// Correctly rounded tables, evaluated by the compiler in double.
//   Tw<P>:  exp(-2 pi i m / P) = c[m] - i s[m], m = 0..P-1 (exact octant
//           reduction in integers, Taylor series on [0, pi/4]).
//   Win<P>: symmetric Hann window of length L = P - T + 1 for T = 1..4,
//           h[T-1][n] = sin^2(pi n / (L-1)) for n < L, 0 beyond.
constexpr double taylor_sin_small(double x) {
  double term = x, sum = x;
  for (int n = 1; n < 16; ++n) {
    term *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos_small(double x) {
  double term = 1.0, sum = 1.0;
  for (int n = 1; n < 16; ++n) {
    term *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
    sum += term;
  }
  return sum;
}
// cos and sin of 2 pi m / P
constexpr void sincos_frac(long long m, long long P, double& c, double& s) {
  long long q4 = ((4 * m) / P) % 4;
  long long rem = (4 * m) % P;  // angle in quadrant = (pi/2) rem / P
  double cc, ss;
  if (2 * rem <= P) {
    const double psi = (kPi / 2.0) * (double)rem / (double)P;
    cc = taylor_cos_small(psi);
    ss = taylor_sin_small(psi);
  } else {
    const double psi = (kPi / 2.0) * (double)(P - rem) / (double)P;
    cc = taylor_sin_small(psi);
    ss = taylor_cos_small(psi);
  }
  if (q4 == 0) { c = cc; s = ss; }
  else if (q4 == 1) { c = -ss; s = cc; }
  else if (q4 == 2) { c = -cc; s = -ss; }
  else { c = ss; s = -cc; }
}
template <int P>
struct TwTab {
  float c[P];
  float s[P];
};
template <int P>
constexpr TwTab<P> make_twtab() {
  TwTab<P> t{};
  for (int m = 0; m < P; ++m) {
    double c = 0, s = 0;
    sincos_frac(m, P, c, s);
    t.c[m] = (float)c;
    t.s[m] = (float)s;
  }
  return t;
}
template <int P>
struct WinTab {
  float h[4][P];
};
template <int P>
constexpr WinTab<P> make_wintab() {
  WinTab<P> w{};
  for (int t = 0; t < 4; ++t) {
    const int L = P - t;
    for (int n = 0; n < P; ++n) {
      double v = 0.0;
      if (n < L && L > 1) {
        // theta = pi n/(L-1) folded to [0, pi/2] with exact integer arithmetic
        const int nn = (2 * n <= L - 1) ? n : (L - 1 - n);
        double c = 0, s = 0;
        sincos_frac(nn, 2LL * (L - 1), c, s);  // angle 2 pi nn / (2(L-1)) = pi nn/(L-1)
        v = s * s;
      }
      w.h[t][n] = (float)v;
    }
  }
  return w;
}
template <int P>
__device__ const TwTab<P> kTwTab = make_twtab<P>();
template <int P>
__device__ const WinTab<P> kWinTab = make_wintab<P>();

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }
constexpr int bitrev(int v, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r |= ((v >> i) & 1) << (bits - 1 - i);
  return r;
}

// Forward DFT of M points held in registers, natural order in and out:
// v[k] <- sum_n v[n] exp(-2 pi i k n / M).  Radix-2 decimation in time; all
// indices and twiddles are compile-time constants after unrolling.
template <int M>
__device__ __forceinline__ void fft_inreg(float2 (&v)[M]) {
  constexpr int LOG = ilog2(M);
  constexpr Tw64 tw = make_tw64();
#pragma unroll
  for (int i = 0; i < M; ++i) {
    const int j = bitrev(i, LOG);
    if (j > i) {
      float2 t = v[i];
      v[i] = v[j];
      v[j] = t;
    }
  }
#pragma unroll
  for (int half = 1; half < M; half *= 2) {
#pragma unroll
    for (int start = 0; start < M; start += 2 * half) {
#pragma unroll
      for (int j = 0; j < half; ++j) {
        const int idx = j * (64 / (2 * half));
        const float2 w = make_float2(tw.c[idx], -tw.s[idx]);
        const float2 a = v[start + j];
        const float2 c = v[start + j + half];
        // idx 0 and 16 are the twiddles 1 and -i (a swap and a sign, exact);
        // products with 0 and +-1 are not folded under IEEE rules, so they
        // are taken apart here (idx is a constant after unrolling)
        const float2 b = (idx == 0) ? c : (idx == 16) ? make_float2(c.y, -c.x) : cmul(c, w);
        v[start + j] = cadd(a, b);
        v[start + j + half] = csub(a, b);
      }
    }
  }
}

// Forward DFT of M points held in registers for M that is not a power of
// two: v[k] <- sum_n v[n] exp(-2 pi i k n / M), evaluated directly with a
// correctly rounded compile-time table (M^2 complex products; used for the
// factors of the 100-pulse transform).
template <int M>
__device__ __forceinline__ void dft_inreg(float2 (&v)[M]) {
  constexpr TwTab<M> tw = make_twtab<M>();
  float2 out[M];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    float2 acc = v[0];
#pragma unroll
    for (int n = 1; n < M; ++n) {
      const int m = (k * n) % M;
      const float c = tw.c[m], sn = -tw.s[m];  // exp(-2 pi i m / M) = c + i sn
      acc.x = fmaf(v[n].x, c, fmaf(-v[n].y, sn, acc.x));
      acc.y = fmaf(v[n].x, sn, fmaf(v[n].y, c, acc.y));
    }
    out[k] = acc;
  }
#pragma unroll
  for (int k = 0; k < M; ++k) v[k] = out[k];
}

template <int M>
__device__ __forceinline__ void dft_any(float2 (&v)[M]) {
  if constexpr ((M & (M - 1)) == 0) fft_inreg<M>(v);
  else dft_inreg<M>(v);
}

// Round-to-nearest-even float -> bf16 bits, and back.
__device__ __forceinline__ uint4 negbf8(uint4 u) {
  return make_uint4(u.x ^ 0x80008000u, u.y ^ 0x80008000u, u.z ^ 0x80008000u, u.w ^ 0x80008000u);
}

// Three-term BF16 split of two floats at once, packed in pairs (a in the low
// half): x = h + m + l to 24 bits, each term rounded to nearest even by the
// hardware pair conversion (v_cvt_pk_bf16_f32); each residual is exact in
// FP32, so the products of terms are exact in FP32.
__device__ __forceinline__ void split3x2(float a, float b, unsigned int& h, unsigned int& m, unsigned int& l) {
  typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
  typedef float f32x2v __attribute__((ext_vector_type(2)));
  const f32x2v x = {a, b};
  const bf16x2v hb = __builtin_convertvector(x, bf16x2v);
  h = __builtin_bit_cast(unsigned int, hb);
  const f32x2v r1 = {a - __uint_as_float(h << 16), b - __uint_as_float(h & 0xFFFF0000u)};
  const bf16x2v mb = __builtin_convertvector(r1, bf16x2v);
  m = __builtin_bit_cast(unsigned int, mb);
  const f32x2v r2 = {r1.x - __uint_as_float(m << 16), r1.y - __uint_as_float(m & 0xFFFF0000u)};
  l = __builtin_bit_cast(unsigned int, __builtin_convertvector(r2, bf16x2v));
}
}  // namespace stap
