// Per-system sample covariance on MFMA, shared by the stage covariance kernel
// and the fused covariance->solve kernel.
//
//   R_hat = (1/N) X_kb X_kb^H,   Re R = Xr Xr^T + Xi Xi^T,   Im R = Xi Xr^T - Xr Xi^T.
//
// 16x16 output tiles of the lower block triangle are spread over the NW waves
// of the workgroup; range cells are staged through LDS in chunks of 32.
//   MODE 0 (FP32)  v_mfma_f32_16x16x4_f32 on the complex64 snapshots, three
//                  real products per complex product (Gauss) up to 128 DOF,
//                  four beyond, accumulated separately within a chunk.
//   MODE 1 (BF16)  every FP32 component is split exactly into three BF16
//                  terms x = h + m + l; the six products hh, hm, mh, hl, lh, mm
//                  run on v_mfma_f32_16x16x32_bf16 with FP32 accumulation, hh
//                  in its own accumulator: FP32-level error at 6/16 of the
//                  FP32-MFMA cost.
//   MODE 2 (FP8)   components scaled by a power of two per system (largest
//                  magnitude mapped into [128, 256)), rounded to OCP E4M3, one
//                  product per element on v_mfma_f32_16x16x32_fp8_fp8.
#pragma once

#include "common.h"

namespace stap {

constexpr int kCovChunk = 32;

template <int DP_, int NW_, int MODE_>
struct CovCfg {
  static constexpr int DP = DP_, NW = NW_, MODE = MODE_;
  static constexpr int NT = NW * 64;
  static constexpr int TB = DP / 16;
  static constexpr int NTILE = TB * (TB + 1) / 2;
  static constexpr int TPW = (NTILE + NW - 1) / NW;
  static constexpr int F32_PITCH = kCovChunk + 1;  // float2 units
  static constexpr int BF_PITCH = kCovChunk + 8;   // bf16 units
  static constexpr int F8_PITCH = kCovChunk + 16;  // bytes
  static constexpr int LDS_BYTES = MODE == 0   ? DP * F32_PITCH * 8
                                   : MODE == 1 ? 6 * DP * BF_PITCH * 2
                                               : 2 * DP * F8_PITCH;
};

__device__ __forceinline__ void cov_tile_of(int t, int& I, int& J) {
  int i = 0;
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  I = i;
  J = t - i * (i + 1) / 2;
}

__device__ __forceinline__ floatx4 mfma_bf16(uint4 a, uint4 b, floatx4 c) {
  typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b),
                                                 c, 0, 0, 0);
}

// E4M3 (OCP, finite max 448) round-to-nearest-even with saturation.
__device__ __forceinline__ unsigned int f2e4m3(float x) {
  const unsigned int s = (__float_as_uint(x) >> 24) & 0x80u;
  float a = fabsf(x);
  if (!(a < 448.f)) return s | 0x7Eu;
  if (a < 0.015625f) {                 // subnormal range, step 2^-9
    const float q = rintf(a * 512.f);  // RNE; q = 8 encodes the smallest normal
    return s | (unsigned int)q;
  }
  unsigned int u = __float_as_uint(a);
  u += 0x7FFFFu + ((u >> 20) & 1u);  // RNE to 3 mantissa bits
  const int e = (int)((u >> 23) & 0xFF) - 127 + 7;
  const unsigned int m = (u >> 20) & 0x7u;
  if (e > 15 || (e == 15 && m == 7)) return s | 0x7Eu;
  return s | ((unsigned int)e << 3) | m;
}

// Accumulate R_hat for one system into accR/accI (tile t = wave + NW*i of the
// lower block triangle, MFMA 16x16 layout: lane l holds rows 4(l/16)+r,
// column l%16).  X points at row 0, range cell 0 of the system's Doppler bin
// (row stride rstride); the N training cells are cm.cell(0 .. N-1).  lds
// holds Cfg::LDS_BYTES; red holds NW floats.  Returns with the accumulators
// scaled to R_hat (1/N, FP8 scale undone).
template <class Cfg>
__device__ __forceinline__ void cov_accumulate(const float2* __restrict__ X, long long rstride, int D, int N,
                                               CellMap cm, unsigned char* lds, float* red,
                                               floatx4 (&accR)[Cfg::TPW], floatx4 (&accI)[Cfg::TPW]) {
  constexpr int DP = Cfg::DP, NW = Cfg::NW, MODE = Cfg::MODE, NT = Cfg::NT, TPW = Cfg::TPW;
  constexpr int NTILE = Cfg::NTILE;
  constexpr int F32_PITCH = Cfg::F32_PITCH, BF_PITCH = Cfg::BF_PITCH, F8_PITCH = Cfg::F8_PITCH;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  floatx4 corR[TPW], corI[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    accR[i] = floatx4{0.f, 0.f, 0.f, 0.f};
    accI[i] = accR[i];
    corR[i] = accR[i];
    corI[i] = accR[i];
  }

  float qscale = 1.f;
  if (MODE == 2) {
    float mx = 0.f;
    for (int e = tid; e < D * N; e += NT) {
      const int row = e / N, cc = e - (e / N) * N;
      const float2 v = X[(long long)row * rstride + cm.cell(cc)];
      mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y)));
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    if (lane == 0) red[wave] = mx;
    __syncthreads();
    float m2 = 0.f;
    for (int w = 0; w < NW; ++w) m2 = fmaxf(m2, red[w]);
    int ex = 0;
    if (m2 > 0.f) frexpf(m2, &ex);  // m2 = f 2^ex, f in [0.5, 1)
    qscale = ldexpf(1.f, 8 - ex);     // largest magnitude lands in [128, 256)
  }

  // Staging is double-buffered through registers: the global loads of chunk
  // c + 1 are issued before the products of chunk c, so their latency hides
  // behind the matrix-core work.  MODE 0 / 2: element e = tid + NT i is
  // (row e / 32, cell e % 32); MODE 1: pair e is (row e / 16, cells 2 (e % 16)
  // and 2 (e % 16) + 1).
  constexpr int NE = MODE == 1 ? DP * (kCovChunk / 2) : DP * kCovChunk;
  constexpr int PF = (NE + NT - 1) / NT;
  constexpr int PV = MODE == 1 ? 2 : 1;
  float2 pf[PF][PV];
  // Training cell c lives at lo[c] for c < nl and at hi[c] beyond (both
  // bases workgroup-uniform; in block mode nl = N and only lo is used).  A
  // pair of cells straddles the two runs only at c = nl - 1.
  const float2* const lo = X + cm.a0;
  const float2* const hi = X + (cm.a1 - cm.nl);
  const int nl = cm.nl;
  auto load_chunk = [&](int c0) {
    const int nc = min(kCovChunk, N - c0);
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int e = tid + NT * i;
      if (MODE == 1) {
        const int row = e / (kCovChunk / 2), cp = e % (kCovChunk / 2);
        float2 v0 = make_float2(0.f, 0.f), v1 = v0;
        if (e < NE && row < D) {
          const int c = c0 + 2 * cp;
          const long long ro = (long long)row * rstride + c;
          if (c + 1 != nl) {
            const float2* src = (c < nl ? lo : hi) + ro;
            if (2 * cp < nc) v0 = src[0];
            if (2 * cp + 1 < nc) v1 = src[1];
          } else {
            if (2 * cp < nc) v0 = lo[ro];
            if (2 * cp + 1 < nc) v1 = hi[ro + 1];
          }
        }
        pf[i][0] = v0;
        pf[i][PV - 1] = v1;
      } else {
        const int row = e / kCovChunk, cc = e % kCovChunk;
        float2 v = make_float2(0.f, 0.f);
        const int c = c0 + cc;
        if (e < NE && row < D && cc < nc) v = (c < nl ? lo : hi)[(long long)row * rstride + c];
        pf[i][0] = v;
      }
    }
  };
  auto store_chunk = [&]() {
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int e = tid + NT * i;
      if (e >= NE) continue;
      if (MODE == 0) {
        float2* xs = reinterpret_cast<float2*>(lds);
        xs[(e / kCovChunk) * F32_PITCH + e % kCovChunk] = pf[i][0];
      } else if (MODE == 1) {
        unsigned int* pl = reinterpret_cast<unsigned int*>(lds);
        constexpr int PS = DP * BF_PITCH / 2;  // plane stride, uint32
        const int row = e / (kCovChunk / 2), cp = e % (kCovChunk / 2);
        const float2 v0 = pf[i][0], v1 = pf[i][PV - 1];
        unsigned int h, m, l;
        const int base = row * (BF_PITCH / 2) + cp;
        split3x2(v0.x, v1.x, h, m, l);
        pl[0 * PS + base] = h;
        pl[1 * PS + base] = m;
        pl[2 * PS + base] = l;
        split3x2(v0.y, v1.y, h, m, l);
        pl[3 * PS + base] = h;
        pl[4 * PS + base] = m;
        pl[5 * PS + base] = l;
      } else {
        unsigned char* pl = lds;
        const int row = e / kCovChunk, cc = e % kCovChunk;
        pl[row * F8_PITCH + cc] = (unsigned char)f2e4m3(pf[i][0].x * qscale);
        pl[DP * F8_PITCH + row * F8_PITCH + cc] = (unsigned char)f2e4m3(pf[i][0].y * qscale);
      }
    }
  };

  load_chunk(0);
  for (int c0 = 0; c0 < N; c0 += kCovChunk) {
    const int nc = min(kCovChunk, N - c0);
    __syncthreads();  // the previous chunk's products are done with the staging buffer
    store_chunk();
    __syncthreads();
    if (c0 + kCovChunk < N) load_chunk(c0 + kCovChunk);

#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int t = wave + NW * i;
      if (t < NTILE) {
        int I, J;
        cov_tile_of(t, I, J);
        const int ra = I * 16 + (lane & 15), rb = J * 16 + (lane & 15);
        if (MODE == 0) {
          const float2* xs = reinterpret_cast<const float2*>(lds);
          const int kq = (nc + 3) & ~3;
          floatx4 rr = floatx4{0.f, 0.f, 0.f, 0.f}, ii = rr, tt = rr, ri = rr;
          if constexpr (DP <= 128) {
            // Gauss's three-product form: with A = Xr, B = Xi of the row
            // blocks, T1 = A A^T, T2 = B B^T, T3 = (A + B)(A - B)^T give
            // Re = T1 + T2 and Im = B A^T - A B^T = T3 - T1 + T2
            for (int kk = 0; kk < kq; kk += 4) {
              const float2 a = xs[ra * F32_PITCH + kk + (lane >> 4)];
              const float2 bb = xs[rb * F32_PITCH + kk + (lane >> 4)];
              rr = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, bb.x, rr, 0, 0, 0);
              ii = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, bb.y, ii, 0, 0, 0);
              tt = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x + a.y, bb.x - bb.y, tt, 0, 0, 0);
            }
            accR[i] += rr + ii;
            accI[i] += (tt - rr) + ii;
          } else {
            // four products (T3 would push the 192-DOF tiles over the
            // register budget): tt = B A^T, ri = A B^T
            for (int kk = 0; kk < kq; kk += 4) {
              const float2 a = xs[ra * F32_PITCH + kk + (lane >> 4)];
              const float2 bb = xs[rb * F32_PITCH + kk + (lane >> 4)];
              rr = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, bb.x, rr, 0, 0, 0);
              ii = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, bb.y, ii, 0, 0, 0);
              tt = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, bb.x, tt, 0, 0, 0);
              ri = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, bb.y, ri, 0, 0, 0);
            }
            accR[i] += rr + ii;
            accI[i] += tt - ri;
          }
        } else if (MODE == 1) {
          const uint4* pl = reinterpret_cast<const uint4*>(lds);
          constexpr int PS4 = DP * BF_PITCH / 8;
          const int oa = ra * (BF_PITCH / 8) + (lane >> 4);
          const int ob = rb * (BF_PITCH / 8) + (lane >> 4);
          uint4 A[6], Bv[6];
#pragma unroll
          for (int p = 0; p < 6; ++p) {
            A[p] = pl[p * PS4 + oa];
            Bv[p] = pl[p * PS4 + ob];
          }
          accR[i] = mfma_bf16(A[0], Bv[0], accR[i]);
          accR[i] = mfma_bf16(A[3], Bv[3], accR[i]);
          accI[i] = mfma_bf16(A[3], Bv[0], accI[i]);
          accI[i] = mfma_bf16(negbf8(A[0]), Bv[3], accI[i]);
          constexpr int PA[5] = {0, 1, 0, 2, 1};
          constexpr int PB[5] = {1, 0, 2, 0, 1};
#pragma unroll
          for (int q = 0; q < 5; ++q) {
            corR[i] = mfma_bf16(A[PA[q]], Bv[PB[q]], corR[i]);
            corR[i] = mfma_bf16(A[3 + PA[q]], Bv[3 + PB[q]], corR[i]);
            corI[i] = mfma_bf16(A[3 + PA[q]], Bv[PB[q]], corI[i]);
            corI[i] = mfma_bf16(negbf8(A[PA[q]]), Bv[3 + PB[q]], corI[i]);
          }
        } else {
          const unsigned char* pl = lds;
          const long ar = *reinterpret_cast<const long*>(pl + ra * F8_PITCH + 8 * (lane >> 4));
          const long ai = *reinterpret_cast<const long*>(pl + DP * F8_PITCH + ra * F8_PITCH + 8 * (lane >> 4));
          const long br = *reinterpret_cast<const long*>(pl + rb * F8_PITCH + 8 * (lane >> 4));
          const long bi = *reinterpret_cast<const long*>(pl + DP * F8_PITCH + rb * F8_PITCH + 8 * (lane >> 4));
          const long nar = ar ^ 0x8080808080808080L;
          accR[i] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(ar, br, accR[i], 0, 0, 0);
          accR[i] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(ai, bi, accR[i], 0, 0, 0);
          accI[i] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(ai, br, accI[i], 0, 0, 0);
          accI[i] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(nar, bi, accI[i], 0, 0, 0);
        }
      }
    }
  }

  const float invs2 = (MODE == 2) ? 1.f / (qscale * qscale) : 1.f;
  const float fN = (float)N;
#pragma unroll
  for (int i = 0; i < TPW; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      accR[i][r] = ((accR[i][r] + corR[i][r]) * invs2) / fN;
      accI[i][r] = ((accI[i][r] + corI[i][r]) * invs2) / fN;
    }
}

// delta = eps * Re tr(R_hat) / D with the trace summed in FP64.  dsum holds
// Cfg::DP doubles; every thread returns the same value.
template <class Cfg>
__device__ __forceinline__ float cov_delta(const floatx4 (&accR)[Cfg::TPW], int D, float eps, double* dsum,
                                           float* s_delta) {
  constexpr int NW = Cfg::NW, TPW = Cfg::TPW, NTILE = Cfg::NTILE;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int t = wave + NW * i;
    if (t < NTILE) {
      int I, J;
      cov_tile_of(t, I, J);
      if (I == J) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = I * 16 + 4 * (lane >> 4) + r, col = J * 16 + (lane & 15);
          if (row == col && row < D) dsum[row] = (double)accR[i][r];
        }
      }
    }
  }
  __syncthreads();
  if (wave == 0) {
    double s = 0.0;
    for (int q = lane; q < D; q += 64) s += dsum[q];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) *s_delta = (float)((double)eps * s / (double)D);
  }
  __syncthreads();
  return *s_delta;
}

// Hand every lower element (row >= col, both < D) of the loaded covariance to
// emit(row, col, value): diagonal real with delta added.
template <class Cfg, class Emit>
__device__ __forceinline__ void cov_emit(const floatx4 (&accR)[Cfg::TPW], const floatx4 (&accI)[Cfg::TPW], int D,
                                         float delta, Emit emit) {
  constexpr int NW = Cfg::NW, TPW = Cfg::TPW, NTILE = Cfg::NTILE;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int t = wave + NW * i;
    if (t < NTILE) {
      int I, J;
      cov_tile_of(t, I, J);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = I * 16 + 4 * (lane >> 4) + r, col = J * 16 + (lane & 15);
        if (row < D && col < D && row >= col) {
          if (row == col) emit(row, col, make_float2(accR[i][r] + delta, 0.f));
          else emit(row, col, make_float2(accR[i][r], accI[i][r]));
        }
      }
    }
  }
}

}  // namespace stap
