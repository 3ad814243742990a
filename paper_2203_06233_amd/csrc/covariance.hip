// Sample covariance per (Doppler bin, training block) with diagonal loading
// (statement U of the STAP kernel, Sec. 4.2; Table 2 row dot_{2D,2D}):
//
//   R_hat = (1/N) X_kb X_kb^H,   delta = eps * Re tr(R_hat) / D,
//   R_L   = R_hat + delta I.
//
// One workgroup per system (k, b).  The complex Hermitian rank-N update runs
// as real MFMA products over 16x16 output tiles of the lower block triangle:
//   Re R = Xr Xr^T + Xi Xi^T,   Im R = Xi Xr^T - Xr Xi^T.
// Range cells are staged through LDS in chunks of 32.
//   FP32  v_mfma_f32_16x16x4_f32 on the complex64 snapshots; the four real
//         product terms accumulate separately within each 32-cell chunk.
//   BF16  every FP32 snapshot component is split exactly into three BF16
//         terms x = h + m + l (24 bits); the six products hh, hm, mh, hl, lh,
//         mm run on v_mfma_f32_16x16x32_bf16 with FP32 accumulation, the hh
//         product in one accumulator and the five small ones in another, so
//         the result carries FP32-level error at 6/16 of the FP32-MFMA cost.
//   FP8   every component is scaled by a power of two per system so that the
//         largest magnitude maps near the E4M3 maximum, rounded to E4M3, and
//         one product per element runs on v_mfma_f32_16x16x32_fp8_fp8.
// The trace is summed in FP64.  Both triangles are written; the upper is the
// bitwise conjugate of the lower and the diagonal is real.
#include "common.h"
#include "kernels.h"

namespace stap {

namespace {

constexpr int kChunk = 32;

__device__ __forceinline__ void tile_of(int t, int& I, int& J) {
  int i = 0;
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  I = i;
  J = t - i * (i + 1) / 2;
}

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 u) { return __builtin_bit_cast(bf16x8, u); }

__device__ __forceinline__ floatx4 mfma_bf16(uint4 a, uint4 b, floatx4 c) {
  typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b),
                                                 c, 0, 0, 0);
}

__device__ __forceinline__ uint4 negbf(uint4 u) {
  return make_uint4(u.x ^ 0x80008000u, u.y ^ 0x80008000u, u.z ^ 0x80008000u, u.w ^ 0x80008000u);
}

// E4M3 (OCP, finite max 448) round-to-nearest-even with saturation.
__device__ __forceinline__ unsigned int f2e4m3(float x) {
  const unsigned int s = (__float_as_uint(x) >> 24) & 0x80u;
  float a = fabsf(x);
  if (!(a < 448.f)) return s | 0x7Eu;  // saturate (also NaN -> max)
  if (a < 0.015625f) {                  // subnormal range: step 2^-9
    const float q = rintf(a * 512.f);   // RNE
    return s | (unsigned int)q;         // q <= 8 -> 0x08 is the smallest normal
  }
  unsigned int u = __float_as_uint(a);
  u += 0x7FFFFu + ((u >> 20) & 1u);     // RNE to 3 mantissa bits
  const int e = (int)((u >> 23) & 0xFF) - 127 + 7;
  const unsigned int m = (u >> 20) & 0x7u;
  if (e > 15 || (e == 15 && m == 7)) return s | 0x7Eu;
  return s | ((unsigned int)e << 3) | m;
}

template <int DP, int NW, int MODE>
__global__ __launch_bounds__(NW * 64) void cov_kernel(const float2* __restrict__ snap,
                                                      float2* __restrict__ cov,
                                                      float* __restrict__ delta_out, Dims d) {
  constexpr int NT = NW * 64;
  constexpr int TB = DP / 16;
  constexpr int NTILE = TB * (TB + 1) / 2;
  constexpr int TPW = (NTILE + NW - 1) / NW;
  // FP32: [row][cell] complex, padded pitch.  BF16: 6 planes [p][row][cell].
  // FP8: 2 planes (re, im) of bytes.
  constexpr int F32_PITCH = kChunk + 1;                 // float2 units
  constexpr int BF_PITCH = kChunk + 8;                  // bf16 units
  constexpr int F8_PITCH = kChunk + 16;                 // bytes
  constexpr int LDS_BYTES = MODE == 0   ? DP * F32_PITCH * 8
                            : MODE == 1 ? 6 * DP * BF_PITCH * 2
                                        : 2 * DP * F8_PITCH;
  __shared__ __align__(16) unsigned char lds[LDS_BYTES];
  __shared__ double dsum[DP];
  __shared__ float s_delta, s_scale;

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int sys = blockIdx.x;
  const int k = sys / d.B, b = sys - (sys / d.B) * d.B;
  const int D = d.D, N = d.N;
  const float2* X = snap + (long long)k * D * d.R + (long long)b * N;

  floatx4 accR[TPW], accI[TPW], corR[TPW], corI[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    accR[i] = floatx4{0.f, 0.f, 0.f, 0.f};
    accI[i] = accR[i];
    corR[i] = accR[i];
    corI[i] = accR[i];
  }

  float qscale = 1.f;  // FP8: per-system power-of-two scale
  if (MODE == 2) {
    // max |component| over the system's snapshots
    float mx = 0.f;
    for (int e = tid; e < D * N; e += NT) {
      const int row = e / N, cc = e - (e / N) * N;
      const float2 v = X[(long long)row * d.R + cc];
      mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y)));
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    float* red = reinterpret_cast<float*>(lds);
    if (lane == 0) red[wave] = mx;
    __syncthreads();
    if (tid == 0) {
      float m2 = 0.f;
      for (int w = 0; w < NW; ++w) m2 = fmaxf(m2, red[w]);
      // largest power of two s with m2 * s <= 256 (E4M3 max is 448)
      int ex = 0;
      if (m2 > 0.f) {
        frexpf(m2, &ex);  // m2 = f * 2^ex, f in [0.5, 1)
      }
      s_scale = ldexpf(1.f, 8 - ex);
    }
    __syncthreads();
    qscale = s_scale;
  }

  for (int c0 = 0; c0 < N; c0 += kChunk) {
    const int nc = min(kChunk, N - c0);
    __syncthreads();
    if (MODE == 0) {
      float2* xs = reinterpret_cast<float2*>(lds);
      for (int e = tid; e < DP * kChunk; e += NT) {
        const int row = e / kChunk, cc = e % kChunk;
        float2 v = make_float2(0.f, 0.f);
        if (row < D && cc < nc) v = X[(long long)row * d.R + c0 + cc];
        xs[row * F32_PITCH + cc] = v;
      }
    } else if (MODE == 1) {
      unsigned int* pl = reinterpret_cast<unsigned int*>(lds);
      for (int e = tid; e < DP * (kChunk / 2); e += NT) {
        const int row = e / (kChunk / 2), cp = e % (kChunk / 2);
        float2 v0 = make_float2(0.f, 0.f), v1 = v0;
        if (row < D) {
          const float2* src = X + (long long)row * d.R + c0 + 2 * cp;
          if (2 * cp < nc) v0 = src[0];
          if (2 * cp + 1 < nc) v1 = src[1];
        }
        unsigned short h0, m0, l0, h1, m1, l1;
        const int base = row * (BF_PITCH / 2) + cp;  // in uint32 units
        constexpr int PS = DP * BF_PITCH / 2;        // plane stride, uint32
        split3(v0.x, h0, m0, l0);
        split3(v1.x, h1, m1, l1);
        pl[0 * PS + base] = h0 | ((unsigned int)h1 << 16);
        pl[1 * PS + base] = m0 | ((unsigned int)m1 << 16);
        pl[2 * PS + base] = l0 | ((unsigned int)l1 << 16);
        split3(v0.y, h0, m0, l0);
        split3(v1.y, h1, m1, l1);
        pl[3 * PS + base] = h0 | ((unsigned int)h1 << 16);
        pl[4 * PS + base] = m0 | ((unsigned int)m1 << 16);
        pl[5 * PS + base] = l0 | ((unsigned int)l1 << 16);
      }
    } else {
      unsigned char* pl = lds;
      for (int e = tid; e < DP * kChunk; e += NT) {
        const int row = e / kChunk, cc = e % kChunk;
        float2 v = make_float2(0.f, 0.f);
        if (row < D && cc < nc) v = X[(long long)row * d.R + c0 + cc];
        pl[row * F8_PITCH + cc] = (unsigned char)f2e4m3(v.x * qscale);
        pl[DP * F8_PITCH + row * F8_PITCH + cc] = (unsigned char)f2e4m3(v.y * qscale);
      }
    }
    __syncthreads();

#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int t = wave + NW * i;
      if (t < NTILE) {
        int I, J;
        tile_of(t, I, J);
        const int ra = I * 16 + (lane & 15), rb = J * 16 + (lane & 15);
        if (MODE == 0) {
          // four product terms in separate chunk accumulators, folded into
          // the running sums once per chunk: fewer roundings per sum
          const float2* xs = reinterpret_cast<const float2*>(lds);
          const int kq = (nc + 3) & ~3;
          floatx4 rr = floatx4{0.f, 0.f, 0.f, 0.f}, ii = rr, ir = rr, ri = rr;
          for (int kk = 0; kk < kq; kk += 4) {
            const float2 a = xs[ra * F32_PITCH + kk + (lane >> 4)];
            const float2 bb = xs[rb * F32_PITCH + kk + (lane >> 4)];
            rr = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, bb.x, rr, 0, 0, 0);
            ii = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, bb.y, ii, 0, 0, 0);
            ir = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, bb.x, ir, 0, 0, 0);
            ri = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, bb.y, ri, 0, 0, 0);
          }
          accR[i] += rr + ii;
          accI[i] += ir - ri;
        } else if (MODE == 1) {
          const uint4* pl = reinterpret_cast<const uint4*>(lds);
          constexpr int PS4 = DP * BF_PITCH / 8;  // plane stride in uint4
          const int oa = ra * (BF_PITCH / 8) + (lane >> 4);
          const int ob = rb * (BF_PITCH / 8) + (lane >> 4);
          uint4 A[6], Bv[6];
#pragma unroll
          for (int p = 0; p < 6; ++p) {
            A[p] = pl[p * PS4 + oa];
            Bv[p] = pl[p * PS4 + ob];
          }
          // real part: re*re + im*im; imaginary part: im*re - re*im
          accR[i] = mfma_bf16(A[0], Bv[0], accR[i]);
          accR[i] = mfma_bf16(A[3], Bv[3], accR[i]);
          accI[i] = mfma_bf16(A[3], Bv[0], accI[i]);
          accI[i] = mfma_bf16(negbf(A[0]), Bv[3], accI[i]);
          constexpr int PA[5] = {0, 1, 0, 2, 1};
          constexpr int PB[5] = {1, 0, 2, 0, 1};
#pragma unroll
          for (int q = 0; q < 5; ++q) {
            corR[i] = mfma_bf16(A[PA[q]], Bv[PB[q]], corR[i]);
            corR[i] = mfma_bf16(A[3 + PA[q]], Bv[3 + PB[q]], corR[i]);
            corI[i] = mfma_bf16(A[3 + PA[q]], Bv[PB[q]], corI[i]);
            corI[i] = mfma_bf16(negbf(A[PA[q]]), Bv[3 + PB[q]], corI[i]);
          }
        } else {
          // FP8: 16x16x32, lane holds 8 bytes of K = 8*(lane/16) .. +7
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

  // combine, scale: R_hat = acc / N  (FP8: / (N * s^2))
  const float invs2 = (MODE == 2) ? 1.f / (qscale * qscale) : 1.f;
  const float fN = (float)N;
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      accR[i][r] = ((accR[i][r] + corR[i][r]) * invs2) / fN;
      accI[i][r] = ((accI[i][r] + corI[i][r]) * invs2) / fN;
    }
  }

  // trace in FP64
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int t = wave + NW * i;
    if (t < NTILE) {
      int I, J;
      tile_of(t, I, J);
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
    if (lane == 0) {
      const float dl = (float)((double)d.eps * s / (double)D);
      s_delta = dl;
      if (delta_out) delta_out[sys] = dl;
    }
  }
  __syncthreads();
  const float dl = s_delta;

  float2* out = cov + (long long)sys * D * D;
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int t = wave + NW * i;
    if (t < NTILE) {
      int I, J;
      tile_of(t, I, J);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = I * 16 + 4 * (lane >> 4) + r, col = J * 16 + (lane & 15);
        if (row < D && col < D && row >= col) {
          if (row == col) {
            out[(long long)row * D + col] = make_float2(accR[i][r] + dl, 0.f);
          } else {
            const float re = accR[i][r], im = accI[i][r];
            out[(long long)row * D + col] = make_float2(re, im);
            out[(long long)col * D + row] = make_float2(re, -im);
          }
        }
      }
    }
  }
}

template <int DP, int NW>
hipError_t go_cov(const Dims& d, const float2* snap, float2* cov, float* delta, hipStream_t st) {
  dim3 grid(d.P * d.B), block(NW * 64);
  switch (d.prec) {
    case STAP_PREC_FP32:
      hipLaunchKernelGGL((cov_kernel<DP, NW, 0>), grid, block, 0, st, snap, cov, delta, d);
      break;
    case STAP_PREC_BF16:
      hipLaunchKernelGGL((cov_kernel<DP, NW, 1>), grid, block, 0, st, snap, cov, delta, d);
      break;
    default:
      hipLaunchKernelGGL((cov_kernel<DP, NW, 2>), grid, block, 0, st, snap, cov, delta, d);
      break;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_covariance(const Dims& d, const float2* snap, float2* cov, float* delta,
                             hipStream_t st) {
  if (d.D <= 16) return go_cov<16, 1>(d, snap, cov, delta, st);
  if (d.D <= 32) return go_cov<32, 2>(d, snap, cov, delta, st);
  if (d.D <= 48) return go_cov<48, 4>(d, snap, cov, delta, st);
  if (d.D <= 64) return go_cov<64, 4>(d, snap, cov, delta, st);
  if (d.D <= 96) return go_cov<96, 8>(d, snap, cov, delta, st);
  if (d.D <= 128) return go_cov<128, 8>(d, snap, cov, delta, st);
  return go_cov<192, 16>(d, snap, cov, delta, st);
}

}  // namespace stap
