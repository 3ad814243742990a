// Weight x snapshot inner products and output power (statement U applied to
// the adaptive weights):
//
//   y[k][s][r] = w_{k,b(r),s}^H X[k][:, r],   power = |y|^2.
//
// One workgroup per system (k, b): a complex (S x D) x (D x N) product,
//   Re y = Wr.Xr + Wi.Xi,   Im y = Wr.Xi - Wi.Xr.
// The weights of the system are staged once in LDS; each wave owns a set of
// 16-cell range tiles and all steering tiles, so every snapshot element is
// read from HBM exactly once, coalesced along range.
//   FP32   v_mfma_f32_16x16x4_f32 on the FP32 operands.
//   BF16   (mixed path) weights and snapshots are split exactly into three
//          BF16 terms each; the six products hh, hm, mh, hl, lh, mm run on
//          v_mfma_f32_16x16x32_bf16, the hh term in its own accumulator, so
//          the output keeps FP32-level error (the filter output cancels the
//          clutter, so a single BF16 term would not).
#include "common.h"
#include "kernels.h"

namespace stap {

namespace {

template <int ST, int DP, int RTW = 2>
__device__ __forceinline__ void inner_system(const float2* __restrict__ wts, const float2* __restrict__ snap,
                                             float* __restrict__ power, float2* __restrict__ yout,
                                             const Dims& d, int sys) {
  constexpr int SP = ST * 16;
  constexpr int WPITCH = DP + 1;
  __shared__ float2 ws[SP * WPITCH];  // [s][d]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int k = sys / d.B, b = sys - (sys / d.B) * d.B;
  const int D = d.D, S = d.S, N = d.N;
  const float2* W = wts + (long long)sys * S * D;
  for (int e = tid; e < SP * DP; e += 256) {
    const int s = e / DP, q = e % DP;
    ws[s * WPITCH + q] = (s < S && q < D) ? W[s * D + q] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  const float2* X = snap + (long long)k * D * d.R + (long long)b * N;
  const int ntile = (N + 15) / 16;
  // each wave takes RTW range tiles at a time (a tuning choice: more tiles
  // give more independent MFMA chains and loads in flight, fewer give more
  // waves work); the snapshot loads of the next 16-row chunk are issued
  // before the MFMAs of the current one
  for (int rt0 = wave * RTW; rt0 < ntile; rt0 += 4 * RTW) {
    int r[RTW];
    bool live[RTW];
#pragma unroll
    for (int w = 0; w < RTW; ++w) {
      r[w] = (rt0 + w) * 16 + (lane & 15);
      live[w] = (rt0 + w < ntile) && r[w] < N;
    }
    floatx4 accR[RTW][ST], accI[RTW][ST];
#pragma unroll
    for (int w = 0; w < RTW; ++w)
#pragma unroll
      for (int t = 0; t < ST; ++t) {
        accR[w][t] = floatx4{0.f, 0.f, 0.f, 0.f};
        accI[w][t] = accR[w][t];
      }
    auto load = [&](int q0, float2 (&xv)[RTW][4]) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = q0 + 4 * u + (lane >> 4);
#pragma unroll
        for (int w = 0; w < RTW; ++w)
          xv[w][u] = (live[w] && q < D) ? X[(long long)q * d.R + r[w]] : make_float2(0.f, 0.f);
      }
    };
    float2 cur[RTW][4], nxt[RTW][4];
    load(0, cur);
#pragma unroll 1
    for (int q0 = 0; q0 < DP; q0 += 16) {
      if (q0 + 16 < DP) load(q0 + 16, nxt);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = q0 + 4 * u + (lane >> 4);
#pragma unroll
        for (int t = 0; t < ST; ++t) {
          const float2 wv = ws[(t * 16 + (lane & 15)) * WPITCH + q];
#pragma unroll
          for (int w = 0; w < RTW; ++w) {
            accR[w][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.x, cur[w][u].x, accR[w][t], 0, 0, 0);
            accR[w][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.y, cur[w][u].y, accR[w][t], 0, 0, 0);
            accI[w][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.x, cur[w][u].y, accI[w][t], 0, 0, 0);
            accI[w][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(-wv.y, cur[w][u].x, accI[w][t], 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int w = 0; w < RTW; ++w)
#pragma unroll
        for (int u = 0; u < 4; ++u) cur[w][u] = nxt[w][u];
    }
#pragma unroll
    for (int w = 0; w < RTW; ++w) {
      if (!live[w]) continue;
      const long long rr = (long long)b * N + r[w];
#pragma unroll
      for (int t = 0; t < ST; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int s = t * 16 + 4 * (lane >> 4) + i;
          if (s < S) {
            const float re = accR[w][t][i], im = accI[w][t][i];
            const long long o = ((long long)k * S + s) * d.R + rr;
            power[o] = re * re + im * im;
            if (yout) yout[o] = make_float2(re, im);
          }
        }
    }
  }
}

__device__ __forceinline__ floatx4 mfma_bf16x(uint4 a, uint4 b, floatx4 c) {
  typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b),
                                                 c, 0, 0, 0);
}


// Split-BF16 variant.  LDS holds the weights as six planes
// [re h, re m, re l, im h, im m, im l][s][d] (d padded to DP, pitch DP + 8).
template <int ST, int DP, int RTW = 1>
__device__ __forceinline__ void inner_bf16_system(const float2* __restrict__ wts, const float2* __restrict__ snap,
                                                  float* __restrict__ power, float2* __restrict__ yout,
                                                  const Dims& d, int sys) {
  constexpr int SP = ST * 16;
  constexpr int PITCH = DP + 8;              // bf16 units per row
  constexpr int PS = SP * PITCH / 2;         // plane stride in uint32
  __shared__ __align__(16) unsigned int wp[6 * PS];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int k = sys / d.B, b = sys - (sys / d.B) * d.B;
  const int D = d.D, S = d.S, N = d.N;
  const float2* W = wts + (long long)sys * S * D;
  for (int e = tid; e < SP * (DP / 2); e += 256) {
    const int s = e / (DP / 2), q = 2 * (e % (DP / 2));
    float2 w0 = make_float2(0.f, 0.f), w1 = w0;
    if (s < S) {
      if (q < D) w0 = W[s * D + q];
      if (q + 1 < D) w1 = W[s * D + q + 1];
    }
    unsigned int h, m, l;
    const int o = s * (PITCH / 2) + q / 2;
    split3x2(w0.x, w1.x, h, m, l);
    wp[0 * PS + o] = h;
    wp[1 * PS + o] = m;
    wp[2 * PS + o] = l;
    split3x2(w0.y, w1.y, h, m, l);
    wp[3 * PS + o] = h;
    wp[4 * PS + o] = m;
    wp[5 * PS + o] = l;
  }
  __syncthreads();
  const uint4* wp4 = reinterpret_cast<const uint4*>(wp);
  const float2* X = snap + (long long)k * D * d.R + (long long)b * N;
  const int ntile = (N + 15) / 16;
  constexpr int PA[5] = {0, 1, 0, 2, 1};
  constexpr int PB[5] = {1, 0, 2, 0, 1};
  // each wave takes RTW range tiles at a time (a tuning choice, as in the
  // FP32 form)
  for (int rt0 = wave * RTW; rt0 < ntile; rt0 += 4 * RTW) {
    int r[RTW];
    bool live[RTW];
#pragma unroll
    for (int w = 0; w < RTW; ++w) {
      r[w] = (rt0 + w) * 16 + (lane & 15);
      live[w] = (rt0 + w < ntile) && r[w] < N;
    }
    floatx4 accR[RTW][ST], accI[RTW][ST], corR[RTW][ST], corI[RTW][ST];
#pragma unroll
    for (int w = 0; w < RTW; ++w)
#pragma unroll
      for (int t = 0; t < ST; ++t) {
        accR[w][t] = floatx4{0.f, 0.f, 0.f, 0.f};
        accI[w][t] = accR[w][t];
        corR[w][t] = accR[w][t];
        corI[w][t] = accR[w][t];
      }
#pragma unroll 1
    for (int q0 = 0; q0 < DP; q0 += 32) {
      // B operand: X[q0 + 8*(lane/16) + j][r], j = 0..7, split into 3 terms
      uint4 Bv[RTW][6];
#pragma unroll
      for (int w = 0; w < RTW; ++w) {
        unsigned int xb[6][4];
#pragma unroll
        for (int j = 0; j < 8; j += 2) {
          const int q = q0 + 8 * (lane >> 4) + j;
          const float2 x0 = (live[w] && q < D) ? X[(long long)q * d.R + r[w]] : make_float2(0.f, 0.f);
          const float2 x1 = (live[w] && q + 1 < D) ? X[(long long)(q + 1) * d.R + r[w]] : make_float2(0.f, 0.f);
          split3x2(x0.x, x1.x, xb[0][j / 2], xb[1][j / 2], xb[2][j / 2]);
          split3x2(x0.y, x1.y, xb[3][j / 2], xb[4][j / 2], xb[5][j / 2]);
        }
#pragma unroll
        for (int p = 0; p < 6; ++p) Bv[w][p] = make_uint4(xb[p][0], xb[p][1], xb[p][2], xb[p][3]);
      }
#pragma unroll
      for (int t = 0; t < ST; ++t) {
        const int o = (t * 16 + (lane & 15)) * (PITCH / 8) + q0 / 8 + (lane >> 4);
        uint4 A[6];
#pragma unroll
        for (int p = 0; p < 6; ++p) A[p] = wp4[p * (PS / 4) + o];
#pragma unroll
        for (int w = 0; w < RTW; ++w) {
          // Re += Wr Xr + Wi Xi ;  Im += Wr Xi - Wi Xr
          accR[w][t] = mfma_bf16x(A[0], Bv[w][0], accR[w][t]);
          accR[w][t] = mfma_bf16x(A[3], Bv[w][3], accR[w][t]);
          accI[w][t] = mfma_bf16x(A[0], Bv[w][3], accI[w][t]);
          accI[w][t] = mfma_bf16x(negbf8(A[3]), Bv[w][0], accI[w][t]);
#pragma unroll
          for (int u = 0; u < 5; ++u) {
            corR[w][t] = mfma_bf16x(A[PA[u]], Bv[w][PB[u]], corR[w][t]);
            corR[w][t] = mfma_bf16x(A[3 + PA[u]], Bv[w][3 + PB[u]], corR[w][t]);
            corI[w][t] = mfma_bf16x(A[PA[u]], Bv[w][3 + PB[u]], corI[w][t]);
            corI[w][t] = mfma_bf16x(negbf8(A[3 + PA[u]]), Bv[w][PB[u]], corI[w][t]);
          }
        }
      }
    }
#pragma unroll
    for (int w = 0; w < RTW; ++w) {
      if (!live[w]) continue;
      const long long rr = (long long)b * N + r[w];
#pragma unroll
      for (int t = 0; t < ST; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int s = t * 16 + 4 * (lane >> 4) + i;
          if (s < S) {
            const float re = accR[w][t][i] + corR[w][t][i], im = accI[w][t][i] + corI[w][t][i];
            const long long o = ((long long)k * S + s) * d.R + rr;
            power[o] = re * re + im * im;
            if (yout) yout[o] = make_float2(re, im);
          }
        }
    }
  }
}

// Two steering tiles and two range tiles per step fit 128 VGPRs at 32..128
// DOF without spills: four workgroups per compute unit instead of three.
template <int ST, int DP, int RTW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ST == 2 && RTW == 2 && DP >= 32 && DP <= 128 ? 4 : 1)))
void inner_kernel(const float2* __restrict__ wts, const float2* __restrict__ snap,
                                                    float* __restrict__ power, float2* __restrict__ yout, Dims d) {
  inner_system<ST, DP, RTW>(wts, snap, power, yout, d, blockIdx.x);
}

// With two steering tiles and one range tile per wave step the register
// allocation fits three workgroups per compute unit (164 VGPRs at D = 96,
// no spills): more snapshot loads in flight for this bandwidth-bound pass.
template <int ST, int DP, int RTW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ST == 2 && RTW == 1 && DP >= 64 ? 3 : 1)))
void inner_bf16_kernel(const float2* __restrict__ wts,
                                                         const float2* __restrict__ snap,
                                                         float* __restrict__ power, float2* __restrict__ yout,
                                                         Dims d) {
  inner_bf16_system<ST, DP, RTW>(wts, snap, power, yout, d, blockIdx.x);
}

// Batched: one workgroup per system of every cube of the table.
// Register budgets that fit without spills: 128 (four workgroups per CU)
// for one steering tile and for FP32 with two, 168 (three) for split BF16
// with two.
template <int ST, int DP, bool BF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ST == 1 ? 4 : ST != 2 ? 1 : BF ? 3 : (DP >= 32 ? 4 : 1))))
void inner_batched_kernel(const ProbDesc* __restrict__ desc, int n) {
  const long long g = blockIdx.x;
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].sys_begin <= g) lo = mid;
    else hi = mid - 1;
  }
  const ProbDesc& pd = desc[lo];
  const Dims d = pd.d;
  if (BF) inner_bf16_system<ST, DP>(pd.w, pd.snap, pd.power, nullptr, d, (int)(g - pd.sys_begin));
  else inner_system<ST, DP>(pd.w, pd.snap, pd.power, nullptr, d, (int)(g - pd.sys_begin));
}

template <int ST, bool BF>
hipError_t go_inner_batched(const ProbDesc* desc, int n, long long total, int max_dof, hipStream_t st) {
  const dim3 grid((unsigned)total), block(256);
  if (max_dof <= 32) hipLaunchKernelGGL((inner_batched_kernel<ST, 32, BF>), grid, block, 0, st, desc, n);
  else if (max_dof <= 64) hipLaunchKernelGGL((inner_batched_kernel<ST, 64, BF>), grid, block, 0, st, desc, n);
  else if (max_dof <= 96) hipLaunchKernelGGL((inner_batched_kernel<ST, 96, BF>), grid, block, 0, st, desc, n);
  else hipLaunchKernelGGL((inner_batched_kernel<ST, 128, BF>), grid, block, 0, st, desc, n);
  return hipGetLastError();
}

// Range tiles per wave step: the tuned choice where given (1, 2 or 4;
// 2 for the split-BF16 form at most), else 2 (FP32) and 1 (split BF16).
template <int ST, int RTW>
hipError_t go_inner_bf16_r(const Dims& d, const float2* w, const float2* snap, float* power, float2* y,
                           hipStream_t st) {
  dim3 grid(d.P * d.B), block(256);
  if (d.D <= 32) hipLaunchKernelGGL((inner_bf16_kernel<ST, 32, RTW>), grid, block, 0, st, w, snap, power, y, d);
  else if (d.D <= 64) hipLaunchKernelGGL((inner_bf16_kernel<ST, 64, RTW>), grid, block, 0, st, w, snap, power, y, d);
  else if (d.D <= 96) hipLaunchKernelGGL((inner_bf16_kernel<ST, 96, RTW>), grid, block, 0, st, w, snap, power, y, d);
  else hipLaunchKernelGGL((inner_bf16_kernel<ST, 128, RTW>), grid, block, 0, st, w, snap, power, y, d);
  return hipGetLastError();
}

template <int ST>
hipError_t go_inner_bf16(const Dims& d, const float2* w, const float2* snap, float* power, float2* y,
                         hipStream_t st, int rtw) {
  return rtw == 2 ? go_inner_bf16_r<ST, 2>(d, w, snap, power, y, st) : go_inner_bf16_r<ST, 1>(d, w, snap, power, y, st);
}

template <int ST, int RTW>
hipError_t go_inner_dp_r(const Dims& d, const float2* w, const float2* snap, float* power, float2* y,
                         hipStream_t st) {
  dim3 grid(d.P * d.B), block(256);
  if (d.D <= 16) hipLaunchKernelGGL((inner_kernel<ST, 16, RTW>), grid, block, 0, st, w, snap, power, y, d);
  else if (d.D <= 32) hipLaunchKernelGGL((inner_kernel<ST, 32, RTW>), grid, block, 0, st, w, snap, power, y, d);
  else if (d.D <= 48) hipLaunchKernelGGL((inner_kernel<ST, 48, RTW>), grid, block, 0, st, w, snap, power, y, d);
  else if (d.D <= 64) hipLaunchKernelGGL((inner_kernel<ST, 64, RTW>), grid, block, 0, st, w, snap, power, y, d);
  else if (d.D <= 96) hipLaunchKernelGGL((inner_kernel<ST, 96, RTW>), grid, block, 0, st, w, snap, power, y, d);
  else if (d.D <= 128) hipLaunchKernelGGL((inner_kernel<ST, 128, RTW>), grid, block, 0, st, w, snap, power, y, d);
  else hipLaunchKernelGGL((inner_kernel<ST, 192, RTW>), grid, block, 0, st, w, snap, power, y, d);
  return hipGetLastError();
}

template <int ST>
hipError_t go_inner_dp(const Dims& d, const float2* w, const float2* snap, float* power, float2* y,
                       hipStream_t st, int rtw) {
  switch (rtw) {
    case 1: return go_inner_dp_r<ST, 1>(d, w, snap, power, y, st);
    case 4: return go_inner_dp_r<ST, 4>(d, w, snap, power, y, st);
  }
  return go_inner_dp_r<ST, 2>(d, w, snap, power, y, st);
}

}  // namespace

hipError_t launch_inner_batched(const ProbDesc* desc, int n, long long total_sys, int max_dof, int max_steer,
                                int prec, hipStream_t st) {
  if (max_dof > 128 || total_sys <= 0) return hipErrorInvalidValue;
  const bool bf = prec != STAP_PREC_FP32;
  switch ((max_steer + 15) / 16) {
    case 1: return bf ? go_inner_batched<1, true>(desc, n, total_sys, max_dof, st)
                      : go_inner_batched<1, false>(desc, n, total_sys, max_dof, st);
    case 2: return bf ? go_inner_batched<2, true>(desc, n, total_sys, max_dof, st)
                      : go_inner_batched<2, false>(desc, n, total_sys, max_dof, st);
    case 3: return bf ? go_inner_batched<3, true>(desc, n, total_sys, max_dof, st)
                      : go_inner_batched<3, false>(desc, n, total_sys, max_dof, st);
    case 4: return bf ? go_inner_batched<4, true>(desc, n, total_sys, max_dof, st)
                      : go_inner_batched<4, false>(desc, n, total_sys, max_dof, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_inner(const Dims& d, const float2* w, const float2* snap, float* power, float2* y,
                        hipStream_t st, int rtw) {
  if (d.prec != STAP_PREC_FP32 && d.D <= 128) {
    switch ((d.S + 15) / 16) {
      case 1: return go_inner_bf16<1>(d, w, snap, power, y, st, rtw);
      case 2: return go_inner_bf16<2>(d, w, snap, power, y, st, rtw);
      case 3: return go_inner_bf16<3>(d, w, snap, power, y, st, rtw);
      case 4: return go_inner_bf16<4>(d, w, snap, power, y, st, rtw);
    }
    return hipErrorInvalidValue;
  }
  switch ((d.S + 15) / 16) {
    case 1: return go_inner_dp<1>(d, w, snap, power, y, st, rtw);
    case 2: return go_inner_dp<2>(d, w, snap, power, y, st, rtw);
    case 3: return go_inner_dp<3>(d, w, snap, power, y, st, rtw);
    case 4: return go_inner_dp<4>(d, w, snap, power, y, st, rtw);
  }
  return hipErrorInvalidValue;
}

}  // namespace stap
