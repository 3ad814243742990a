// Weight x snapshot inner products and output power (statement U applied to
// the adaptive weights):
//
//   y[k][s][r] = w_{k,b(r),s}^H X[k][:, r],   power = |y|^2.
//
// One workgroup per system (k, b): a complex (S x D) x (D x N) product on
// v_mfma_f32_16x16x4_f32,
//   Re y = Wr.Xr + Wi.Xi,   Im y = Wr.Xi - Wi.Xr.
// The weights of the system are staged once in LDS; each wave owns a set of
// 16-cell range tiles and all steering tiles, so every snapshot element is
// read from HBM exactly once, coalesced along range.
#include "common.h"
#include "kernels.h"

namespace stap {

namespace {

template <int ST, int DP>
__global__ __launch_bounds__(256) void inner_kernel(const float2* __restrict__ wts,
                                                    const float2* __restrict__ snap,
                                                    float* __restrict__ power, float2* __restrict__ yout,
                                                    Dims d) {
  constexpr int SP = ST * 16;
  constexpr int WPITCH = DP + 1;
  __shared__ float2 ws[SP * WPITCH];  // [s][d]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int sys = blockIdx.x;
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
  for (int rt = wave; rt < ntile; rt += 4) {
    const int r = rt * 16 + (lane & 15);
    const bool live = r < N;
    floatx4 accR[ST], accI[ST];
#pragma unroll
    for (int t = 0; t < ST; ++t) {
      accR[t] = floatx4{0.f, 0.f, 0.f, 0.f};
      accI[t] = accR[t];
    }
#pragma unroll 1
    for (int q0 = 0; q0 < DP; q0 += 16) {
      float2 xv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = q0 + 4 * u + (lane >> 4);
        xv[u] = (live && q < D) ? X[(long long)q * d.R + r] : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = q0 + 4 * u + (lane >> 4);
#pragma unroll
        for (int t = 0; t < ST; ++t) {
          const float2 wv = ws[(t * 16 + (lane & 15)) * WPITCH + q];
          accR[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.x, xv[u].x, accR[t], 0, 0, 0);
          accR[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.y, xv[u].y, accR[t], 0, 0, 0);
          accI[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.x, xv[u].y, accI[t], 0, 0, 0);
          accI[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(-wv.y, xv[u].x, accI[t], 0, 0, 0);
        }
      }
    }
    if (live) {
      const long long rr = (long long)b * N + r;
#pragma unroll
      for (int t = 0; t < ST; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int s = t * 16 + 4 * (lane >> 4) + i;
          if (s < S) {
            const float re = accR[t][i], im = accI[t][i];
            const long long o = ((long long)k * S + s) * d.R + rr;
            power[o] = re * re + im * im;
            if (yout) yout[o] = make_float2(re, im);
          }
        }
    }
  }
}

template <int ST>
hipError_t go_inner_dp(const Dims& d, const float2* w, const float2* snap, float* power, float2* y,
                       hipStream_t st) {
  dim3 grid(d.P * d.B), block(256);
  if (d.D <= 16) hipLaunchKernelGGL((inner_kernel<ST, 16>), grid, block, 0, st, w, snap, power, y, d);
  else if (d.D <= 32) hipLaunchKernelGGL((inner_kernel<ST, 32>), grid, block, 0, st, w, snap, power, y, d);
  else if (d.D <= 48) hipLaunchKernelGGL((inner_kernel<ST, 48>), grid, block, 0, st, w, snap, power, y, d);
  else if (d.D <= 64) hipLaunchKernelGGL((inner_kernel<ST, 64>), grid, block, 0, st, w, snap, power, y, d);
  else if (d.D <= 96) hipLaunchKernelGGL((inner_kernel<ST, 96>), grid, block, 0, st, w, snap, power, y, d);
  else if (d.D <= 128) hipLaunchKernelGGL((inner_kernel<ST, 128>), grid, block, 0, st, w, snap, power, y, d);
  else hipLaunchKernelGGL((inner_kernel<ST, 192>), grid, block, 0, st, w, snap, power, y, d);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_inner(const Dims& d, const float2* w, const float2* snap, float* power, float2* y,
                        hipStream_t st) {
  switch ((d.S + 15) / 16) {
    case 1: return go_inner_dp<1>(d, w, snap, power, y, st);
    case 2: return go_inner_dp<2>(d, w, snap, power, y, st);
    case 3: return go_inner_dp<3>(d, w, snap, power, y, st);
    case 4: return go_inner_dp<4>(d, w, snap, power, y, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace stap
