// Stage kernel for the sample covariance per (Doppler bin, training block)
// with diagonal loading (statement U of the STAP kernel, Sec. 4.2; Table 2
// row dot_{2D,2D}):
//
//   R_hat = (1/N) X_kb X_kb^H,   delta = eps * Re tr(R_hat) / D,
//   R_L   = R_hat + delta I,
//
// with X_kb the snapshots of bin k at the N training cells of block b (the
// block itself, or the nearest cells outside it and its guard cells).
//
// One workgroup per system; the MFMA work is cov_accumulate() (cov_impl.h).
// Both triangles are written: the upper is the bitwise conjugate of the
// lower and the diagonal is real.
#include "common.h"
#include "cov_impl.h"
#include "kernels.h"

namespace stap {

namespace {

// Up to 96 DOF on 8 waves the register allocation is capped at 128, two
// workgroups per compute unit.
template <int DP, int NW, int MODE>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(DP <= 96 && NW == 8 ? 4 : 1)))
void cov_kernel(const float2* __restrict__ snap,
                                                      float2* __restrict__ cov,
                                                      float* __restrict__ delta_out, Dims d) {
  using Cfg = CovCfg<DP, NW, MODE>;
  __shared__ __align__(16) unsigned char lds[Cfg::LDS_BYTES];
  __shared__ double dsum[DP];
  __shared__ float red[NW];
  __shared__ float s_delta;
  const int sys = blockIdx.x;
  const int k = sys / d.B, b = sys - (sys / d.B) * d.B;
  const int D = d.D;
  const float2* X = snap + (long long)k * D * d.R;
  floatx4 accR[Cfg::TPW], accI[Cfg::TPW];
  cov_accumulate<Cfg>(X, d.R, D, d.N, train_cells(d, b), lds, red, accR, accI);
  const float dl = cov_delta<Cfg>(accR, D, d.eps, dsum, &s_delta);
  if (delta_out && threadIdx.x == 0) delta_out[sys] = dl;
  float2* out = cov + (long long)sys * D * D;
  // lower triangle: for each register the 16 lanes of a row write 16
  // consecutive elements of one matrix row
  cov_emit<Cfg>(accR, accI, D, dl, [&](int row, int col, float2 v) {
    out[(long long)row * D + col] = v;
  });
  // upper triangle as the conjugate transpose: the lane's four registers
  // are four consecutive elements of one matrix row of the upper part, so
  // off-diagonal tiles inside D go out as two 16-byte stores per lane
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const bool vec_ok = (reinterpret_cast<uintptr_t>(out) & 15) == 0;  // the ABI asks for 8-byte alignment only
#pragma unroll
  for (int i = 0; i < Cfg::TPW; ++i) {
    const int t = wave + NW * i;
    if (t < Cfg::NTILE) {
      int I, J;
      cov_tile_of(t, I, J);
      const int col = J * 16 + (lane & 15), row0 = I * 16 + 4 * (lane >> 4);
      if (I > J && 16 * I + 16 <= D && (D & 1) == 0 && vec_ok) {
        float4* dst = reinterpret_cast<float4*>(out + (long long)col * D + row0);
        dst[0] = make_float4(accR[i][0], -accI[i][0], accR[i][1], -accI[i][1]);
        dst[1] = make_float4(accR[i][2], -accI[i][2], accR[i][3], -accI[i][3]);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = row0 + r;
          if (row < D && col < D && row > col) out[(long long)col * D + row] = make_float2(accR[i][r], -accI[i][r]);
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

// Waves per system: the tuned choice where the DOF class offers one (48 and
// 64: 4 or 8; 96: 4, 8 or 16; 128: 8 or 16), else the default of the class.
// Every choice computes each output tile the same way, only the assignment
// of tiles to waves differs, so the covariance is the same bit for bit.
hipError_t launch_covariance(const Dims& d, const float2* snap, float2* cov, float* delta,
                             hipStream_t st, int nw) {
  if (d.D <= 16) return go_cov<16, 1>(d, snap, cov, delta, st);
  if (d.D <= 32) return go_cov<32, 2>(d, snap, cov, delta, st);
  if (d.D <= 48) return nw == 8 ? go_cov<48, 8>(d, snap, cov, delta, st) : go_cov<48, 4>(d, snap, cov, delta, st);
  if (d.D <= 64) return nw == 8 ? go_cov<64, 8>(d, snap, cov, delta, st) : go_cov<64, 4>(d, snap, cov, delta, st);
  if (d.D <= 96) {
    if (nw == 4) return go_cov<96, 4>(d, snap, cov, delta, st);
    if (nw == 16) return go_cov<96, 16>(d, snap, cov, delta, st);
    return go_cov<96, 8>(d, snap, cov, delta, st);
  }
  if (d.D <= 128) return nw == 16 ? go_cov<128, 16>(d, snap, cov, delta, st) : go_cov<128, 8>(d, snap, cov, delta, st);
  return go_cov<192, 16>(d, snap, cov, delta, st);
}

}  // namespace stap
