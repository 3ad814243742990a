// Adaptive weights by Cholesky solves (textbook STAP weight solve):
//
//   R_L = L L^H,  a_s = L^-1 v_s,  gamma_s = ||a_s||^2 = v_s^H R_L^-1 v_s,
//   u_s = L^-H a_s,  w_s = u_s / sqrt(gamma_s),
//
// plus optional iterative refinement: r_s = v_s - R_L u_s formed in FP64 from
// the FP32 matrix, u_s += R_L^-1 r_s with the FP32 factor.
//
// Stage kernel: one workgroup per system reads the loaded covariance from
// global memory and runs solve_system() (solve_impl.h).
#include "common.h"
#include "kernels.h"
#include "solve_impl.h"

namespace stap {

namespace {

// Covariance source for the stage kernel: the full matrix in global memory;
// only the lower triangle is read.
struct GlobalR {
  const float2* A;
  int D;
  __device__ float2 lower(int i, int k) const { return A[(long long)i * D + k]; }
};

template <int TY, int NA, int NB, int NVS, bool REFINE>
__global__ __launch_bounds__(16 * TY) void solve_kernel(const float2* __restrict__ cov,
                                                        const float2* __restrict__ steer,
                                                        float2* __restrict__ wout, int* __restrict__ info_out,
                                                        Dims d) {
  using K = SolveCfg<TY, NA, NB, NVS>;
  __shared__ SolveShared<K> sh;
  extern __shared__ __align__(16) float2 dyn[];  // refinement: packed R_L, residual slab
  const int sys = blockIdx.x;
  GlobalR src{cov + (long long)sys * d.D * d.D, d.D};
  if (REFINE && K::kPackedInLds) {
    for (int i = threadIdx.x / 16; i < d.D; i += TY)
      for (int k = threadIdx.x % 16; k <= i; k += 16) dyn[i * (i + 1) / 2 + k] = src.lower(i, k);
  }
  solve_system<K, REFINE, K::kPackedInLds>(src, dyn, dyn + (K::kPackedInLds ? K::kPacked : 0),
                                           steer + steer_offset(d, sys),
                                           wout + (long long)sys * d.S * d.D,
                                           info_out ? info_out + sys : nullptr, d, sh);
}

template <int TY, int NA, int NB, int NVS>
hipError_t go_solve(const Dims& d, const float2* cov, const float2* steer, float2* w, int* info,
                    hipStream_t st) {
  using K = SolveCfg<TY, NA, NB, NVS>;
  const dim3 grid(d.P * d.B), block(16 * TY);
  if (d.refine == 0) {
    hipLaunchKernelGGL((solve_kernel<TY, NA, NB, NVS, false>), grid, block, 0, st, cov, steer, w, info, d);
    return hipGetLastError();
  }
  const size_t dyn = K::refine_lds_bytes();
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&solve_kernel<TY, NA, NB, NVS, true>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((solve_kernel<TY, NA, NB, NVS, true>), grid, block, dyn, st, cov, steer, w, info, d);
  return hipGetLastError();
}

template <int NB>
hipError_t go_solve16(const Dims& d, const float2* cov, const float2* steer, float2* w, int* info,
                      hipStream_t st) {
  if (d.S <= 16) return go_solve<16, NB, NB, 1>(d, cov, steer, w, info, st);
  if (d.S <= 32) return go_solve<16, NB, NB, 2>(d, cov, steer, w, info, st);
  if (d.S <= 48) return go_solve<16, NB, NB, 3>(d, cov, steer, w, info, st);
  return go_solve<16, NB, NB, 4>(d, cov, steer, w, info, st);
}

template <int NB>
hipError_t go_solve32(const Dims& d, const float2* cov, const float2* steer, float2* w, int* info,
                      hipStream_t st) {
  constexpr int NA = (16 * NB + 31) / 32;
  if (d.S <= 32) return go_solve<32, NA, NB, 1>(d, cov, steer, w, info, st);
  return go_solve<32, NA, NB, 2>(d, cov, steer, w, info, st);
}

}  // namespace

hipError_t launch_solve(const Dims& d, const float2* cov, const float2* steer, float2* w, int* info,
                        hipStream_t st) {
  switch ((d.D + 15) / 16) {
    case 1: return go_solve16<1>(d, cov, steer, w, info, st);
    case 2: return go_solve16<2>(d, cov, steer, w, info, st);
    case 3: return go_solve16<3>(d, cov, steer, w, info, st);
    case 4: return go_solve16<4>(d, cov, steer, w, info, st);
    case 5: return go_solve16<5>(d, cov, steer, w, info, st);
    case 6: return go_solve16<6>(d, cov, steer, w, info, st);
    case 7: return go_solve16<7>(d, cov, steer, w, info, st);
    case 8: return go_solve16<8>(d, cov, steer, w, info, st);
    case 9: case 10: return go_solve32<10>(d, cov, steer, w, info, st);
    case 11: case 12: return go_solve32<12>(d, cov, steer, w, info, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace stap
