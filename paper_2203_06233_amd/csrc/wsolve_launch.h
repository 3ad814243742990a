// Kernel and launch of the one-wave stage solve for one (steering class,
// refinement) pair; included by wsolve_{r0,r1}_s{1,2}.hip.
#pragma once

#include "kernels.h"
#include "wsolve_impl.h"

namespace stap {
namespace wsv {

template <int NB, int NS, bool REFINE>
__global__ __launch_bounds__(64) void wsolve_kernel(const float2* __restrict__ cov, const float2* __restrict__ steer,
                                                    float2* __restrict__ wout, int* __restrict__ info_out, Dims d) {
  __shared__ __align__(16) float2 lds[WsLds<NB, REFINE>::COMPLEX];
  const int sys = blockIdx.x;
  wsolve_system<NB, NS, REFINE>(cov + (long long)sys * d.D * d.D, steer + steer_offset(d, sys), wout + (long long)sys * d.S * d.D,
                                info_out ? info_out + sys : nullptr, d, lds);
}

template <int NB, int NS, bool REFINE>
hipError_t go(const Dims& d, const float2* cov, const float2* steer, float2* w, int* info, hipStream_t st) {
  hipLaunchKernelGGL((wsolve_kernel<NB, NS, REFINE>), dim3(d.P * d.B), dim3(64), 0, st, cov, steer, w, info, d);
  return hipGetLastError();
}

template <int NS, bool REFINE>
hipError_t by_nb(const Dims& d, const float2* cov, const float2* steer, float2* w, int* info, hipStream_t st) {
  switch ((d.D + 15) / 16) {
    case 1: return go<1, NS, REFINE>(d, cov, steer, w, info, st);
    case 2: return go<2, NS, REFINE>(d, cov, steer, w, info, st);
    case 3: return go<3, NS, REFINE>(d, cov, steer, w, info, st);
    case 4: return go<4, NS, REFINE>(d, cov, steer, w, info, st);
    case 5: return go<5, NS, REFINE>(d, cov, steer, w, info, st);
    case 6: return go<6, NS, REFINE>(d, cov, steer, w, info, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace wsv
}  // namespace stap
