// Stage weight solve on the matrix cores: one workgroup per system reads the
// loaded covariance from global memory and runs bsolve_system()
// (bsolve_impl.h), with or without FP64 refinement.
#include "bsolve_impl.h"
#include "kernels.h"

namespace stap {

namespace {

struct GlobalRB {
  const float2* A;
  int D;
  __device__ float2 lower(int i, int k) const { return A[(long long)i * D + k]; }
};

// With refinement and 8 waves the register allocation is capped at 128 so
// that two systems share a compute unit.
template <int NSL, int NSM, int NW, bool REFINE>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(REFINE && NW == 8 ? 4 : 1)))
void bsolve_kernel(const float2* __restrict__ cov,
                                                         const float2* __restrict__ steer,
                                                         float2* __restrict__ wout, int* __restrict__ info_out,
                                                         Dims d) {
  using C = BCfg<NSL, NSM, NW>;
  extern __shared__ __align__(16) unsigned char lds[];
  const int sys = blockIdx.x;
  bsolve_system<C, REFINE>(GlobalRB{cov + (long long)sys * d.D * d.D, d.D}, steer + steer_offset(d, sys),
                           wout + (long long)sys * d.S * d.D, info_out ? info_out + sys : nullptr, d, lds);
}

template <int NSL, int NSM, int NW, bool REFINE>
hipError_t go_r(const Dims& d, const float2* cov, const float2* steer, float2* w, int* info, hipStream_t st) {
  const size_t lds = BCfg<NSL, NSM, NW>::lds_bytes((d.D + 15) / 16, (d.S + 15) / 16);
  if (lds > 48 * 1024) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&bsolve_kernel<NSL, NSM, NW, REFINE>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((bsolve_kernel<NSL, NSM, NW, REFINE>), dim3(d.P * d.B), dim3(64 * NW), lds, st, cov, steer, w,
                     info, d);
  return hipGetLastError();
}

template <int NSL, int NSM, int NW>
hipError_t go(const Dims& d, const float2* cov, const float2* steer, float2* w, int* info, hipStream_t st) {
  return d.refine == 0 ? go_r<NSL, NSM, NW, false>(d, cov, steer, w, info, st)
                       : go_r<NSL, NSM, NW, true>(d, cov, steer, w, info, st);
}

template <int NW>
int round_up(int need, const int* opts, int n) {
  for (int i = 0; i < n; ++i)
    if (need <= opts[i]) return opts[i];
  return 0;
}

}  // namespace

// Slot counts instantiated per wave count: L slots {1, 2, 3, 5} (4 waves),
// {2, 3, 5} (8 waves) or {3, 5} (16 waves), M slots {1, 2, 4} ({2, 3} with
// 16 waves).  Variant 8 runs D > 128 (up to 12 block columns) with 16 waves.
static const int kL4[] = {1, 2, 3, 5}, kL8[] = {2, 3, 5}, kL16[] = {3, 5}, kM[] = {1, 2, 4}, kM16[] = {2, 3};

static int waves_for(const Dims& d, int waves) { return waves == 8 && d.D > 128 ? 16 : waves; }

static bool slots_for(const Dims& d, int waves, int& nl, int& nm) {
  const int NB = (d.D + 15) / 16, NS = (d.S + 15) / 16;
  if (waves == 4) {
    nl = round_up<4>(BCfg<1, 1, 4>::lslots(NB), kL4, 4);
    nm = round_up<4>(BCfg<1, 1, 4>::mslots(NB, NS), kM, 3);
  } else if (waves == 8) {
    nl = round_up<8>(BCfg<1, 1, 8>::lslots(NB), kL8, 3);
    nm = round_up<8>(BCfg<1, 1, 8>::mslots(NB, NS), kM, 3);
  } else if (waves == 16) {
    nl = round_up<16>(BCfg<1, 1, 16>::lslots(NB), kL16, 2);
    nm = round_up<16>(BCfg<1, 1, 16>::mslots(NB, NS), kM16, 2);
  } else {
    return false;
  }
  return nl > 0 && nm > 0;
}

bool bsolve_supported(const Dims& d, int waves) {
  int nl, nm;
  return d.D <= kMaxDof && slots_for(d, waves_for(d, waves), nl, nm);
}

hipError_t launch_bsolve(const Dims& d, const float2* cov, const float2* steer, float2* w, int* info,
                         hipStream_t st, int waves_asked) {
  int nl, nm;
  const int waves = waves_for(d, waves_asked);
  if (!slots_for(d, waves, nl, nm)) return hipErrorInvalidValue;
#define STAP_BS(L, M, W) \
  if (nl == L && nm == M && waves == W) return go<L, M, W>(d, cov, steer, w, info, st);
  STAP_BS(1, 1, 4) STAP_BS(1, 2, 4) STAP_BS(1, 4, 4)
  STAP_BS(2, 1, 4) STAP_BS(2, 2, 4) STAP_BS(2, 4, 4)
  STAP_BS(3, 1, 4) STAP_BS(3, 2, 4) STAP_BS(3, 4, 4)
  STAP_BS(5, 1, 4) STAP_BS(5, 2, 4) STAP_BS(5, 4, 4)
  STAP_BS(2, 1, 8) STAP_BS(2, 2, 8) STAP_BS(2, 4, 8)
  STAP_BS(3, 1, 8) STAP_BS(3, 2, 8) STAP_BS(3, 4, 8)
  STAP_BS(5, 1, 8) STAP_BS(5, 2, 8) STAP_BS(5, 4, 8)
  STAP_BS(3, 2, 16) STAP_BS(3, 3, 16) STAP_BS(5, 2, 16) STAP_BS(5, 3, 16)
#undef STAP_BS
  return hipErrorInvalidValue;
}

}  // namespace stap
