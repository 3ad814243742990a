// Stage weight solve on the matrix cores: one workgroup per system reads the
// loaded covariance from global memory and runs bsolve_system()
// (bsolve_impl.h).  D <= 128, no refinement.
#include "bsolve_impl.h"
#include "kernels.h"

namespace stap {

namespace {

struct GlobalRB {
  const float2* A;
  int D;
  __device__ float2 lower(int i, int k) const { return A[(long long)i * D + k]; }
};

template <int NSLOT, int NW>
__global__ __launch_bounds__(64 * NW) void bsolve_kernel(const float2* __restrict__ cov,
                                                         const float2* __restrict__ steer,
                                                         float2* __restrict__ wout, int* __restrict__ info_out,
                                                         Dims d) {
  using C = BCfg<NSLOT, NW>;
  extern __shared__ __align__(16) unsigned char lds[];
  const int sys = blockIdx.x;
  bsolve_system<C>(GlobalRB{cov + (long long)sys * d.D * d.D, d.D}, steer, wout + (long long)sys * d.S * d.D,
                   info_out ? info_out + sys : nullptr, d, lds);
}

template <int NSLOT, int NW>
hipError_t go(const Dims& d, const float2* cov, const float2* steer, float2* w, int* info, hipStream_t st) {
  const size_t lds = BCfg<NSLOT, NW>::lds_bytes((d.D + 15) / 16, (d.S + 15) / 16);
  hipLaunchKernelGGL((bsolve_kernel<NSLOT, NW>), dim3(d.P * d.B), dim3(64 * NW), lds, st, cov, steer, w, info, d);
  return hipGetLastError();
}

}  // namespace

// Register blocks per wave the (D, S) shape needs with `waves` waves; the
// instantiated slot counts are 2, 3, 4, 5, 7, 9, 12 (4 waves) and 3, 5, 7, 9
// (8 waves).
int bsolve_slots(int D, int S, int waves) {
  const int NB = (D + 15) / 16, NS = (S + 15) / 16;
  const int need = (NB * (NB + 1) / 2 + NS * NB + waves - 1) / waves;
  static const int s4[] = {2, 3, 4, 5, 7, 9, 12}, s8[] = {3, 5, 7, 9};
  if (waves == 4) {
    for (int v : s4)
      if (need <= v) return v;
  } else if (waves == 8) {
    for (int v : s8)
      if (need <= v) return v;
  }
  return 0;
}

bool bsolve_supported(const Dims& d, int waves) {
  return d.D <= 128 && d.refine == 0 && bsolve_slots(d.D, d.S, waves) > 0;
}

hipError_t launch_bsolve(const Dims& d, const float2* cov, const float2* steer, float2* w, int* info,
                         hipStream_t st, int waves) {
  if (!bsolve_supported(d, waves)) return hipErrorInvalidValue;
  const int ns = bsolve_slots(d.D, d.S, waves);
  if (waves == 4) {
    switch (ns) {
      case 2: return go<2, 4>(d, cov, steer, w, info, st);
      case 3: return go<3, 4>(d, cov, steer, w, info, st);
      case 4: return go<4, 4>(d, cov, steer, w, info, st);
      case 5: return go<5, 4>(d, cov, steer, w, info, st);
      case 7: return go<7, 4>(d, cov, steer, w, info, st);
      case 9: return go<9, 4>(d, cov, steer, w, info, st);
      case 12: return go<12, 4>(d, cov, steer, w, info, st);
    }
  } else {
    switch (ns) {
      case 3: return go<3, 8>(d, cov, steer, w, info, st);
      case 5: return go<5, 8>(d, cov, steer, w, info, st);
      case 7: return go<7, 8>(d, cov, steer, w, info, st);
      case 9: return go<9, 8>(d, cov, steer, w, info, st);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace stap
