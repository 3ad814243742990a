// Launch helpers of the fused covariance -> blocked matrix-core solve
// (fused_impl.h, bsolve_impl.h): dispatch over the covariance block columns,
// the steering class and the wave count.  Included by one translation unit
// per (precision, single or batched) so the instantiations build in
// parallel.
#pragma once

#include <type_traits>

#include "fused_impl.h"

namespace stap {
namespace bfused {


// register blocks per wave for NB block columns and NS steering blocks
constexpr int nsl(int NB, int NW) { return (NB * (NB + 1) / 2 + NW - 1) / NW; }
constexpr int nsm(int NB, int NS, int NW) { return (NS * NB + NW - 1) / NW; }

template <int NB, int NS, int NW, int MODE>
hipError_t go1(const Dims& d, const float2* snap, const float2* steer, float2* w, int* info, hipStream_t st) {
  constexpr int L = nsl(NB, NW), M = nsm(NB, NS, NW);
  if (d.refine == 0)
    hipLaunchKernelGGL((bfused_kernel<NB, NS, L, M, NW, MODE, false>), dim3(d.P * d.B), dim3(64 * NW), 0, st, snap, steer,
                       w, info, d);
  else
    hipLaunchKernelGGL((bfused_kernel<NB, NS, L, M, NW, MODE, true>), dim3(d.P * d.B), dim3(64 * NW), 0, st, snap, steer,
                       w, info, d);
  return hipGetLastError();
}

template <int NB, int NS, int NW, int MODE>
hipError_t gob(const ProbDesc* desc, int n, long long total, int refine, hipStream_t st, unsigned long long* queue) {
  constexpr int L = nsl(NB, NW), M = nsm(NB, NS, NW);
  // enough workgroups to fill every CU a few times over, never more than systems
  const long long want = 256LL * (NW == 4 ? 4 : 2);
  const dim3 grid((unsigned)(total < want ? total : want)), block(64 * NW);
  if (refine == 0)
    hipLaunchKernelGGL((bfused_batched_kernel<NB, NS, L, M, NW, MODE, false>), grid, block, 0, st, desc, n, total,
                       queue);
  else
    hipLaunchKernelGGL((bfused_batched_kernel<NB, NS, L, M, NW, MODE, true>), grid, block, 0, st, desc, n, total,
                       queue);
  return hipGetLastError();
}

// one switch for the single-cube and batched launches
template <int MODE, class F>
hipError_t pick(int D, int S, int waves, F&& f) {
  const int nb = (D + 15) / 16;
  const int ns = S <= 16 ? 1 : S <= 32 ? 2 : 4;
  auto by_s = [&](auto nbc, auto nwc) -> hipError_t {
    constexpr int NB = decltype(nbc)::value, NW = decltype(nwc)::value;
    if (ns == 1) return f(std::integral_constant<int, NB>{}, std::integral_constant<int, 1>{}, nwc);
    if (ns == 2) return f(std::integral_constant<int, NB>{}, std::integral_constant<int, 2>{}, nwc);
    return f(std::integral_constant<int, NB>{}, std::integral_constant<int, 4>{}, nwc);
  };
  using W4 = std::integral_constant<int, 4>;
  using W8 = std::integral_constant<int, 8>;
  switch (nb) {
    case 1: return by_s(std::integral_constant<int, 1>{}, W4{});
    case 2: return by_s(std::integral_constant<int, 2>{}, W4{});
    case 3: return by_s(std::integral_constant<int, 3>{}, W4{});
    case 4: return by_s(std::integral_constant<int, 4>{}, W4{});
    case 5: case 6:
      return waves == 8 ? by_s(std::integral_constant<int, 6>{}, W8{}) : by_s(std::integral_constant<int, 6>{}, W4{});
    case 7: case 8: return by_s(std::integral_constant<int, 8>{}, W8{});
  }
  return hipErrorInvalidValue;
}

// The wave count pick() takes for D and the requested waves.
inline int pick_waves(int D, int waves) {
  const int nb = (D + 15) / 16;
  return nb <= 4 ? 4 : nb <= 6 ? (waves == 8 ? 8 : 4) : 8;
}

// One-cube launches of the shapes that run on NWSEL waves (the 4- and 8-wave
// kernels live in separate translation units, built with different
// lane_tid() forms).
template <int MODE, int NWSEL>
hipError_t single(const Dims& d, const float2* snap, const float2* steer, float2* w, int* info, hipStream_t st,
                  int waves) {
  return pick<MODE>(d.D, d.S, waves, [&](auto nb, auto ns, auto nw) -> hipError_t {
    if constexpr (decltype(nw)::value == NWSEL)
      return go1<decltype(nb)::value, decltype(ns)::value, decltype(nw)::value, MODE>(d, snap, steer, w, info, st);
    else
      return hipErrorInvalidValue;
  });
}

template <int MODE>
hipError_t batched(const ProbDesc* desc, int n, long long total, int max_dof, int max_steer, int refine, int waves,
                   hipStream_t st, unsigned long long* queue) {
  return pick<MODE>(max_dof, max_steer, waves, [&](auto nb, auto ns, auto nw) {
    return gob<decltype(nb)::value, decltype(ns)::value, decltype(nw)::value, MODE>(desc, n, total, refine, st,
                                                                                   queue);
  });
}

}  // namespace bfused
}  // namespace stap
