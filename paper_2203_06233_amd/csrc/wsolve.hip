// Stage weight solve with one wave per system (wsolve_impl.h): dispatch over
// the steering class and refinement; the instantiations live in
// wsolve_{r0,r1}_s{1,2}.hip so they build in parallel.
#include "kernels.h"

namespace stap {

hipError_t launch_wsolve_r0_s1(const Dims&, const float2*, const float2*, float2*, int*, hipStream_t);
hipError_t launch_wsolve_r0_s2(const Dims&, const float2*, const float2*, float2*, int*, hipStream_t);
hipError_t launch_wsolve_r1_s1(const Dims&, const float2*, const float2*, float2*, int*, hipStream_t);
hipError_t launch_wsolve_r1_s2(const Dims&, const float2*, const float2*, float2*, int*, hipStream_t);

bool wsolve_supported(const Dims& d) { return d.D >= 1 && d.D <= 96 && d.S >= 1 && d.S <= 32; }

hipError_t launch_wsolve(const Dims& d, const float2* cov, const float2* steer, float2* w, int* info,
                         hipStream_t st) {
  if (!wsolve_supported(d)) return hipErrorInvalidValue;
  if (d.refine == 0)
    return d.S <= 16 ? launch_wsolve_r0_s1(d, cov, steer, w, info, st) : launch_wsolve_r0_s2(d, cov, steer, w, info, st);
  return d.S <= 16 ? launch_wsolve_r1_s1(d, cov, steer, w, info, st) : launch_wsolve_r1_s2(d, cov, steer, w, info, st);
}

}  // namespace stap
