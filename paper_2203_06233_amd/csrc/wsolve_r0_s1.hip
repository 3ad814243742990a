// One-wave stage solve, steering class 1 (S <= 16), refinement off.
#define STAP_TID_DIRECT
#include "wsolve_launch.h"

namespace stap {

hipError_t launch_wsolve_r0_s1(const Dims& d, const float2* cov, const float2* steer, float2* w, int* info,
                                  hipStream_t st) {
  return wsv::by_nb<1, false>(d, cov, steer, w, info, st);
}

}  // namespace stap
