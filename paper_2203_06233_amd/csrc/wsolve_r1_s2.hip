// One-wave stage solve, steering class 2 (S <= 32), refinement on.
#define STAP_TID_DIRECT
#include "wsolve_launch.h"

namespace stap {

hipError_t launch_wsolve_r1_s2(const Dims& d, const float2* cov, const float2* steer, float2* w, int* info,
                                  hipStream_t st) {
  return wsv::by_nb<2, true>(d, cov, steer, w, info, st);
}

}  // namespace stap
