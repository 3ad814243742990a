// Fused covariance -> blocked matrix-core solve, FP32 covariance products:
// the one-cube launches of the 4-wave shapes.
#include "bfused_launch.h"

namespace stap {

hipError_t launch_bfused_f32_w4(const Dims& d, const float2* snap, const float2* steer, float2* w, int* info,
                                 hipStream_t st, int waves) {
  return bfused::single<0, 4>(d, snap, steer, w, info, st, waves);
}

}  // namespace stap
