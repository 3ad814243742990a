// Fused covariance -> blocked matrix-core solve, split-BF16 covariance products:
// the one-cube launches, 8-wave shapes here (lane offsets kept live, the
// residual's operands loaded ahead), 4-wave shapes in bfused_bf16_w4.hip.
#define STAP_TID_DIRECT
#define STAP_RESIDUAL_LOADS_AHEAD
#include "bfused_launch.h"

namespace stap {

hipError_t launch_bfused_bf16_w4(const Dims& d, const float2* snap, const float2* steer, float2* w, int* info,
                                 hipStream_t st, int waves);

hipError_t launch_bfused_bf16(const Dims& d, const float2* snap, const float2* steer, float2* w, int* info,
                              hipStream_t st, int waves) {
  if (bfused::pick_waves(d.D, waves) == 4) return launch_bfused_bf16_w4(d, snap, steer, w, info, st, waves);
  return bfused::single<1, 8>(d, snap, steer, w, info, st, waves);
}

}  // namespace stap
