// Fused covariance -> blocked matrix-core solve, split-BF16, batched covariance products.
#include "bfused_launch.h"

namespace stap {

hipError_t launch_bfused_batched_bf16(const ProbDesc* desc, int n, long long total, int max_dof, int max_steer,
                                     int refine, int waves, hipStream_t st, unsigned long long* queue) {
  return bfused::batched<1>(desc, n, total, max_dof, max_steer, refine, waves, st, queue);
}

}  // namespace stap
