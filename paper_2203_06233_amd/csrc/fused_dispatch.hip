// Dispatch of the fused covariance -> solve kernel between its thread grids.
#include "kernels.h"

namespace stap {

bool fused_supported(const Dims& d) { return d.D <= 128 && d.prec != STAP_PREC_FP8; }

hipError_t launch_bfused_f32(const Dims& d, const float2* snap, const float2* steer, float2* w, int* info,
                             hipStream_t st, int waves);
hipError_t launch_bfused_bf16(const Dims& d, const float2* snap, const float2* steer, float2* w, int* info,
                              hipStream_t st, int waves);
hipError_t launch_bfused_batched_f32(const ProbDesc* desc, int n, long long total, int max_dof, int max_steer,
                                     int refine, int waves, hipStream_t st, unsigned long long* queue);
hipError_t launch_bfused_batched_bf16(const ProbDesc* desc, int n, long long total, int max_dof, int max_steer,
                                      int refine, int waves, hipStream_t st, unsigned long long* queue);

bool bfused_supported(const Dims& d) { return fused_supported(d); }

hipError_t launch_fused(const Dims& d, const float2* snap, const float2* steer, float2* w, int* info,
                        hipStream_t st, int ty) {
  if (!fused_supported(d)) return hipErrorInvalidValue;
  if ((ty == 4 || ty == 8) && bfused_supported(d))
    return d.prec == STAP_PREC_FP32 ? launch_bfused_f32(d, snap, steer, w, info, st, ty)
                                    : launch_bfused_bf16(d, snap, steer, w, info, st, ty);
  if (ty == 32 && d.D > 32) return launch_fused32(d, snap, steer, w, info, st);
  return launch_fused16(d, snap, steer, w, info, st);
}

hipError_t launch_fused_batched16(const ProbDesc* desc, int n, long long total, int max_dof, int max_steer,
                                  int prec, int refine, hipStream_t st, unsigned long long* queue);
hipError_t launch_fused_batched32(const ProbDesc* desc, int n, long long total, int max_dof, int max_steer,
                                  int prec, int refine, hipStream_t st, unsigned long long* queue);

hipError_t launch_fused_batched(const ProbDesc* desc, int n, long long total_sys, int max_dof, int max_steer,
                                int prec, int refine, int ty, hipStream_t st, unsigned long long* queue) {
  if (max_dof > 128 || prec == STAP_PREC_FP8 || total_sys <= 0) return hipErrorInvalidValue;
  if (ty == 4 || ty == 8)
    return prec == STAP_PREC_FP32 ? launch_bfused_batched_f32(desc, n, total_sys, max_dof, max_steer, refine, ty, st, queue)
                                  : launch_bfused_batched_bf16(desc, n, total_sys, max_dof, max_steer, refine, ty, st, queue);
  if (ty == 32 && max_dof > 32) return launch_fused_batched32(desc, n, total_sys, max_dof, max_steer, prec, refine, st, queue);
  return launch_fused_batched16(desc, n, total_sys, max_dof, max_steer, prec, refine, st, queue);
}

}  // namespace stap
