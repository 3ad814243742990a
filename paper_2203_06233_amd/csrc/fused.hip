// Fused covariance -> solve, 16 x 16 thread grid (fused_impl.h).
#include "fused_impl.h"

namespace stap {

namespace {

template <int NB, int MODE>
hipError_t go16_s(const Dims& d, const float2* snap, const float2* steer, float2* w, int* info,
                  hipStream_t st) {
  if (d.S <= 16) return go_fused<16, NB, NB, 1, MODE>(d, snap, steer, w, info, st);
  if (d.S <= 32) return go_fused<16, NB, NB, 2, MODE>(d, snap, steer, w, info, st);
  return go_fused<16, NB, NB, 4, MODE>(d, snap, steer, w, info, st);
}

template <int MODE>
hipError_t go16_d(const Dims& d, const float2* snap, const float2* steer, float2* w, int* info,
                  hipStream_t st) {
  if (d.D <= 16) return go16_s<1, MODE>(d, snap, steer, w, info, st);
  if (d.D <= 32) return go16_s<2, MODE>(d, snap, steer, w, info, st);
  if (d.D <= 48) return go16_s<3, MODE>(d, snap, steer, w, info, st);
  if (d.D <= 64) return go16_s<4, MODE>(d, snap, steer, w, info, st);
  if (d.D <= 96) return go16_s<6, MODE>(d, snap, steer, w, info, st);
  return go16_s<8, MODE>(d, snap, steer, w, info, st);
}

template <int NB, int MODE>
hipError_t gob16_s(const ProbDesc* desc, int n, long long total, int max_steer, int refine, hipStream_t st,
                    unsigned long long* queue) {
  if (max_steer <= 16) return go_fused_batched<16, NB, NB, 1, MODE>(desc, n, total, refine, st, queue);
  if (max_steer <= 32) return go_fused_batched<16, NB, NB, 2, MODE>(desc, n, total, refine, st, queue);
  return go_fused_batched<16, NB, NB, 4, MODE>(desc, n, total, refine, st, queue);
}

template <int MODE>
hipError_t gob16_d(const ProbDesc* desc, int n, long long total, int max_dof, int max_steer, int refine,
                   hipStream_t st, unsigned long long* queue) {
  if (max_dof <= 16) return gob16_s<1, MODE>(desc, n, total, max_steer, refine, st, queue);
  if (max_dof <= 32) return gob16_s<2, MODE>(desc, n, total, max_steer, refine, st, queue);
  if (max_dof <= 48) return gob16_s<3, MODE>(desc, n, total, max_steer, refine, st, queue);
  if (max_dof <= 64) return gob16_s<4, MODE>(desc, n, total, max_steer, refine, st, queue);
  if (max_dof <= 96) return gob16_s<6, MODE>(desc, n, total, max_steer, refine, st, queue);
  return gob16_s<8, MODE>(desc, n, total, max_steer, refine, st, queue);
}

}  // namespace

hipError_t launch_fused_batched16(const ProbDesc* desc, int n, long long total, int max_dof, int max_steer,
                                  int prec, int refine, hipStream_t st, unsigned long long* queue) {
  return prec == STAP_PREC_FP32 ? gob16_d<0>(desc, n, total, max_dof, max_steer, refine, st, queue)
                                : gob16_d<1>(desc, n, total, max_dof, max_steer, refine, st, queue);
}

hipError_t launch_fused16(const Dims& d, const float2* snap, const float2* steer, float2* w, int* info,
                          hipStream_t st) {
  return d.prec == STAP_PREC_FP32 ? go16_d<0>(d, snap, steer, w, info, st)
                                  : go16_d<1>(d, snap, steer, w, info, st);
}

}  // namespace stap
