// Fused covariance -> solve, 32 x 16 thread grid (fused_impl.h): twice the
// threads per system, half the registers per thread; for D in (32, 128].
#include "fused_impl.h"

namespace stap {

namespace {

template <int NB, int MODE>
hipError_t go32_s(const Dims& d, const float2* snap, const float2* steer, float2* w, int* info,
                  hipStream_t st) {
  constexpr int NA = (16 * NB + 31) / 32;
  if (d.S <= 32) return go_fused<32, NA, NB, 1, MODE>(d, snap, steer, w, info, st);
  return go_fused<32, NA, NB, 2, MODE>(d, snap, steer, w, info, st);
}

template <int MODE>
hipError_t go32_d(const Dims& d, const float2* snap, const float2* steer, float2* w, int* info,
                  hipStream_t st) {
  if (d.D <= 48) return go32_s<3, MODE>(d, snap, steer, w, info, st);
  if (d.D <= 64) return go32_s<4, MODE>(d, snap, steer, w, info, st);
  if (d.D <= 96) return go32_s<6, MODE>(d, snap, steer, w, info, st);
  return go32_s<8, MODE>(d, snap, steer, w, info, st);
}

template <int NB, int MODE>
hipError_t gob32_s(const ProbDesc* desc, int n, long long total, int max_steer, int refine, hipStream_t st,
                    unsigned long long* queue) {
  constexpr int NA = (16 * NB + 31) / 32;
  if (max_steer <= 32) return go_fused_batched<32, NA, NB, 1, MODE>(desc, n, total, refine, st, queue);
  return go_fused_batched<32, NA, NB, 2, MODE>(desc, n, total, refine, st, queue);
}

template <int MODE>
hipError_t gob32_d(const ProbDesc* desc, int n, long long total, int max_dof, int max_steer, int refine,
                   hipStream_t st, unsigned long long* queue) {
  if (max_dof <= 48) return gob32_s<3, MODE>(desc, n, total, max_steer, refine, st, queue);
  if (max_dof <= 64) return gob32_s<4, MODE>(desc, n, total, max_steer, refine, st, queue);
  if (max_dof <= 96) return gob32_s<6, MODE>(desc, n, total, max_steer, refine, st, queue);
  return gob32_s<8, MODE>(desc, n, total, max_steer, refine, st, queue);
}

}  // namespace

hipError_t launch_fused_batched32(const ProbDesc* desc, int n, long long total, int max_dof, int max_steer,
                                  int prec, int refine, hipStream_t st, unsigned long long* queue) {
  return prec == STAP_PREC_FP32 ? gob32_d<0>(desc, n, total, max_dof, max_steer, refine, st, queue)
                                : gob32_d<1>(desc, n, total, max_dof, max_steer, refine, st, queue);
}

hipError_t launch_fused32(const Dims& d, const float2* snap, const float2* steer, float2* w, int* info,
                          hipStream_t st) {
  return d.prec == STAP_PREC_FP32 ? go32_d<0>(d, snap, steer, w, info, st)
                                  : go32_d<1>(d, snap, steer, w, info, st);
}

}  // namespace stap
