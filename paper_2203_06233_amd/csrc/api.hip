// C ABI of libstap.so: host-side validation, workspace layout and the launch
// sequence of the STAP hot path.  Every argument check happens before the
// first HIP call, so invalid requests return an error without touching the
// device.
#include <math.h>
#include <string.h>

#include "common.h"
#include "kernels.h"

using stap::Dims;

namespace {

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

bool pow2_pulse(int p) {
  return p == 32 || p == 64 || p == 128 || p == 256 || p == 512;
}

stap_status check(const stap_problem* q) {
  if (!q) return STAP_ERR_ARG;
  if (q->reserved != 0) return STAP_ERR_ARG;
  if (!(q->load_eps >= 0.f) || !isfinite(q->load_eps)) return STAP_ERR_ARG;
  if (q->precision < STAP_PREC_FP32 || q->precision > STAP_PREC_FP8) return STAP_ERR_ARG;
  if (q->refine_steps < 0 || q->refine_steps > 4) return STAP_ERR_ARG;
  if (q->n_chan < 1 || q->n_range < 1 || q->n_block < 1 || q->n_steer < 1 || q->tdof < 1)
    return STAP_ERR_SHAPE;
  if (!pow2_pulse(q->n_pulse)) return STAP_ERR_SHAPE;
  if (q->tdof > stap::kMaxTdof || q->tdof >= q->n_pulse) return STAP_ERR_SHAPE;
  if ((long long)q->tdof * q->n_chan > stap::kMaxDof) return STAP_ERR_SHAPE;
  if (q->n_steer > stap::kMaxSteer) return STAP_ERR_SHAPE;
  if (q->n_range % q->n_block != 0) return STAP_ERR_SHAPE;
  if ((long long)q->n_pulse * q->n_block > 0x7fffffffLL) return STAP_ERR_SHAPE;
  const long long sp = q->cube_stride_pulse ? q->cube_stride_pulse : q->n_range;
  const long long sc = q->cube_stride_chan ? q->cube_stride_chan : (long long)q->n_pulse * sp;
  if (sp < q->n_range || sc < 0) return STAP_ERR_SHAPE;
  if (q->n_chan > 1 && sc < (long long)(q->n_pulse - 1) * sp + q->n_range) return STAP_ERR_SHAPE;
  return STAP_OK;
}

Dims dims_of(const stap_problem* q) {
  Dims d;
  d.C = q->n_chan;
  d.P = q->n_pulse;
  d.R = q->n_range;
  d.T = q->tdof;
  d.B = q->n_block;
  d.S = q->n_steer;
  d.D = d.T * d.C;
  d.N = d.R / d.B;
  d.L = d.P - d.T + 1;
  d.eps = q->load_eps;
  d.prec = q->precision;
  d.refine = q->refine_steps;
  d.sp = q->cube_stride_pulse ? q->cube_stride_pulse : d.R;
  d.sc = q->cube_stride_chan ? q->cube_stride_chan : (long long)d.P * d.sp;
  return d;
}

// The register-resident solve handles D <= 128.
stap_status check_solvable(const stap_problem* q) {
  return (q->tdof * q->n_chan > 128) ? STAP_ERR_UNSUPPORTED : STAP_OK;
}

stap_status hip_status(hipError_t e) { return e == hipSuccess ? STAP_OK : STAP_ERR_HIP; }

constexpr size_t kAlign = 256;
size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Parts {
  size_t snap, cov, delta, w, info;
};
Parts parts_of(const stap_problem* q) {
  const size_t P = q->n_pulse, D = (size_t)q->tdof * q->n_chan, R = q->n_range, B = q->n_block,
               S = q->n_steer;
  Parts p;
  p.snap = up(P * D * R * 8);
  p.cov = up(P * B * D * D * 8);
  p.delta = up(P * B * 4);
  p.w = up(P * B * S * D * 8);
  p.info = up(P * B * 4);
  return p;
}

}  // namespace

extern "C" {

stap_status stap_check_problem(const stap_problem* prob) { return check(prob); }

stap_status stap_doppler(const stap_problem* prob, const stap_cf32* cube, stap_cf32* snap, void* stream) {
  stap_status s = check(prob);
  if (s != STAP_OK) return s;
  if (!cube || !snap) return STAP_ERR_ARG;
  if (!aligned(cube, 8) || !aligned(snap, 8)) return STAP_ERR_ALIGN;
  const Dims d = dims_of(prob);
  return hip_status(stap::launch_doppler(d, reinterpret_cast<const float2*>(cube),
                                         reinterpret_cast<float2*>(snap), (hipStream_t)stream));
}

stap_status stap_covariance(const stap_problem* prob, const stap_cf32* snap, stap_cf32* cov, float* delta,
                            void* stream) {
  stap_status s = check(prob);
  if (s != STAP_OK) return s;
  if (!snap || !cov) return STAP_ERR_ARG;
  if (!aligned(snap, 8) || !aligned(cov, 8) || !aligned(delta, 4)) return STAP_ERR_ALIGN;
  const Dims d = dims_of(prob);
  return hip_status(stap::launch_covariance(d, reinterpret_cast<const float2*>(snap),
                                            reinterpret_cast<float2*>(cov), delta, (hipStream_t)stream));
}

stap_status stap_solve_weights(const stap_problem* prob, const stap_cf32* cov, const stap_cf32* steer,
                               stap_cf32* w, int32_t* info, void* stream) {
  stap_status s = check(prob);
  if (s != STAP_OK) return s;
  if (!cov || !steer || !w || !info) return STAP_ERR_ARG;
  if (!aligned(cov, 8) || !aligned(steer, 8) || !aligned(w, 8) || !aligned(info, 4)) return STAP_ERR_ALIGN;
  if ((s = check_solvable(prob)) != STAP_OK) return s;
  const Dims d = dims_of(prob);
  return hip_status(stap::launch_solve(d, reinterpret_cast<const float2*>(cov),
                                       reinterpret_cast<const float2*>(steer), reinterpret_cast<float2*>(w),
                                       info, (hipStream_t)stream));
}

stap_status stap_inner_products(const stap_problem* prob, const stap_cf32* w, const stap_cf32* snap,
                                float* power, stap_cf32* y, void* stream) {
  stap_status s = check(prob);
  if (s != STAP_OK) return s;
  if (!w || !snap || !power) return STAP_ERR_ARG;
  if (!aligned(w, 8) || !aligned(snap, 8) || !aligned(power, 4) || !aligned(y, 8)) return STAP_ERR_ALIGN;
  const Dims d = dims_of(prob);
  return hip_status(stap::launch_inner(d, reinterpret_cast<const float2*>(w),
                                       reinterpret_cast<const float2*>(snap), power,
                                       reinterpret_cast<float2*>(y), (hipStream_t)stream));
}

size_t stap_workspace_size(const stap_problem* probs, int32_t n_probs) {
  if (!probs || n_probs < 1) return 0;
  size_t total = 0;
  for (int i = 0; i < n_probs; ++i) {
    if (check(&probs[i]) != STAP_OK) return 0;
    const Parts p = parts_of(&probs[i]);
    total += p.snap + p.cov + p.delta + p.w + p.info;
  }
  return total;
}

stap_status stap_run(const stap_problem* probs, int32_t n_probs, const stap_cf32* const* cubes,
                     const stap_cf32* const* steers, float* const* powers, stap_cf32* const* weights,
                     int32_t* const* info, void* workspace, size_t workspace_bytes, void* stream) {
  if (!probs || n_probs < 1 || !cubes || !steers || !powers) return STAP_ERR_ARG;
  for (int i = 0; i < n_probs; ++i) {
    stap_status s = check(&probs[i]);
    if (s != STAP_OK) return s;
    if ((s = check_solvable(&probs[i])) != STAP_OK) return s;
    if (probs[i].precision != probs[0].precision || probs[i].refine_steps != probs[0].refine_steps)
      return STAP_ERR_ARG;
    if (!cubes[i] || !steers[i] || !powers[i]) return STAP_ERR_ARG;
    if (!aligned(cubes[i], 8) || !aligned(steers[i], 8) || !aligned(powers[i], 4)) return STAP_ERR_ALIGN;
    if (weights && !aligned(weights[i], 8)) return STAP_ERR_ALIGN;
    if (info && !aligned(info[i], 4)) return STAP_ERR_ALIGN;
  }
  const size_t need = stap_workspace_size(probs, n_probs);
  if (!workspace || workspace_bytes < need) return STAP_ERR_WORKSPACE;
  if (!aligned(workspace, kAlign)) return STAP_ERR_ALIGN;

  hipStream_t st = (hipStream_t)stream;
  char* ws = static_cast<char*>(workspace);
  for (int i = 0; i < n_probs; ++i) {
    const Dims d = dims_of(&probs[i]);
    const Parts p = parts_of(&probs[i]);
    float2* snap = reinterpret_cast<float2*>(ws);
    ws += p.snap;
    float2* cov = reinterpret_cast<float2*>(ws);
    ws += p.cov;
    float* delta = reinterpret_cast<float*>(ws);
    ws += p.delta;
    float2* w = reinterpret_cast<float2*>(ws);
    ws += p.w;
    int* inf = reinterpret_cast<int*>(ws);
    ws += p.info;
    if (weights && weights[i]) w = reinterpret_cast<float2*>(weights[i]);
    if (info && info[i]) inf = info[i];
    hipError_t e = stap::launch_doppler(d, reinterpret_cast<const float2*>(cubes[i]), snap, st);
    if (e == hipSuccess) e = stap::launch_covariance(d, snap, cov, delta, st);
    if (e == hipSuccess)
      e = stap::launch_solve(d, cov, reinterpret_cast<const float2*>(steers[i]), w, inf, st);
    if (e == hipSuccess) e = stap::launch_inner(d, w, snap, powers[i], nullptr, st);
    if (e != hipSuccess) return STAP_ERR_HIP;
  }
  return STAP_OK;
}

const char* stap_status_string(stap_status status) {
  switch (status) {
    case STAP_OK: return "ok";
    case STAP_ERR_ARG: return "invalid argument (null pointer or value out of range)";
    case STAP_ERR_SHAPE: return "dimensions outside the supported limits";
    case STAP_ERR_ALIGN: return "misaligned device pointer";
    case STAP_ERR_WORKSPACE: return "workspace missing or too small";
    case STAP_ERR_HIP: return "HIP runtime error";
    case STAP_ERR_UNSUPPORTED: return "request not supported by this build";
  }
  return "unknown status";
}

const char* stap_version(void) { return "0.1.0"; }

}  // extern "C"
