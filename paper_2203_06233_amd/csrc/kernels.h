// Launchers of the gfx950 kernels (internal to libstap.so).  Each enqueues on
// `st` and returns the launch status; shapes are validated by the caller.
#pragma once

#include "common.h"

namespace stap {

// One cube of a batched stap_run, as the kernels read it from the device
// table in the workspace.
struct ProbDesc {
  Dims d;
  const float2* cube;
  const float2* steer;
  float* power;
  float2* w;
  int* info;
  float2* snap;
  long long sys_begin;  // first system index within the cube's shape class of the batch
};

// Kernel argument of a batched Doppler launch: up to kMaxBatchArg cubes with
// the same P, their indices in the table and their first workgroup.
constexpr int kMaxBatchArg = 64;
struct BatchIndex {
  int n;
  int prob[kMaxBatchArg];
  int tile_begin[kMaxBatchArg + 1];
};

// Workgroups of the Doppler kernel for one cube; batched Doppler launch.
int doppler_tiles(const Dims& d);
hipError_t launch_doppler_batched(int P, const ProbDesc* desc, const BatchIndex& bi, int tiles, hipStream_t st);

// Persistent fused covariance -> solve over every system of every cube of the
// table (all fused_supported, one precision; max_dof / max_steer the largest
// D and S): workgroups take systems from the work queue `queue`, a counter
// that must be zero at launch.
hipError_t launch_fused_batched(const ProbDesc* desc, int n, long long total_sys, int max_dof, int max_steer,
                                int prec, int refine, int ty, hipStream_t st, unsigned long long* queue);

// Inner products over every system of every cube of the table.
hipError_t launch_inner_batched(const ProbDesc* desc, int n, long long total_sys, int max_dof, int max_steer,
                                int prec, hipStream_t st);

// X[P][D][R] <- windowed, time-staggered Doppler DFT of cube[C][P][R].
hipError_t launch_doppler(const Dims& d, const float2* cube, float2* snap, hipStream_t st);

// cov[P][B][D][D] (loaded, full Hermitian) and delta[P][B] from X; nw =
// waves per system (0 = default of the DOF class).
hipError_t launch_covariance(const Dims& d, const float2* snap, float2* cov, float* delta,
                             hipStream_t st, int nw = 0);

// W[P][B][S][D] and info[P][B] from loaded covariances and steering V[S][D].
hipError_t launch_solve(const Dims& d, const float2* cov, const float2* steer, float2* w, int* info,
                        hipStream_t st);

// Blocked matrix-core solve with 4 or 8 waves per system (8 means 16 for
// D > 128).
bool bsolve_supported(const Dims& d, int waves);
// one wave per system, every block in registers (D <= 96, S <= 32)
bool wsolve_supported(const Dims& d);
hipError_t launch_wsolve(const Dims& d, const float2* cov, const float2* steer, float2* w, int* info,
                         hipStream_t st);
hipError_t launch_bsolve(const Dims& d, const float2* cov, const float2* steer, float2* w, int* info,
                         hipStream_t st, int waves);

// Fused covariance -> solve (D <= 128, FP32 or BF16): W and info from X.
// `ty` selects the thread grid (16 x 16 or 32 x 16; 32 needs D > 32).
bool fused_supported(const Dims& d);
hipError_t launch_fused(const Dims& d, const float2* snap, const float2* steer, float2* w, int* info,
                        hipStream_t st, int ty);
hipError_t launch_fused16(const Dims& d, const float2* snap, const float2* steer, float2* w, int* info,
                          hipStream_t st);
hipError_t launch_fused32(const Dims& d, const float2* snap, const float2* steer, float2* w, int* info,
                          hipStream_t st);

// detect[P][S][R] (1 = detection) from power[P][S][R] by CA-CFAR along range.
hipError_t launch_cfar(const Dims& d, int n_ref, int n_guard, double alpha, const float* power,
                       unsigned char* detect, hipStream_t st);

// power[P][S][R] (and y if non-null) from W and X; rtw = range tiles per
// wave step (0 = default).
hipError_t launch_inner(const Dims& d, const float2* w, const float2* snap, float* power, float2* y,
                        hipStream_t st, int rtw = 0);

}  // namespace stap
