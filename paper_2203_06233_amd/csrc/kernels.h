// Launchers of the gfx950 kernels (internal to libstap.so).  Each enqueues on
// `st` and returns the launch status; shapes are validated by the caller.
#pragma once

#include "common.h"

namespace stap {

// X[P][D][R] <- windowed, time-staggered Doppler DFT of cube[C][P][R].
hipError_t launch_doppler(const Dims& d, const float2* cube, float2* snap, hipStream_t st);

// cov[P][B][D][D] (loaded, full Hermitian) and delta[P][B] from X.
hipError_t launch_covariance(const Dims& d, const float2* snap, float2* cov, float* delta,
                             hipStream_t st);

// W[P][B][S][D] and info[P][B] from loaded covariances and steering V[S][D].
hipError_t launch_solve(const Dims& d, const float2* cov, const float2* steer, float2* w, int* info,
                        hipStream_t st);

// power[P][S][R] (and y if non-null) from W and X.
hipError_t launch_inner(const Dims& d, const float2* w, const float2* snap, float* power, float2* y,
                        hipStream_t st);

}  // namespace stap
