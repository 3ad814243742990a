// Fused covariance -> Cholesky -> solve per system (the path of stap_run):
// the loaded covariance of a (Doppler bin, training block) never leaves the
// compute unit.
//   phase 1  cov_accumulate() (cov_impl.h) on MFMA; the FP64 trace gives
//            delta; the tiles are written into LDS as the packed lower
//            triangle of R_L, reusing the snapshot staging buffer;
//   phase 2  solve_system() (solve_impl.h) reads R_L from that packed copy,
//            which also feeds the FP64 refinement residual.
// Compared with the stage kernels this saves the covariance round trip
// through HBM (P*B*D*D*8 bytes written and half of it read back).
#pragma once

#include "bsolve_impl.h"
#include "common.h"
#include "cov_impl.h"
#include "kernels.h"
#include "solve_impl.h"

namespace stap {


struct PackedR {
  const float2* Rp;
  __device__ float2 lower(int i, int k) const { return Rp[i * (i + 1) / 2 + k]; }
};

// System `sys` of one cube: wout and info_out are the cube's arrays.
template <int TY, int NA, int NB, int NVS, int MODE, bool REFINE>
__device__ __forceinline__ void fused_system(const float2* __restrict__ snap, const float2* __restrict__ steer,
                                             float2* __restrict__ wout, int* __restrict__ info_out,
                                             const Dims& d, int sys) {
  using K = SolveCfg<TY, NA, NB, NVS>;
  using C = CovCfg<K::DPC, K::NT / 64, MODE>;
  constexpr int PACK = (K::kPacked + (REFINE ? K::kSlab : 0)) * 8;  // packed R_L (+ residual slab)
  constexpr int BYTES = C::LDS_BYTES > PACK ? C::LDS_BYTES : PACK;
  __shared__ __align__(16) unsigned char lds[BYTES];
  __shared__ SolveShared<K> sh;
  __shared__ double dsum[K::DPC];
  __shared__ float red[K::NT / 64];
  __shared__ float s_delta;

  const int k = sys / d.B, b = sys - (sys / d.B) * d.B;
  const int D = d.D;
  const float2* X = snap + (long long)k * D * d.R;
  floatx4 accR[C::TPW], accI[C::TPW];
  cov_accumulate<C>(X, d.R, D, d.N, train_cells(d, b), lds, red, accR, accI);
  const float dl = cov_delta<C>(accR, D, d.eps, dsum, &s_delta);
  __syncthreads();  // the staging buffer is dead: reuse it for R_L
  float2* Rp = reinterpret_cast<float2*>(lds);
  cov_emit<C>(accR, accI, D, dl, [&](int row, int col, float2 v) { Rp[row * (row + 1) / 2 + col] = v; });
  __syncthreads();
  solve_system<K, REFINE, true>(PackedR{Rp}, Rp, Rp + K::kPacked, steer + steer_offset(d, sys),
                                wout + (long long)sys * d.S * D,
                                info_out ? info_out + sys : nullptr, d, sh);
}


template <int TY, int NA, int NB, int NVS, int MODE, bool REFINE>
__global__ __launch_bounds__(16 * TY) void fused_kernel(const float2* __restrict__ snap,
                                                        const float2* __restrict__ steer,
                                                        float2* __restrict__ wout, int* __restrict__ info_out,
                                                        Dims d) {
  fused_system<TY, NA, NB, NVS, MODE, REFINE>(snap, steer, wout, info_out, d, blockIdx.x);
}

// Persistent workgroups take the next system from a device work queue: one
// 64-bit counter (reset by the launch that writes the problem table) that
// each workgroup advances atomically when it finishes a system.  Cubes are
// ordered by cost (largest first), so the most expensive systems are handed
// out first and the cheap ones fill in behind them.  Every workgroup leaves
// when the counter has passed the last system.
__device__ __forceinline__ long long next_system(unsigned long long* queue, long long* slot) {
  if (lane_tid() == 0) *slot = (long long)atomicAdd(queue, 1ULL);
  __syncthreads();
  const long long g = *slot;
  __syncthreads();  // every thread has read the slot before the next claim overwrites it
  return g;
}

template <int TY, int NA, int NB, int NVS, int MODE, bool REFINE>
__global__ __launch_bounds__(16 * TY) void fused_batched_kernel(const ProbDesc* __restrict__ desc, int n,
                                                                long long total, unsigned long long* queue) {
  __shared__ long long slot;
  for (long long g = next_system(queue, &slot); g < total; g = next_system(queue, &slot)) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (desc[mid].sys_begin <= g) lo = mid;
      else hi = mid - 1;
    }
    const ProbDesc& pd = desc[lo];
    const Dims d = pd.d;
    fused_system<TY, NA, NB, NVS, MODE, REFINE>(pd.snap, pd.steer, pd.w, pd.info, d, (int)(g - pd.sys_begin));
    __syncthreads();
  }
}

// The same with the blocked matrix-core solve (bsolve_impl.h): NB block
// columns of the covariance (compile time, for the covariance tiles), NS
// steering blocks at most, NW waves, NSL / NSM register blocks per wave.  With REFINE the packed R_L stays in LDS for the FP64 residual and the
// solver's exchange blocks follow it; without, they reuse the same bytes.
template <int NB, int NS, int NSL, int NSM, int NW, int MODE, bool REFINE>
__device__ __forceinline__ void bfused_system(const float2* __restrict__ snap, const float2* __restrict__ steer,
                                              float2* __restrict__ wout, int* __restrict__ info_out,
                                              const Dims& d, int sys) {
  using C = CovCfg<16 * NB, NW, MODE>;
  using B = BCfg<NSL, NSM, NW>;
  constexpr int PACK = (16 * NB * (16 * NB + 1) / 2 * 8 + 255) / 256 * 256;
  constexpr int EXCH = (int)B::lds_bytes(NB, NS);
  constexpr int B1 = C::LDS_BYTES > PACK ? C::LDS_BYTES : PACK;
  constexpr int B2 = REFINE ? PACK + EXCH : EXCH;
  constexpr int BYTES = B1 > B2 ? B1 : B2;
  __shared__ __align__(16) unsigned char lds[BYTES];
  __shared__ double dsum[16 * NB];
  __shared__ float red[NW];
  __shared__ float s_delta;

  const int k = sys / d.B, b = sys - (sys / d.B) * d.B;
  const int D = d.D;
  const float2* X = snap + (long long)k * D * d.R;
  floatx4 accR[C::TPW], accI[C::TPW];
  cov_accumulate<C>(X, d.R, D, d.N, train_cells(d, b), lds, red, accR, accI);
  const float dl = cov_delta<C>(accR, D, d.eps, dsum, &s_delta);
  __syncthreads();
  float2* Rp = reinterpret_cast<float2*>(lds);
  cov_emit<C>(accR, accI, D, dl, [&](int row, int col, float2 v) { Rp[row * (row + 1) / 2 + col] = v; });
  __syncthreads();
  // the packed R_L is dead after the last residual: u of that step is kept
  // there when it fits
  constexpr bool PARK = REFINE && PACK >= NS * NB * 256 * 8;
  bsolve_system<B, REFINE>(PackedR{Rp}, steer + steer_offset(d, sys), wout + (long long)sys * d.S * D,
                           info_out ? info_out + sys : nullptr,
                           d, lds + (REFINE ? PACK : 0), PARK ? Rp : nullptr);
}

// With 8 waves and up to 6 block columns the register allocation is capped
// at 128 so that two systems share a compute unit (with refinement a few
// registers spill).  With 4 waves and up to 2 block rows of steering
// vectors: the one-cube kernel is capped at 168 up to 4 block columns (three
// systems per compute unit instead of two); the persistent batched kernel,
// which left to itself holds more registers across its loop (up to 196),
// at 128 up to 2 block columns and 168 at 3 (four and three systems per
// compute unit) -- all without spills.
template <int NB, int NS, int NW, bool BATCHED>
constexpr int bfused_min_waves() {
  if (NW == 8 && NB <= 6) return 4;
  if (NW == 4 && NS <= 2) return BATCHED ? (NB <= 2 ? 4 : NB == 3 ? 3 : 1) : (NB <= 4 ? 3 : 1);
  return 1;
}

template <int NB, int NS, int NSL, int NSM, int NW, int MODE, bool REFINE>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(bfused_min_waves<NB, NS, NW, false>())))
void bfused_kernel(const float2* __restrict__ snap,
                                                         const float2* __restrict__ steer,
                                                         float2* __restrict__ wout, int* __restrict__ info_out,
                                                         Dims d) {
  bfused_system<NB, NS, NSL, NSM, NW, MODE, REFINE>(snap, steer, wout, info_out, d, blockIdx.x);
}

template <int NB, int NS, int NSL, int NSM, int NW, int MODE, bool REFINE>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(bfused_min_waves<NB, NS, NW, true>())))
void bfused_batched_kernel(const ProbDesc* __restrict__ desc, int n,
                                                                 long long total, unsigned long long* queue) {
  __shared__ long long slot;
  for (long long g = next_system(queue, &slot); g < total; g = next_system(queue, &slot)) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (desc[mid].sys_begin <= g) lo = mid;
      else hi = mid - 1;
    }
    const ProbDesc& pd = desc[lo];
    const Dims d = pd.d;
    bfused_system<NB, NS, NSL, NSM, NW, MODE, REFINE>(pd.snap, pd.steer, pd.w, pd.info, d, (int)(g - pd.sys_begin));
    __syncthreads();
  }
}

template <int TY, int NA, int NB, int NVS, int MODE>
hipError_t go_fused_batched(const ProbDesc* desc, int n, long long total, int refine, hipStream_t st,
                            unsigned long long* queue) {
  // enough workgroups to fill every CU a few times over, never more than systems
  const long long want = 256LL * (TY == 16 ? 4 : 2);
  const dim3 grid((unsigned)(total < want ? total : want)), block(16 * TY);
  if (refine == 0)
    hipLaunchKernelGGL((fused_batched_kernel<TY, NA, NB, NVS, MODE, false>), grid, block, 0, st, desc, n, total,
                       queue);
  else
    hipLaunchKernelGGL((fused_batched_kernel<TY, NA, NB, NVS, MODE, true>), grid, block, 0, st, desc, n, total,
                       queue);
  return hipGetLastError();
}

template <int TY, int NA, int NB, int NVS, int MODE>
hipError_t go_fused(const Dims& d, const float2* snap, const float2* steer, float2* w, int* info,
                    hipStream_t st) {
  const dim3 grid(d.P * d.B), block(16 * TY);
  if (d.refine == 0)
    hipLaunchKernelGGL((fused_kernel<TY, NA, NB, NVS, MODE, false>), grid, block, 0, st, snap, steer, w, info, d);
  else
    hipLaunchKernelGGL((fused_kernel<TY, NA, NB, NVS, MODE, true>), grid, block, 0, st, snap, steer, w, info, d);
  return hipGetLastError();
}

}  // namespace stap
