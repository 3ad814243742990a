// Cell-averaging CFAR detection along range on the AMF power map
// power[P][S][R] (the textbook CA-CFAR detector applied to the output of the
// STAP chain; not part of the paper's kernel, which ends at the output
// power).  For cell r of a row the reference cells are n_ref cells on each
// side beyond n_guard guard cells; cells outside [0, R) are left out and
// n_used counts the rest.  Detection: power[r] * n_used > alpha * sum.
//
// The decision is an integer result of floating-point arithmetic, so its
// arithmetic is fixed: the reference cells are added in FP64, one at a time,
// in increasing offset order (left window, then right window, a missing
// cell adding 0), and the test is taken in FP64 with no fused multiply-add.
// Any implementation that keeps this order returns the same mask bit for bit.
//
// One workgroup takes kTile cells of one (bin, steering) row plus a halo of
// n_guard + n_ref cells per side, staged once through LDS (one pad word
// every 32, so the lanes' strided reads fall in distinct banks).  Each thread
// owns kRun consecutive cells and slides a ring of kRun window values in
// registers over each window: one LDS read and one conversion per step feed
// kRun FP64 additions, so the kernel is bound by the FP64 adds (2 n_ref per
// cell) and the HBM traffic (4 bytes in, 1 byte out per cell).
#include "common.h"
#include "kernels.h"

namespace stap {

namespace {

constexpr int kRun = 8;                   // consecutive cells per thread
constexpr int kThreads = 256;
constexpr int kTile = kRun * kThreads;    // cells per workgroup
constexpr int kMaxHalo = kMaxCfarRef + kMaxCfarGuard;
constexpr int kSpan = kTile + 2 * kMaxHalo;
constexpr int kLdsWords = (kSpan + kRun) + (kSpan + kRun) / 32 + 1;  // + the ring's look-ahead

__device__ __forceinline__ int lds_index(int i) { return i + (i >> 5); }

// Sum of n window values in order for each of the thread's kRun cells: cell j
// adds w[j], w[j+1], ..., w[j+n-1] with w[m] = lds value at index base + m.
__device__ __forceinline__ void window_sums(const float* s, int base, int n, double (&acc)[kRun]) {
  double ring[kRun];
#pragma unroll
  for (int m = 0; m < kRun; ++m) ring[m] = (double)s[lds_index(base + m)];
  for (int i0 = 0; i0 < n; i0 += kRun) {
#pragma unroll
    for (int u = 0; u < kRun; ++u) {
      if (i0 + u < n) {
        // step i = i0 + u: ring slot (i + j) % kRun holds w[i + j]
#pragma unroll
        for (int j = 0; j < kRun; ++j) acc[j] += ring[(u + j) % kRun];
        ring[u] = (double)s[lds_index(base + i0 + u + kRun)];
      }
    }
  }
}

__global__ __launch_bounds__(kThreads) void cfar_kernel(const float* __restrict__ power,
                                                        unsigned char* __restrict__ detect, int R, int tiles_per_row,
                                                        int n_ref, int n_guard, double alpha) {
#pragma clang fp contract(off)
  __shared__ float s[kLdsWords];
  const int row = blockIdx.x / tiles_per_row;
  const int tile = blockIdx.x - row * tiles_per_row;
  const int t0 = tile * kTile;          // first cell of the tile
  const int H = n_ref + n_guard;        // halo per side
  const int span = kTile + 2 * H;
  const float* prow = power + (long long)row * R;
  // stage cells t0 - H .. t0 + kTile + H - 1 (zero outside the row), plus
  // kRun spare zeros for the ring's look-ahead
  for (int i = threadIdx.x; i < span + kRun; i += kThreads) {
    const int c = t0 - H + i;
    s[lds_index(i)] = (i < span && c >= 0 && c < R) ? prow[c] : 0.f;
  }
  __syncthreads();

  const int c0 = t0 + kRun * threadIdx.x;  // the thread's first cell
  if (c0 >= R) return;
  double acc[kRun];
#pragma unroll
  for (int j = 0; j < kRun; ++j) acc[j] = 0.0;
  // local index of cell c is c - t0 + H
  window_sums(s, c0 - n_guard - n_ref - t0 + H, n_ref, acc);  // left: offsets -(g+n) .. -(g+1)
  window_sums(s, c0 + n_guard + 1 - t0 + H, n_ref, acc);      // right: offsets g+1 .. g+n
  unsigned long long bits = 0;
#pragma unroll
  for (int j = 0; j < kRun; ++j) {
    const int c = c0 + j;
    // reference cells that exist: left [c-g-n, c-g-1], right [c+g+1, c+g+n]
    const int l_lo = max(c - n_guard - n_ref, 0), l_hi = min(c - n_guard - 1, R - 1);
    const int r_lo = max(c + n_guard + 1, 0), r_hi = min(c + n_guard + n_ref, R - 1);
    const int used = max(l_hi - l_lo + 1, 0) + max(r_hi - r_lo + 1, 0);
    const double p = (double)s[lds_index(c - t0 + H)];
    const bool hit = c < R && p * (double)used > alpha * acc[j];
    bits |= (unsigned long long)(hit ? 1u : 0u) << (8 * j);
  }
  unsigned char* out = detect + (long long)row * R + c0;
  if (c0 + kRun <= R && ((reinterpret_cast<uintptr_t>(out) & 7) == 0)) {
    *reinterpret_cast<unsigned long long*>(out) = bits;
  } else {
#pragma unroll
    for (int j = 0; j < kRun; ++j)
      if (c0 + j < R) out[j] = (unsigned char)((bits >> (8 * j)) & 1u);
  }
}

}  // namespace

hipError_t launch_cfar(const Dims& d, int n_ref, int n_guard, double alpha, const float* power,
                       unsigned char* detect, hipStream_t st) {
  const int tiles = (d.R + kTile - 1) / kTile;
  const long long rows = (long long)d.P * d.S;
  if (rows * tiles > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(cfar_kernel, dim3((unsigned)(rows * tiles)), dim3(kThreads), 0, st, power, detect, d.R, tiles,
                     n_ref, n_guard, alpha);
  return hipGetLastError();
}

}  // namespace stap
