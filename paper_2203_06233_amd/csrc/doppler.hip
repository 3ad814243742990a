// Doppler filtering with time-staggered DOF (statements S and T of the STAP
// kernel, Sec. 4.2; Table 2 row fft_{2D,axis=1}).
//
//   X[k][t*C+c][r] = sum_p h[p-t] x[c][p][r] exp(-2 pi i k p / P)
//
// or, with each tap referenced to its own first pulse (relative phase),
// exp(-2 pi i k (p - t) / P), i.e. the absolute form times exp(2 pi i k t / P).
//
// One workgroup takes one channel c and RT consecutive range cells.  The
// length-P DFT is split as P = P1 * P2 (p = P2*n1 + n2, k = k1 + P1*k2):
//   pass 1  each thread owns one (n2, cell) and keeps the P1 samples
//           x[P2*n1 + n2], n1 = 0..P1-1, in registers (loaded once, coalesced
//           along range), windows them for tap t, runs a P1-point DFT in
//           registers and multiplies by exp(-2 pi i k1 n2 / P);
//   LDS     one transpose through a [k1][n2][cell] tile;
//   pass 2  each (k1, cell) runs a P2-point DFT in registers and stores bins
//           k1 + P1*k2 straight to X[k][d][r] (range fastest, coalesced).
// The cube is read from HBM once for all T taps; with subarrays, each
// channel's samples are the sum of its elements, formed as they are loaded.
// P = 100 (the paper's pulse count) runs the same passes as 10 x 10 with
// direct in-register DFTs.  Twiddles of the inner DFTs
// are compile-time constants; the P-point twiddles and the Hann window come
// from correctly rounded compile-time tables, staged once per workgroup in LDS.
#include "common.h"
#include "kernels.h"

namespace stap {

template <int P>
struct FftShape {
  static constexpr int LOG = ilog2(P);
  static constexpr int P1 = 1 << ((LOG + 1) / 2);
  static constexpr int P2 = P / P1;
  static constexpr int NT = 256;       // threads per workgroup
  static constexpr int RT = NT / P2;   // range cells per workgroup
};
// The paper's 100 pulses: 10 x 10 on 320 threads, 32 cells per workgroup, so
// that every wave reads whole 128-byte lines of two pulse rows.
template <>
struct FftShape<100> {
  static constexpr int P1 = 10, P2 = 10, NT = 320, RT = 32;
};

// One workgroup's tile: channel c, range cells r0 .. r0+RT-1 of one cube.
template <int P>
__device__ __forceinline__ void doppler_tile(const float2* __restrict__ cube, float2* __restrict__ snap,
                                             const Dims& d, int c, int r0) {
  using Sh = FftShape<P>;
  constexpr int P1 = Sh::P1, P2 = Sh::P2, RT = Sh::RT, NT = Sh::NT;
  __shared__ float2 ybuf[P1 * P2 * RT];  // [k1][n2][cell]
  __shared__ float2 tw[P];
  __shared__ float hwin[P];

  const int tid = threadIdx.x;

  for (int m = tid; m < P; m += NT) {
    tw[m] = make_float2(kTwTab<P>.c[m], -kTwTab<P>.s[m]);
    hwin[m] = kWinTab<P>.h[d.T - 1][m];
  }

  const int col = tid % RT, n2 = tid / RT;
  const int r = r0 + col;
  const bool live = r < d.R && n2 < P2;
  float2 x[P1];
#pragma unroll
  for (int n1 = 0; n1 < P1; ++n1) x[n1] = make_float2(0.f, 0.f);
  if (live && d.sub == 1) {
    const float2* src = cube + (long long)c * d.sc + r;
#pragma unroll
    for (int n1 = 0; n1 < P1; ++n1) x[n1] = load_stream(src + (long long)(P2 * n1 + n2) * d.sp);
  } else if (live) {
    // channel c is the sum of array elements c*sub .. c*sub + sub - 1,
    // added in element order; with few samples per thread the loads of four
    // elements are issued before their additions so that enough of them are
    // in flight to stream the cube (more would cost the registers that set
    // the occupancy of the whole kernel)
    constexpr int EU = P1 <= 10 ? 4 : 1;
    int e = 0;
    for (; e + EU <= d.sub; e += EU) {
      float2 v[EU][P1];
#pragma unroll
      for (int u = 0; u < EU; ++u) {
        const float2* src = cube + (long long)(c * d.sub + e + u) * d.sc + r;
#pragma unroll
        for (int n1 = 0; n1 < P1; ++n1) v[u][n1] = load_stream(src + (long long)(P2 * n1 + n2) * d.sp);
      }
#pragma unroll
      for (int u = 0; u < EU; ++u)
#pragma unroll
        for (int n1 = 0; n1 < P1; ++n1) {
          x[n1].x += v[u][n1].x;
          x[n1].y += v[u][n1].y;
        }
    }
    for (; e < d.sub; ++e) {
      const float2* src = cube + (long long)(c * d.sub + e) * d.sc + r;
#pragma unroll
      for (int n1 = 0; n1 < P1; ++n1) {
        const float2 v = load_stream(src + (long long)(P2 * n1 + n2) * d.sp);
        x[n1].x += v.x;
        x[n1].y += v.y;
      }
    }
  }
  __syncthreads();

  for (int t = 0; t < d.T; ++t) {
    float2 v[P1];
#pragma unroll
    for (int n1 = 0; n1 < P1; ++n1) {
      const int q = P2 * n1 + n2 - t;
      const float h = (q >= 0 && q < P) ? hwin[q] : 0.f;
      v[n1] = make_float2(x[n1].x * h, x[n1].y * h);
    }
    dft_any<P1>(v);
    if (n2 < P2) {
#pragma unroll
      for (int k1 = 0; k1 < P1; ++k1) {
        const float2 y = (k1 == 0) ? v[k1] : cmul(v[k1], tw[k1 * n2]);
        ybuf[(k1 * P2 + n2) * RT + col] = y;
      }
    }
    __syncthreads();
    const int dof = t * d.C + c;
    for (int task = tid; task < P1 * RT; task += NT) {
      const int c3 = task % RT, k1 = task / RT;
      float2 z[P2];
#pragma unroll
      for (int m2 = 0; m2 < P2; ++m2) z[m2] = ybuf[(k1 * P2 + m2) * RT + c3];
      dft_any<P2>(z);
      const int r3 = r0 + c3;
      if (d.tap_rel && t > 0) {
        // tap t referenced to its own first pulse: times exp(+2 pi i k t / P)
#pragma unroll
        for (int k2 = 0; k2 < P2; ++k2) z[k2] = cmulc(z[k2], tw[((k1 + P1 * k2) * t) % P]);
      }
      if (r3 < d.R) {
        float2* dst = snap + (long long)dof * d.R + r3;
#pragma unroll
        for (int k2 = 0; k2 < P2; ++k2) store_stream(dst + (long long)(k1 + P1 * k2) * d.D * d.R, z[k2]);
      }
    }
    __syncthreads();
  }
}

// More workgroups per compute unit for more loads in flight, where the
// registers allow it without spills: three at 256 pulses (168 VGPRs), three
// 320-thread groups at 100 pulses (128 VGPRs).
template <int P>
__global__ __launch_bounds__(FftShape<P>::NT) __attribute__((amdgpu_waves_per_eu(P == 256 ? 3 : P == 100 ? 4 : 1)))
void doppler_kernel(const float2* __restrict__ cube,
                                                      float2* __restrict__ snap, Dims d) {
  doppler_tile<P>(cube, snap, d, blockIdx.y, blockIdx.x * FftShape<P>::RT);
}

// Batched: the workgroups of several cubes with the same P in one grid.
template <int P>
__global__ __launch_bounds__(FftShape<P>::NT) __attribute__((amdgpu_waves_per_eu(P == 256 ? 3 : P == 100 ? 4 : 1)))
void doppler_batched_kernel(const ProbDesc* __restrict__ desc, BatchIndex bi) {
  constexpr int RT = FftShape<P>::RT;
  const int g = blockIdx.x;
  int j = 0;
  while (j + 1 < bi.n && bi.tile_begin[j + 1] <= g) ++j;
  const ProbDesc& pd = desc[bi.prob[j]];
  const Dims d = pd.d;
  const int local = g - bi.tile_begin[j];
  const int ntr = (d.R + RT - 1) / RT;
  doppler_tile<P>(pd.cube, pd.snap, d, local / ntr, (local % ntr) * RT);
}

int doppler_tiles(const Dims& d) {
  int rt = 0;
  switch (d.P) {
    case 32: rt = FftShape<32>::RT; break;
    case 64: rt = FftShape<64>::RT; break;
    case 100: rt = FftShape<100>::RT; break;
    case 128: rt = FftShape<128>::RT; break;
    case 256: rt = FftShape<256>::RT; break;
    case 512: rt = FftShape<512>::RT; break;
    default: return 0;
  }
  return ((d.R + rt - 1) / rt) * d.C;
}

hipError_t launch_doppler_batched(int P, const ProbDesc* desc, const BatchIndex& bi, int tiles, hipStream_t st) {
  if (tiles <= 0) return hipSuccess;
  switch (P) {
    case 32: hipLaunchKernelGGL(doppler_batched_kernel<32>, dim3(tiles), dim3(FftShape<32>::NT), 0, st, desc, bi); break;
    case 64: hipLaunchKernelGGL(doppler_batched_kernel<64>, dim3(tiles), dim3(FftShape<64>::NT), 0, st, desc, bi); break;
    case 100: hipLaunchKernelGGL(doppler_batched_kernel<100>, dim3(tiles), dim3(FftShape<100>::NT), 0, st, desc, bi); break;
    case 128: hipLaunchKernelGGL(doppler_batched_kernel<128>, dim3(tiles), dim3(FftShape<128>::NT), 0, st, desc, bi); break;
    case 256: hipLaunchKernelGGL(doppler_batched_kernel<256>, dim3(tiles), dim3(FftShape<256>::NT), 0, st, desc, bi); break;
    case 512: hipLaunchKernelGGL(doppler_batched_kernel<512>, dim3(tiles), dim3(FftShape<512>::NT), 0, st, desc, bi); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_doppler(const Dims& d, const float2* cube, float2* snap, hipStream_t st) {
  auto go = [&](auto kern, int rt, int nt) {
    dim3 grid((d.R + rt - 1) / rt, d.C);
    hipLaunchKernelGGL(kern, grid, dim3(nt), 0, st, cube, snap, d);
    return hipGetLastError();
  };
  switch (d.P) {
    case 32: return go(doppler_kernel<32>, FftShape<32>::RT, FftShape<32>::NT);
    case 64: return go(doppler_kernel<64>, FftShape<64>::RT, FftShape<64>::NT);
    case 100: return go(doppler_kernel<100>, FftShape<100>::RT, FftShape<100>::NT);
    case 128: return go(doppler_kernel<128>, FftShape<128>::RT, FftShape<128>::NT);
    case 256: return go(doppler_kernel<256>, FftShape<256>::RT, FftShape<256>::NT);
    case 512: return go(doppler_kernel<512>, FftShape<512>::RT, FftShape<512>::NT);
  }
  return hipErrorInvalidValue;
}

}  // namespace stap
