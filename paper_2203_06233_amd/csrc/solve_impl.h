// Register-resident Cholesky solve of one system, shared by the stage solve
// kernel and the fused covariance->solve kernel.
//
// A workgroup of TY x 16 threads (ty, tx), TY = 16 or 32, holds
// M = [R_L ; V^H] ((D+S) x D) in registers block-cyclically: thread (ty, tx)
// owns M[ty + TY*a][tx + 16*b].  R_L keeps only the slots that touch its
// lower triangle (16 b <= TY a + TY - 1); the steering part keeps all.
//   factorisation  right-looking over columns j; the owners of column j+1
//                  publish it through a double-buffered LDS vector after
//                  their own update, one barrier per column.  The steering
//                  rows ride along and end as conj(L^-1 V) (forward solve).
//   back solve     backward column sweep, row j of L and c_s = conj(u_s[j])
//                  published per column, one barrier per column.
//   refinement     r = v - R_L u in FP64 (FP32 operands, exact products),
//                  then forward and back sweeps with the FP32 factor.
// The loops over 16-column blocks are unrolled, so every register slot index
// is a compile-time constant; only the 16 columns inside a block run in a
// runtime loop.  Steering rows are stored conjugated (vm = conj(work)).
#pragma once

#include "common.h"

namespace stap {

template <int TY_, int NA_, int NB_, int NVS_>
struct SolveCfg {
  static constexpr int TY = TY_;    // rows per register slot
  static constexpr int NA = NA_;    // row slots of R_L (TY * NA >= D)
  static constexpr int NB = NB_;    // column slots (16 * NB >= D)
  static constexpr int NVS = NVS_;  // row slots of the steering part (TY * NVS >= S)
  static constexpr int NT = 16 * TY;
  static constexpr int DPR = TY * NA;
  static constexpr int DPC = 16 * NB;
  static constexpr int DPX = DPR > DPC ? DPR : DPC;
  static constexpr int SPR = TY * NVS;
  static constexpr bool kPackedInLds = DPC <= 128;
  static constexpr int kPacked = DPC * (DPC + 1) / 2;
  __host__ __device__ static constexpr bool slot(int a, int b) { return 16 * b <= TY * a + TY - 1; }
  static constexpr int kSlab = 16 * DPC;  // refinement residual exchange (complex values)
  static size_t refine_lds_bytes() { return ((kPackedInLds ? (size_t)kPacked : 0) + kSlab) * sizeof(float2); }
};

template <class K>
struct SolveShared {
  float2 colL[2][K::DPX];  // column j below the pivot (zero at and above it)
  float2 colV[2][K::SPR];  // column j of the steering rows
  double colP[2];          // the pivot of column j in FP64
  float invd[K::DPX];
  float gam[K::SPR];
  double d64[K::DPX];      // row sums of |L[i][k]|^2 over the finished columns, FP64
  float rdiag[K::DPX];     // loaded diagonal R_L[i][i]
};

__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }

// x -= a * conj(b), four FMAs
__device__ __forceinline__ void sub_mulc(float2& x, float2 a, float2 b) {
  x.x = fmaf(-a.x, b.x, x.x);
  x.x = fmaf(-a.y, b.y, x.x);
  x.y = fmaf(-a.y, b.x, x.y);
  x.y = fmaf(a.x, b.y, x.y);
}
// x -= a * b, four FMAs
__device__ __forceinline__ void sub_mul(float2& x, float2 a, float2 b) {
  x.x = fmaf(-a.x, b.x, x.x);
  x.x = fmaf(a.y, b.y, x.x);
  x.y = fmaf(-a.x, b.y, x.y);
  x.y = fmaf(-a.y, b.x, x.y);
}

// Backward column sweep L^H u = a in conjugated storage:
//   c_s = x_s[j] / L[j][j]  (= conj(u_s[j])),   x_s[k] -= L[j][k] c_s  (k < j).
template <class K>
__device__ __forceinline__ void sweep_back(float2 (&x)[K::NVS][K::NB], const float2 (&lm)[K::NA][K::NB],
                                           int D, SolveShared<K>& sh) {
  constexpr int TY = K::TY, NB = K::NB, NVS = K::NVS;
  const int tx = lane_tid() & 15, ty = lane_tid() >> 4;
  __syncthreads();
#pragma unroll
  for (int jb = NB - 1; jb >= 0; --jb) {
    const int aj = (16 * jb) / TY;
    const int jend = min(16, D - 16 * jb);
    for (int jt = jend - 1; jt >= 0; --jt) {
      const int j = 16 * jb + jt;
      const int buf = jt & 1;
      if (ty == j - TY * aj) {
#pragma unroll
        for (int b = 0; b <= jb; ++b) {
          const int k = tx + 16 * b;
          sh.colL[buf][k] = (k < j) ? lm[aj][b] : make_float2(0.f, 0.f);
        }
      }
      if (tx == jt) {
        const float iv = sh.invd[j];
#pragma unroll
        for (int a = 0; a < NVS; ++a) {
          const float2 c = make_float2(x[a][jb].x * iv, x[a][jb].y * iv);
          x[a][jb] = c;
          sh.colV[buf][ty + TY * a] = c;
        }
      }
      __syncthreads();
#pragma unroll
      for (int b = 0; b <= jb; ++b) {
        const float2 l = sh.colL[buf][tx + 16 * b];
#pragma unroll
        for (int a = 0; a < NVS; ++a) sub_mul(x[a][b], l, sh.colV[buf][ty + TY * a]);
      }
    }
  }
  __syncthreads();
}

// Forward column sweep L z = r in conjugated storage:
//   c_s = x_s[j] / L[j][j],   x_s[k] -= conj(L[k][j]) c_s  (k > j).
template <class K>
__device__ __forceinline__ void sweep_fwd(float2 (&x)[K::NVS][K::NB], const float2 (&lm)[K::NA][K::NB],
                                          int D, SolveShared<K>& sh) {
  constexpr int TY = K::TY, NA = K::NA, NB = K::NB, NVS = K::NVS;
  const int tx = lane_tid() & 15, ty = lane_tid() >> 4;
  __syncthreads();
#pragma unroll
  for (int jb = 0; jb < NB; ++jb) {
    const int a0 = (16 * jb) / TY;
    const int jend = min(16, D - 16 * jb);
    for (int jt = 0; jt < jend; ++jt) {
      const int j = 16 * jb + jt;
      const int buf = jt & 1;
      if (tx == jt) {
        const float iv = sh.invd[j];
#pragma unroll
        for (int a = a0; a < NA; ++a) {
          const int i = ty + TY * a;
          sh.colL[buf][i] = (i > j) ? lm[a][jb] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int a = 0; a < NVS; ++a) {
          const float2 c = make_float2(x[a][jb].x * iv, x[a][jb].y * iv);
          x[a][jb] = c;
          sh.colV[buf][ty + TY * a] = c;
        }
      }
      __syncthreads();
#pragma unroll
      for (int b = jb; b < NB; ++b) {
        const float2 l = sh.colL[buf][tx + 16 * b];
#pragma unroll
        for (int a = 0; a < NVS; ++a) sub_mulc(x[a][b], sh.colV[buf][ty + TY * a], l);
      }
    }
  }
  __syncthreads();
}

// Refinement residual on the FP64 matrix cores: conj(r_s) = conj(v_s - R_L u_s)
// into rv, for u_s held as vm = conj(u_s).  The steering vectors are taken
// 16 at a time (a slab): the threads holding them publish u for the slab to
// LDS as U[k][s], then each wave forms 16 x 16 output blocks (rows I) as
// sum over K of R_L[I][K] U[K] with v_mfma_f64_16x16x4 (four real products
// per complex one: three real products in the Gauss form; FP32 operands
// converted exactly, FP64 accumulation), takes
// r = v - R_L u in FP64, rounds it to FP32 and hands it back through the same
// slab.  FP64 MFMA lane layout (lane l, m = l % 16, q = l / 16): A operand
// A[m][q], B operand B[q][m], result register i holds D[q + 4i][m] (rows
// interleaved, unlike the FP32 16 x 16 x 4 form).
template <class K, bool RP_LDS, class RSrc>
__device__ __forceinline__ void residual_mfma(const RSrc& src, const float2* Rp, float2* slab,
                                              const float2 (&vm)[K::NVS][K::NB], float2 (&rv)[K::NVS][K::NB],
                                              const float2* __restrict__ steer, int D, int S) {
  constexpr int TY = K::TY, NB = K::NB, NVS = K::NVS, NW = K::NT / 64;
  constexpr int NI = (NB + NW - 1) / NW;  // output row blocks per wave
  const int tid = lane_tid(), tx = tid & 15, ty = tid >> 4;
  const int lane = tid & 63, wave = tid >> 6, m16 = lane & 15, q = lane >> 4;
  const int nslab = (S + 15) >> 4;
#pragma unroll
  for (int a = 0; a < NVS; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) rv[a][b] = make_float2(0.f, 0.f);
  // R_L[m][k] from the stored lower triangle, zero outside D x D
  auto relem = [&](int m, int k) -> float2 {
    const int mc = min(m, D - 1), kc = min(k, D - 1);
    const bool lower = kc <= mc;
    const int hi = lower ? mc : kc, lo = lower ? kc : mc;
    float2 v = RP_LDS ? Rp[hi * (hi + 1) / 2 + lo] : src.lower(hi, lo);
    v.y = lower ? v.y : -v.y;
    return (m < D && k < D) ? v : make_float2(0.f, 0.f);
  };
  for (int N = 0; N < nslab; ++N) {
#pragma unroll
    for (int a = 0; a < NVS; ++a) {
      const int s = ty + TY * a;
      if ((s >> 4) == N) {
#pragma unroll
        for (int b = 0; b < NB; ++b) slab[(tx + 16 * b) * 16 + (s & 15)] = conjf2(vm[a][b]);
      }
    }
    __syncthreads();
    float2 res[NI][4];
#pragma unroll
    for (int ii = 0; ii < NI; ++ii) {
      const int I = wave + NW * ii;
      if (I < NB) {
        // three real products per complex one (a1 = ar ur, a2 = ai ui,
        // a3 = (ar + ai)(ur + ui); Re = a1 - a2, Im = a3 - a1 - a2)
        doublex4 a1 = {0.0, 0.0, 0.0, 0.0}, a2 = a1, a3 = a1;
        const int m = 16 * I + m16;
#pragma unroll 1
        for (int kb = 0; kb < NB; ++kb) {
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const int k = 16 * kb + 4 * s4 + q;
            const float2 r = relem(m, k);
            const float2 u = slab[k * 16 + m16];
            const double ar = r.x, ai = r.y, ur = u.x, ui = u.y;
            a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, ur, a1, 0, 0, 0);
            a2 = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, ui, a2, 0, 0, 0);
            a3 = __builtin_amdgcn_mfma_f64_16x16x4f64(ar + ai, ur + ui, a3, 0, 0, 0);
          }
        }
        const doublex4 cr = a1 - a2, ci = a3 - a1 - a2;
        const int s = 16 * N + m16;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int k = 16 * I + q + 4 * i;
          float2 v = make_float2(0.f, 0.f);
          if (s < S && k < D) v = steer[s * D + k];
          res[ii][i] = make_float2((float)((double)v.x - cr[i]), (float)((double)v.y - ci[i]));
        }
      }
    }
    __syncthreads();  // every wave has read U
#pragma unroll
    for (int ii = 0; ii < NI; ++ii) {
      const int I = wave + NW * ii;
      if (I < NB) {
#pragma unroll
        for (int i = 0; i < 4; ++i) slab[(16 * I + q + 4 * i) * 16 + m16] = res[ii][i];
      }
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < NVS; ++a) {
      const int s = ty + TY * a;
      if ((s >> 4) == N) {
#pragma unroll
        for (int b = 0; b < NB; ++b) rv[a][b] = conjf2(slab[(tx + 16 * b) * 16 + (s & 15)]);
      }
    }
    __syncthreads();  // the slab is rewritten for the next 16 steering vectors
  }
}

// Solve one system.  src.lower(i, k) (k <= i) yields the loaded covariance;
// with RP_LDS the refinement residual reads the same lower triangle packed
// row-major from LDS at Rp (row i at i(i+1)/2), else through src.  slab is
// LDS for 16 * DPC complex values (refinement only).  W is this system's
// [S][D] output, info its status word (may be null).
template <class K, bool REFINE, bool RP_LDS, class RSrc>
__device__ __forceinline__ void solve_system(const RSrc& src, const float2* Rp, float2* slab,
                                             const float2* __restrict__ steer, float2* __restrict__ W,
                                             int* __restrict__ info, const Dims& d, SolveShared<K>& sh) {
  constexpr int TY = K::TY, NA = K::NA, NB = K::NB, NVS = K::NVS, NT = K::NT, DPC = K::DPC;
  const int tid = lane_tid(), tx = tid & 15, ty = tid >> 4;
  const int D = d.D, S = d.S;

  float2 lm[NA][NB];
  float2 vm[NVS][NB];
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
      if (K::slot(a, b)) {
        const int i = ty + TY * a, k = tx + 16 * b;
        lm[a][b] = (i < D && k <= i) ? src.lower(i, k) : make_float2(0.f, 0.f);
      }
#pragma unroll
  for (int a = 0; a < NVS; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int s = ty + TY * a, k = tx + 16 * b;
      vm[a][b] = (s < S && k < D) ? conjf2(steer[s * D + k]) : make_float2(0.f, 0.f);
    }

  // The pivots are taken in FP64: d64[i] sums |L[i][k]|^2 (the FP32 factor
  // entries, squared and added in FP64) over the finished columns k, and the
  // pivot of column j is rdiag[j] - d64[j] in FP64, tested > 0 in FP64 and
  // used rounded to FP32.  Row i's sum is updated by the one thread that
  // finalises L[i][j] and read by the one that publishes column j + 1, in the
  // same wave and in that order.
  for (int i = tid; i < K::DPX; i += NT) {
    sh.d64[i] = 0.0;
    sh.rdiag[i] = i < D ? src.lower(i, i).x : 1.f;
  }
  __syncthreads();

  // Column j is published already masked: colL holds rows i > j (zero at
  // and above the pivot), colP the pivot.  Every thread then forms
  // li = c_i / piv for its rows and lk = c_k for its columns with no
  // per-element test; finished rows and columns contribute zeros.
  int fail = 0;
#pragma unroll
  for (int jb = 0; jb < NB; ++jb) {
    const int a0 = (16 * jb) / TY;
    const int j0 = 16 * jb;
    if (tx == 0) {
#pragma unroll
      for (int a = a0; a < NA; ++a) {
        const int i = ty + TY * a;
        sh.colL[0][i] = (i > j0) ? lm[a][jb] : make_float2(0.f, 0.f);
        if (i == j0) sh.colP[0] = (double)sh.rdiag[j0] - sh.d64[j0];
      }
#pragma unroll
      for (int a = 0; a < NVS; ++a) sh.colV[0][ty + TY * a] = vm[a][jb];
    }
    __syncthreads();
    const int jend = min(16, D - 16 * jb);
    for (int jt = 0; jt < jend; ++jt) {
      const int j = j0 + jt;
      const int buf = jt & 1;
      const double piv64 = sh.colP[buf];
      if (!(piv64 > 0.0)) {
        fail = j + 1;
        break;
      }
      const float piv = (float)piv64;
      const float dj = sqrtf(piv), rs = 1.f / dj, ip = rs * rs;
      float2 li[NA], lk[NB], lv[NVS];
#pragma unroll
      for (int a = a0; a < NA; ++a) {
        const float2 c = sh.colL[buf][ty + TY * a];
        li[a] = make_float2(c.x * ip, c.y * ip);
      }
#pragma unroll
      for (int b = jb; b < NB; ++b) lk[b] = sh.colL[buf][tx + 16 * b];
#pragma unroll
      for (int a = 0; a < NVS; ++a) {
        const float2 c = sh.colV[buf][ty + TY * a];
        lv[a] = make_float2(c.x * ip, c.y * ip);
      }
      if (tid == 0) sh.invd[j] = rs;
      if (tx == jt) {  // finalise column j from the owners' own raw values
#pragma unroll
        for (int a = a0; a < NA; ++a) {
          const int i = ty + TY * a;
          const float2 c = lm[a][jb];
          if (i > j) {
            const float2 l = make_float2(c.x * rs, c.y * rs);
            lm[a][jb] = l;
            sh.d64[i] += (double)l.x * (double)l.x + (double)l.y * (double)l.y;
          } else if (i == j) {
            lm[a][jb] = make_float2(dj, 0.f);
          }
        }
#pragma unroll
        for (int a = 0; a < NVS; ++a) vm[a][jb] = make_float2(vm[a][jb].x * rs, vm[a][jb].y * rs);
      }
#pragma unroll
      for (int a = a0; a < NA; ++a)
#pragma unroll
        for (int b = jb; b < NB; ++b)
          if (K::slot(a, b)) sub_mulc(lm[a][b], li[a], lk[b]);
#pragma unroll
      for (int a = 0; a < NVS; ++a)
#pragma unroll
        for (int b = jb; b < NB; ++b) sub_mulc(vm[a][b], lv[a], lk[b]);
      if (jt + 1 < jend && tx == jt + 1) {  // publish column j+1, masked
#pragma unroll
        for (int a = a0; a < NA; ++a) {
          const int i = ty + TY * a;
          sh.colL[buf ^ 1][i] = (i > j + 1) ? lm[a][jb] : make_float2(0.f, 0.f);
          if (i == j + 1) sh.colP[buf ^ 1] = (double)sh.rdiag[j + 1] - sh.d64[j + 1];
        }
#pragma unroll
        for (int a = 0; a < NVS; ++a) sh.colV[buf ^ 1][ty + TY * a] = vm[a][jb];
      }
      __syncthreads();
    }
    if (fail) break;
  }

  if (fail) {
    for (int e = tid; e < S * D; e += NT) W[e] = make_float2(0.f, 0.f);
    if (tid == 0 && info) *info = fail;
    return;
  }

  // gamma_s = ||a_s||^2 from the forward-solved steering rows
#pragma unroll
  for (int a = 0; a < NVS; ++a) {
    float g = 0.f;
#pragma unroll
    for (int b = 0; b < NB; ++b) g += vm[a][b].x * vm[a][b].x + vm[a][b].y * vm[a][b].y;
    g += __shfl_xor(g, 8, 16);
    g += __shfl_xor(g, 4, 16);
    g += __shfl_xor(g, 2, 16);
    g += __shfl_xor(g, 1, 16);
    if (tx == 0) sh.gam[ty + TY * a] = g;
  }

  sweep_back<K>(vm, lm, D, sh);

  if (REFINE) {
    for (int it = 0; it < d.refine; ++it) {
      float2 rv[NVS][NB];
      residual_mfma<K, RP_LDS>(src, Rp, slab, vm, rv, steer, D, S);
      sweep_fwd<K>(rv, lm, D, sh);
      sweep_back<K>(rv, lm, D, sh);
#pragma unroll
      for (int a = 0; a < NVS; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) vm[a][b] = cadd(vm[a][b], rv[a][b]);
    }
    // gamma_s = Re(v_s^H u_s) in FP64 for the refined u
#pragma unroll
    for (int a = 0; a < NVS; ++a) {
      double g = 0.0;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int s = ty + TY * a, k = tx + 16 * b;
        if (s < S && k < D) {
          const float2 v = steer[s * D + k];
          g += (double)v.x * vm[a][b].x - (double)v.y * vm[a][b].y;  // Re(conj(v) u), u = conj(vm)
        }
      }
      g += __shfl_xor(g, 8, 16);
      g += __shfl_xor(g, 4, 16);
      g += __shfl_xor(g, 2, 16);
      g += __shfl_xor(g, 1, 16);
      if (tx == 0) sh.gam[ty + TY * a] = (float)g;
    }
    __syncthreads();
  }

  // w_s = u_s / sqrt(gamma_s)
#pragma unroll
  for (int a = 0; a < NVS; ++a) {
    const int s = ty + TY * a;
    if (s < S) {
      const float sc = 1.f / sqrtf(sh.gam[s]);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int k = tx + 16 * b;
        if (k < D) W[s * D + k] = make_float2(vm[a][b].x * sc, -vm[a][b].y * sc);
      }
    }
  }
  if (tid == 0 && info) *info = 0;
}

}  // namespace stap
