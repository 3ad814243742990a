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
  static size_t refine_lds_bytes() { return (kPackedInLds ? (size_t)kPacked : 0) * sizeof(float2); }
};

template <class K>
struct SolveShared {
  float2 colL[2][K::DPX];  // column j below the pivot (zero at and above it)
  float2 colV[2][K::SPR];  // column j of the steering rows
  float colP[2];           // the pivot M[j][j]
  float invd[K::DPX];
  float gam[K::SPR];
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
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
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
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
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

// Solve one system.  src.lower(i, k) (k <= i) yields the loaded covariance;
// with RP_LDS the refinement residual reads the same lower triangle packed
// row-major from LDS at Rp (row i at i(i+1)/2), else through src.  W is this
// system's [S][D] output, info its status word (may be null).
template <class K, bool REFINE, bool RP_LDS, class RSrc>
__device__ __forceinline__ void solve_system(const RSrc& src, const float2* Rp,
                                             const float2* __restrict__ steer, float2* __restrict__ W,
                                             int* __restrict__ info, const Dims& d, SolveShared<K>& sh) {
  constexpr int TY = K::TY, NA = K::NA, NB = K::NB, NVS = K::NVS, NT = K::NT, DPC = K::DPC;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
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
        if (i == j0) sh.colP[0] = lm[a][jb].x;
      }
#pragma unroll
      for (int a = 0; a < NVS; ++a) sh.colV[0][ty + TY * a] = vm[a][jb];
    }
    __syncthreads();
    const int jend = min(16, D - 16 * jb);
    for (int jt = 0; jt < jend; ++jt) {
      const int j = j0 + jt;
      const int buf = jt & 1;
      const float piv = sh.colP[buf];
      if (!(piv > 0.f)) {
        fail = j + 1;
        break;
      }
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
          if (i > j) lm[a][jb] = make_float2(c.x * rs, c.y * rs);
          else if (i == j) lm[a][jb] = make_float2(dj, 0.f);
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
          if (i == j + 1) sh.colP[buf ^ 1] = lm[a][jb].x;
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
      // conj(r_s[k]) = conj(v_s[k]) - sum_q conj(R[k][q]) conj(u_s[q]) in FP64.
      // conj(u_s[q]) for q = tx' + 16 b sits in register vm[a][b] of lane
      // tx' of the same 16-lane group (same ty), so it is broadcast with a
      // shuffle.  conj(R[k][q]) is the stored lower element (k, q) conjugated
      // when q <= k, else the stored (q, k): a select, not a branch.
      float2 rv[NVS][NB];
      int kb[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int k = min(tx + 16 * b, D - 1);
        kb[b] = k * (k + 1) / 2;
      }
      auto fetch = [&](int q, int b) -> float2 {
        const int k = tx + 16 * b;
        const int kc = min(k, D - 1);
        const bool lower = q <= kc;
        float2 v;
        if (RP_LDS) {
          v = Rp[lower ? kb[b] + q : q * (q + 1) / 2 + kc];
        } else {
          v = src.lower(lower ? kc : q, lower ? q : kc);
        }
        v.y = lower ? -v.y : v.y;
        return (k < D) ? v : make_float2(0.f, 0.f);
      };
#pragma unroll
      for (int a = 0; a < NVS; ++a) {
        double accr[NB], acci[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          accr[b] = 0.0;
          acci[b] = 0.0;
        }
#pragma unroll
        for (int bq = 0; bq < NB; ++bq) {
          const int qn = min(16, D - 16 * bq);
          for (int t = 0; t < qn; ++t) {
            const int q = 16 * bq + t;
            const float ur_f = __shfl(vm[a][bq].x, t, 16);
            const float ui_f = __shfl(vm[a][bq].y, t, 16);
            const double ur = ur_f, ui = ui_f;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
              const float2 v = fetch(q, b);
              const double rr = v.x, ri = v.y;
              accr[b] = fma(rr, ur, fma(-ri, ui, accr[b]));
              acci[b] = fma(rr, ui, fma(ri, ur, acci[b]));
            }
          }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int s = ty + TY * a, k = tx + 16 * b;
          if (s < S && k < D) {
            const float2 v = steer[s * D + k];
            rv[a][b] = make_float2((float)((double)v.x - accr[b]), (float)(-(double)v.y - acci[b]));
          } else {
            rv[a][b] = make_float2(0.f, 0.f);
          }
        }
      }
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
