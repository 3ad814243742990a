// Blocked Cholesky solve of one system inside one wave, every block held in
// that wave's registers for the whole solve (up to NB = 6 block columns of
// R_L and NS = 2 blocks of steering vectors: D <= 96, S <= 32).
//
// The steps and the block algebra are those of bsolve_system()
// (bsolve_impl.h): right-looking factorisation with the in-wave diagonal
// factor-and-invert, the forward solve of the steering rows M = V^H riding
// along as extra rows, the back solve in row form Z L = Y^H, and the FP64
// refinement residual conj(r) = conj(v) - Z R_L.  What differs is the
// placement: with the block coordinates known at compile time every loop is
// unrolled, the operands of a block product are read straight from the
// registers of the blocks they come from (no exchange through LDS and no
// barrier), and the only LDS traffic is the transposition of the L blocks a
// back-solve step multiplies by (and the reordering of a residual block).
// One wave per system leaves the four SIMDs of a compute unit on four
// systems at once; the instruction stream of the wave interleaves the
// serial diagonal work with the matrix-core products of the same step.
#pragma once

#include "bsolve_impl.h"

namespace stap {
namespace wsv {

constexpr int tri(int I, int J) { return I * (I + 1) / 2 + J; }

// x -/+= P Q^H, operands straight from accumulator registers (the lane's
// P.re[s], P.im[s] are its X[m][4q + s]).
template <bool SUB>
__device__ __forceinline__ void pqh(Acc& x, const Acc& P, const Acc& Q) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const float qr = SUB ? -Q.re[s] : Q.re[s], qi = SUB ? -Q.im[s] : Q.im[s];
    x.re = mfma4(qr, P.re[s], x.re);  // Re(conj(q) p) = qr pr + qi pi
    x.re = mfma4(qi, P.im[s], x.re);
    x.im = mfma4(qr, P.im[s], x.im);  // Im(conj(q) p) = qr pi - qi pr
    x.im = mfma4(-qi, P.re[s], x.im);
  }
}

// x -/+= P Q with Qt the fragment of Q^T.
template <bool SUB>
__device__ __forceinline__ void pq(Acc& x, const Acc& P, const Frag& Qt) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const float qr = SUB ? -Qt.v[s].x : Qt.v[s].x, qi = SUB ? -Qt.v[s].y : Qt.v[s].y;
    x.re = mfma4(qr, P.re[s], x.re);  // Re(q p) = qr pr - qi pi
    x.re = mfma4(-qi, P.im[s], x.re);
    x.im = mfma4(qr, P.im[s], x.im);  // Im(q p) = qr pi + qi pr
    x.im = mfma4(qi, P.re[s], x.im);
  }
}

// Back solve in row form, Z L = Y^H (M holds Y^H on entry, Z on exit): for J
// descending, Z_J = M_J Linv_JJ, then M_I -= Z_J L_JI for I < J.  The
// transposes of row J of L pass through LDS (tb, SLOTS blocks), SLOTS at a
// time, the diagonal block first.
template <int NB, int NS, int SLOTS>
__device__ __forceinline__ void back_solve(const Acc (&L)[NB * (NB + 1) / 2], Acc (&M)[NS * NB], float2* tb) {
#pragma unroll
  for (int J = NB - 1; J >= 0; --J) {
#pragma unroll
    for (int I0 = J; I0 >= 0; I0 -= SLOTS) {
      __syncthreads();  // earlier reads of tb are done
#pragma unroll
      for (int g = 0; g < SLOTS && I0 - g >= 0; ++g) frag_store_t(tb + g * 256, to_frag(L[tri(J, I0 - g)]));
      __syncthreads();
#pragma unroll
      for (int g = 0; g < SLOTS && I0 - g >= 0; ++g) {
        const int I = I0 - g;
        const Frag Lt = frag_load(tb + g * 256);
        if (I == J) {
#pragma unroll
          for (int N = 0; N < NS; ++N) {
            Acc x = acc_zero();
            pq<false>(x, M[N * NB + J], Lt);
            M[N * NB + J] = x;
          }
        } else {
#pragma unroll
          for (int N = 0; N < NS; ++N) pq<true>(M[N * NB + I], M[N * NB + J], Lt);
        }
      }
    }
  }
}

// Forward solve Y^H L^H = M with the factor in L (Linv_JJ on the diagonal):
// M_J := M_J Linv_JJ^H, then M_K -= M_J L_KJ^H for K > J.
template <int NB, int NS>
__device__ __forceinline__ void forward_solve(const Acc (&L)[NB * (NB + 1) / 2], Acc (&M)[NS * NB]) {
#pragma unroll
  for (int J = 0; J < NB; ++J) {
#pragma unroll
    for (int N = 0; N < NS; ++N) {
      Acc x = acc_zero();
      pqh<false>(x, M[N * NB + J], L[tri(J, J)]);
      M[N * NB + J] = x;
    }
#pragma unroll
    for (int K = J + 1; K < NB; ++K)
#pragma unroll
      for (int N = 0; N < NS; ++N) pqh<true>(M[N * NB + K], M[N * NB + J], L[tri(K, J)]);
  }
}

// The trailing updates of factorisation step J other than the one of
// diagonal block J+1, numbered 0..COUNT-1: first the L blocks (I, K),
// K = J+1.., I = K.., then the M blocks (N, K).
template <int NB, int NS, int J>
struct StepWork {
  static constexpr int NLU = (NB - J - 1) * (NB - J) / 2 - (J + 1 < NB ? 1 : 0);
  static constexpr int COUNT = NLU + (NB - J - 1) * NS;
  struct Item {
    bool isL;
    int I, K, N;
  };
  static constexpr Item item(int p) {
    int n = 0;
    for (int K = J + 1; K < NB; ++K)
      for (int I = K; I < NB; ++I) {
        if (K == J + 1 && I == J + 1) continue;
        if (n == p) return Item{true, I, K, 0};
        ++n;
      }
    for (int K = J + 1; K < NB; ++K)
      for (int N = 0; N < NS; ++N) {
        if (n == p) return Item{false, 0, K, N};
        ++n;
      }
    return Item{false, -1, -1, -1};
  }
};

template <int NB, int NS, int J, int P, int END>
__device__ __forceinline__ void step_work(Acc (&L)[NB * (NB + 1) / 2], Acc (&M)[NS * NB]) {
  if constexpr (P < END) {
    constexpr auto it = StepWork<NB, NS, J>::item(P);
    if constexpr (it.isL) pqh<true>(L[tri(it.I, it.K)], L[tri(it.I, J)], L[tri(it.K, J)]);
    else pqh<true>(M[it.N * NB + it.K], M[it.N * NB + J], L[tri(it.K, J)]);
    step_work<NB, NS, J, P + 1, END>(L, M);
  }
}

// Columns j.. of diag_factor_inv() with the share of step J's trailing
// updates that goes with each column issued right after it, so the wave's
// instruction stream interleaves the serial VALU work of diagonal block
// J+1 with independent matrix-core products.
template <int NB, int NS, int J, int j>
__device__ __forceinline__ void diag_cols_work(Frag& A, Frag& X, int m, float& rsm, int& fail, double& p64,
                                               Acc (&L)[NB * (NB + 1) / 2], Acc (&M)[NS * NB]) {
  constexpr int C = StepWork<NB, NS, J>::COUNT;
  diag_col<j>(A, X, m, rsm, fail, p64);
  step_work<NB, NS, J, j * C / 16, (j + 1) * C / 16>(L, M);
  if constexpr (j < 15) diag_cols_work<NB, NS, J, j + 1>(A, X, m, rsm, fail, p64, L, M);
}

// Factorisation step J (diagonal block J already holds Linv_JJ): panel,
// the update and factorisation of diagonal block J+1 interleaved with the
// remaining updates of the step, then step J+1.  d64 (LDS) collects the
// FP64 row sums of |L|^2 over the finished block columns and rdiag holds
// the loaded diagonal: the FP64 pivots of block J+1 start from their
// difference.
template <int NB, int NS, int J>
__device__ __forceinline__ void fact_step(Acc (&L)[NB * (NB + 1) / 2], Acc (&M)[NS * NB], int& fail, double* d64,
                                          const float* rdiag) {
  const int lane = lane_tid() & 63;
#pragma unroll
  for (int I = J + 1; I < NB; ++I) {
    Acc x = acc_zero();
    pqh<false>(x, L[tri(I, J)], L[tri(J, J)]);
    L[tri(I, J)] = x;
    const double pn = frag_row_norm2(x);
    if (lane < 16) d64[16 * I + lane] += pn;
  }
#pragma unroll
  for (int N = 0; N < NS; ++N) {
    Acc x = acc_zero();
    pqh<false>(x, M[N * NB + J], L[tri(J, J)]);
    M[N * NB + J] = x;
  }
  if constexpr (J + 1 < NB) {
    pqh<true>(L[tri(J + 1, J + 1)], L[tri(J + 1, J)], L[tri(J + 1, J)]);
    const int l = lane_tid() & 63, m = l & 15, q = l >> 4;
    Frag A = to_frag(L[tri(J + 1, J + 1)]), X;
#pragma unroll
    for (int i = 0; i < 4; ++i) X.v[i] = make_float2(m == 4 * q + i ? 1.f : 0.f, 0.f);
    int f = 0;
    float rsm = 1.f;
    double p64 = (double)rdiag[16 * (J + 1) + m] - d64[16 * (J + 1) + m];
    diag_cols_work<NB, NS, J, 0>(A, X, m, rsm, f, p64, L, M);
#pragma unroll
    for (int i = 0; i < 4; ++i) X.v[i] = make_float2(X.v[i].x * rsm, X.v[i].y * rsm);
    fail = (fail == 0 && f != 0) ? 16 * (J + 1) + f : fail;
    L[tri(J + 1, J + 1)] = to_acc(X);
    fact_step<NB, NS, J + 1>(L, M, fail, d64, rdiag);
  }
}

// LDS of one system: transpose slots, then (REFINE) the packed lower
// triangle of R_L, row r at offset r (r + 1) / 2, then the FP64 row sums of
// |L|^2 (16 NB doubles) and the loaded diagonal (16 NB floats) for the
// pivots.
template <int NB, bool REFINE>
struct WsLds {
  static constexpr int SLOTS = REFINE ? 1 : NB;
  static constexpr int PACK = REFINE ? 16 * NB * (16 * NB + 1) / 2 : 0;
  static constexpr int PIV = 16 * NB + 8 * NB;  // in complex (8-byte) units
  static constexpr int COMPLEX = SLOTS * 256 + PACK + PIV;
};

// Solve one system: R is its loaded covariance, full Hermitian [D][D]
// row-major, W its [S][D] weights, info its status word (may be null);
// D <= 16 NB, S <= 16 NS.  lds points at WsLds<NB, REFINE>::COMPLEX complex
// of 16-byte aligned LDS.  Blocks beyond D carry the identity, steering rows
// beyond S are zero.  With REFINE the lower triangle of R is also kept in
// LDS for the FP64 residual, and the current u is parked in W between the
// residual and the correction (each lane reads back only what it wrote).
template <int NB, int NS, bool REFINE>
__device__ __forceinline__ void wsolve_system(const float2* __restrict__ R, const float2* __restrict__ steer,
                                              float2* __restrict__ W, int* __restrict__ info, const Dims& d,
                                              float2* lds) {
  using LY = WsLds<NB, REFINE>;
  constexpr int NL = NB * (NB + 1) / 2;
  const int D = d.D, S = d.S;
  const int lane = lane_tid() & 63, m = lane & 15, q = lane >> 4;
  float2* tb = lds;
  float2* Rp = lds + LY::SLOTS * 256;
  double* d64 = reinterpret_cast<double*>(Rp + LY::PACK);
  float* rdiag = reinterpret_cast<float*>(d64 + 16 * NB);
  for (int r = lane; r < 16 * NB; r += 64) d64[r] = 0.0;

  Acc L[NL], M[NS * NB];
#pragma unroll
  for (int I = 0; I < NB; ++I) {
#pragma unroll
    for (int J = 0; J <= I; ++J) {
      const int r = 16 * I + m;
      Acc a;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = 16 * J + 4 * q + i;
        const float2 v = (r < D && c < D) ? R[(long long)r * D + c] : make_float2(r == c ? 1.f : 0.f, 0.f);
        a.re[i] = v.x;
        a.im[i] = v.y;
        if (REFINE && c <= r && r < D) Rp[r * (r + 1) / 2 + c] = v;
        if (I == J && c == r) rdiag[r] = v.x;
      }
      L[tri(I, J)] = a;
    }
  }
#pragma unroll
  for (int N = 0; N < NS; ++N) {
#pragma unroll
    for (int J = 0; J < NB; ++J) {
      const int s = 16 * N + m;
      Acc a;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = 16 * J + 4 * q + i;
        const float2 v = (s < S && k < D) ? steer[s * D + k] : make_float2(0.f, 0.f);
        a.re[i] = v.x;
        a.im[i] = -v.y;
      }
      M[N * NB + J] = a;
    }
  }

  // ---- factorisation with the forward solve of the steering rows
  int fail = 0;
  {
    Frag A = to_frag(L[0]), X;
    const int f = diag_factor_inv(A, X, (double)frag_diag(A));
    fail = f != 0 ? f : 0;
    L[0] = to_acc(X);
  }
  fact_step<NB, NS, 0>(L, M, fail, d64, rdiag);
  if (fail) {
    for (int e = lane; e < S * D; e += 64) W[e] = make_float2(0.f, 0.f);
    if (lane == 0 && info) *info = fail;
    return;
  }

  // ---- gamma_s = ||y_s||^2 (no refinement), summed over the row's blocks
  double gam[NS];
#pragma unroll
  for (int N = 0; N < NS; ++N) {
    gam[N] = 0.0;
#pragma unroll
    for (int J = 0; J < NB; ++J) {
      const Acc& y = M[N * NB + J];
      float p = 0.f;
#pragma unroll
      for (int i = 0; i < 4; ++i) p = fmaf(y.re[i], y.re[i], fmaf(y.im[i], y.im[i], p));
      p += __shfl_xor(p, 16);
      p += __shfl_xor(p, 32);
      gam[N] += p;
    }
  }

  back_solve<NB, NS, LY::SLOTS>(L, M, tb);

  if (REFINE) {
    for (int it = 0; it < d.refine; ++it) {
      // park u = conj(Z) in W (the lane's own elements)
#pragma unroll
      for (int N = 0; N < NS; ++N) {
        const int s = 16 * N + m;
#pragma unroll
        for (int J = 0; J < NB; ++J)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int k = 16 * J + 4 * q + i;
            if (s < S && k < D) W[s * D + k] = make_float2(M[N * NB + J].re[i], -M[N * NB + J].im[i]);
          }
      }
      // the parked values are read from memory again below: keeping them in
      // registers across the residual and the solves would cost more
      asm volatile("" ::: "memory");
      // residual conj(r) = conj(v) - Z R_L in FP64 (exact products of the
      // FP32 values): block (N, I) sums Z_NJ R_JI over J.  The lane's Z
      // operand is its own element Z_NJ[m][4q + s4], read back from W; R
      // comes from the packed copy.  The FP64 result has column q + 4i of
      // the block in register i; a pass through tb restores fragment order.
#pragma unroll
      for (int N = 0; N < NS; ++N) {
        const int s = 16 * N + m;
#pragma unroll
        for (int I = 0; I < NB; ++I) {
          // three real products per complex one: a1 = sum qr pr,
          // a2 = sum qi pi, a3 = sum (qr + qi)(pr + pi); Re = a1 - a2,
          // Im = a3 - a1 - a2 (the FP64 sums of FP32 values are exact)
          doublex4 a1 = {0.0, 0.0, 0.0, 0.0}, a2 = a1, a3 = a1;
          const int c = 16 * I + m;
          // operands of block row J: R[16J + 4q + s4][c] and the lane's
          // Z_NJ[m][4q + s4]; fetched one step ahead of their MFMAs
          auto fetch = [&](int J, float2 (&rv)[4], float2 (&z)[4]) {
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
              const int r = 16 * J + 4 * q + s4;
              if (r < D && c < D) {
                rv[s4] = r >= c ? Rp[r * (r + 1) / 2 + c] : Rp[c * (c + 1) / 2 + r];
                if (r < c) rv[s4].y = -rv[s4].y;
              } else {
                rv[s4] = make_float2(r == c ? 1.f : 0.f, 0.f);
              }
              const float2 u = (s < S && r < D) ? W[s * D + r] : make_float2(0.f, 0.f);
              z[s4] = make_float2(u.x, -u.y);
            }
          };
          float2 rv[4], z[4];
          fetch(0, rv, z);
#pragma unroll 1
          for (int J = 0; J < NB; ++J) {
            float2 rn[4], zn[4];
            fetch(J + 1 < NB ? J + 1 : J, rn, zn);
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
              const double qr = rv[s4].x, qi = rv[s4].y, pr = z[s4].x, pi = z[s4].y;
              a1 = mfma64(qr, pr, a1);
              a2 = mfma64(qi, pi, a2);
              a3 = mfma64(qr + qi, pr + pi, a3);
            }
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
              rv[s4] = rn[s4];
              z[s4] = zn[s4];
            }
          }
          const doublex4 cr = a1 - a2, ci = a3 - a1 - a2;
          __syncthreads();  // earlier reads of tb are done
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int k = 16 * I + q + 4 * i;
            const float2 v = (s < S && k < D) ? steer[s * D + k] : make_float2(0.f, 0.f);
            tb[bofs(m, q + 4 * i)] = make_float2((float)((double)v.x - cr[i]), (float)(-(double)v.y - ci[i]));
          }
          __syncthreads();
          M[N * NB + I] = to_acc(frag_load(tb));
        }
      }
      forward_solve<NB, NS>(L, M);
      back_solve<NB, NS, LY::SLOTS>(L, M, tb);
      asm volatile("" ::: "memory");
      // Z += the correction (u parked in W)
#pragma unroll
      for (int N = 0; N < NS; ++N) {
        const int s = 16 * N + m;
#pragma unroll
        for (int J = 0; J < NB; ++J)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int k = 16 * J + 4 * q + i;
            if (s < S && k < D) {
              const float2 u = W[s * D + k];
              M[N * NB + J].re[i] += u.x;
              M[N * NB + J].im[i] -= u.y;
            }
          }
      }
    }
    if (d.refine > 0) {
      // gamma_s = Re(v_s^H u_s) in FP64 for the refined u = conj(Z)
#pragma unroll
      for (int N = 0; N < NS; ++N) {
        const int s = 16 * N + m;
        double p = 0.0;
#pragma unroll
        for (int J = 0; J < NB; ++J) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int k = 16 * J + 4 * q + i;
            if (s < S && k < D) {
              const float2 v = steer[s * D + k];
              p += (double)v.x * M[N * NB + J].re[i] - (double)v.y * M[N * NB + J].im[i];
            }
          }
        }
        p += __shfl_xor(p, 16);
        p += __shfl_xor(p, 32);
        gam[N] = p;
      }
    }
  }

  // ---- w_s = u_s / sqrt(gamma_s), u_s = conj(z_s)
#pragma unroll
  for (int N = 0; N < NS; ++N) {
    const int s = 16 * N + m;
    const float sc = 1.f / sqrtf((float)gam[N]);
    if (s < S) {
#pragma unroll
      for (int J = 0; J < NB; ++J) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int k = 16 * J + 4 * q + i;
          if (k < D) W[s * D + k] = make_float2(M[N * NB + J].re[i] * sc, -M[N * NB + J].im[i] * sc);
        }
      }
    }
  }
  if (lane == 0 && info) *info = 0;
}

}  // namespace wsv
}  // namespace stap
