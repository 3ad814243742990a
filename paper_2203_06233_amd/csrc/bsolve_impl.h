// Blocked Cholesky solve of one system on the FP32 matrix cores.
//
// The loaded covariance R_L (D x D, padded to 16 NB with an identity tail)
// and the conjugated steering rows M = V^H (S x D, padded to 16 NS rows with
// zeros) are cut into 16 x 16 complex blocks.  Each block lives in the
// registers of one wave for the whole solve (static round-robin ownership),
// so the right-looking updates never move the block they update; only the
// operands of a step pass through LDS.
//
//   factorisation  for each block column J: the owner of the diagonal block
//                  factors it (16 sequential columns inside one wave) and
//                  forms its triangular inverse Linv_JJ; the owners of the
//                  panel blocks form L_IJ = A_IJ Linv_JJ^H (and M_NJ :=
//                  M_NJ Linv_JJ^H, the forward solve riding along as extra
//                  rows); every later block X takes X -= P Q^H with P, Q
//                  from the published panel.  M ends as Y^H = (L^-1 V)^H.
//   gamma          gamma_s = ||y_s||^2.
//   back solve     in row form Z L = Y^H with Z = U^H: for J descending,
//                  Z_J = M_J Linv_JJ, then M_I -= Z_J L_JI for I < J.
//   output         w_s = u_s / sqrt(gamma_s), u_s = conj(row s of Z).
//
// Block products are 16 x 16 x 16 complex, four real 16 x 16 x 4 MFMAs per
// k-quarter.  Fragment layout (lane l, m = l % 16, q = l / 16): the lane holds
// X[m][4q + i], i = 0..3.  This is the MFMA result layout of X^T, and the A
// and B operand layouts of a product whose k index runs over the block
// columns, so every product is formed transposed (X^T -= conj(Q) P^T) and no
// block is ever shuffled.  In LDS a block keeps the same order (registers
// 0-1 of all lanes, then registers 2-3), so a fragment load is two 16-byte
// reads per lane with consecutive lanes on consecutive addresses.
#pragma once

#include "common.h"

namespace stap {

// The FP64 refinement residual either loads the operands of a block column's
// four k-steps before their products (more registers, less exposed LDS
// latency) or interleaves loads and products step by step.  Measured: the
// first is faster in the 8-wave one-cube fused kernel (7.16 -> 7.03 ms on
// the 32 x 256 x 16384 cube), the second in the persistent batched one
// (48.0 against 50.0 ms on the uneven batch); translation units choose with
// STAP_RESIDUAL_LOADS_AHEAD.
#ifdef STAP_RESIDUAL_LOADS_AHEAD
constexpr bool kResidualLoadsAhead = true;
#else
constexpr bool kResidualLoadsAhead = false;
#endif


struct Frag {
  float2 v[4];
};
struct Acc {
  floatx4 re, im;
};

// Complex offset of element (r, c) of a block stored in fragment order: the
// lane holding it is l = r + 16 (c / 4), its register i = c % 4; registers
// 0-1 of every lane come first (16 bytes per lane), then registers 2-3, so
// each of the two 16-byte accesses of a fragment covers one contiguous
// kilobyte across the wave.
__device__ __forceinline__ int bofs(int r, int c) {
  const int l = r + 16 * (c >> 2), i = c & 3;
  return (i < 2 ? 0 : 128) + 2 * l + (i & 1);
}

__device__ __forceinline__ Frag frag_load(const float2* blk) {
  const int l = lane_tid() & 63;
  const float4 a = *reinterpret_cast<const float4*>(blk + 2 * l);
  const float4 b = *reinterpret_cast<const float4*>(blk + 128 + 2 * l);
  Frag f;
  f.v[0] = make_float2(a.x, a.y);
  f.v[1] = make_float2(a.z, a.w);
  f.v[2] = make_float2(b.x, b.y);
  f.v[3] = make_float2(b.z, b.w);
  return f;
}
__device__ __forceinline__ void frag_store(float2* blk, const Frag& f) {
  const int l = lane_tid() & 63;
  *reinterpret_cast<float4*>(blk + 2 * l) = make_float4(f.v[0].x, f.v[0].y, f.v[1].x, f.v[1].y);
  *reinterpret_cast<float4*>(blk + 128 + 2 * l) = make_float4(f.v[2].x, f.v[2].y, f.v[3].x, f.v[3].y);
}
// Store X^T: the lane's X[m][4q + i] goes to element (4q + i, m).
__device__ __forceinline__ void frag_store_t(float2* blk, const Frag& f) {
  const int l = lane_tid() & 63, m = l & 15, q = l >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) blk[bofs(4 * q + i, m)] = f.v[i];
}
__device__ __forceinline__ Frag to_frag(const Acc& a) {
  Frag f;
#pragma unroll
  for (int i = 0; i < 4; ++i) f.v[i] = make_float2(a.re[i], a.im[i]);
  return f;
}
__device__ __forceinline__ Acc to_acc(const Frag& f) {
  Acc a;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    a.re[i] = f.v[i].x;
    a.im[i] = f.v[i].y;
  }
  return a;
}
__device__ __forceinline__ Acc acc_zero() {
  Acc a;
  a.re = floatx4{0.f, 0.f, 0.f, 0.f};
  a.im = floatx4{0.f, 0.f, 0.f, 0.f};
  return a;
}

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// x -= P Q^H (SUB) or x += P Q^H.  As x^T -/+= conj(Q) P^T: MFMA A operand
// conj(Q)[m][k], B operand P[m][k], k-quarter s covering k = 4 q' + s.
template <bool SUB>
__device__ __forceinline__ void mma_pqh(Acc& x, const Frag& P, const Frag& Q) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const float qr = SUB ? -Q.v[s].x : Q.v[s].x, qi = SUB ? -Q.v[s].y : Q.v[s].y;
    const float pr = P.v[s].x, pi = P.v[s].y;
    x.re = mfma4(qr, pr, x.re);  // Re(conj(q) p) = qr pr + qi pi
    x.re = mfma4(qi, pi, x.re);
    x.im = mfma4(qr, pi, x.im);  // Im(conj(q) p) = qr pi - qi pr
    x.im = mfma4(-qi, pr, x.im);
  }
}

// x -= P Q (SUB) or x += P Q, with Qt the fragment of Q^T.  As x^T -/+= Q^T P^T.
template <bool SUB>
__device__ __forceinline__ void mma_pq(Acc& x, const Frag& P, const Frag& Qt) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const float qr = SUB ? -Qt.v[s].x : Qt.v[s].x, qi = SUB ? -Qt.v[s].y : Qt.v[s].y;
    const float pr = P.v[s].x, pi = P.v[s].y;
    x.re = mfma4(qr, pr, x.re);  // Re(q p) = qr pr - qi pi
    x.re = mfma4(-qi, pi, x.re);
    x.im = mfma4(qr, pi, x.im);  // Im(q p) = qr pi + qi pr
    x.im = mfma4(qi, pr, x.im);
  }
}

__device__ __forceinline__ float2 shfl2(float2 v, int src) {
  return make_float2(__shfl(v.x, src), __shfl(v.y, src));
}
__device__ __forceinline__ float bcast(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Broadcast lane J of every 16-lane row to the whole row (DPP row_newbcast).
template <int J>
__device__ __forceinline__ float rowb(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x150 + J, 0xF, 0xF, true));
}
template <int J>
__device__ __forceinline__ float2 rowb2(float2 v) {
  return make_float2(rowb<J>(v.x), rowb<J>(v.y));
}

__device__ __forceinline__ double bcast64(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Column j of the in-wave factorisation of diag_factor_inv().  Rows and
// columns at or before j are never read again once column j is done, so the
// update of A needs no mask: with l = A[m][j] / d_j^2 (unmasked) the lanes
// take A[m][c] -= l A[j][c], which is right wherever m, c > j and harmless
// elsewhere.  The inverse is kept with unscaled rows Y (X[m] = Y[m] / d_m):
// rows below j take Y[m] -= (l_mj / d_j) Y[j]; the lane of row j records
// 1 / d_j for the final scaling.
//
// The pivot is taken in FP64: every lane keeps, for its row m, p64 =
// (loaded diagonal R_mm) - (sum over earlier block columns of |L_mk|^2, FP64
// sums of the FP32 factor) - (sum over earlier columns of this block of
// |l_mk|^2, accumulated here in FP64), so d_j^2 = p64 of row j (read from the
// lane holding the block's diagonal element j) and the status test is
// p64 > 0 in FP64; the factorisation continues with d_j^2 rounded to FP32.
// There is no branch: after a non-positive pivot the remaining columns run
// on meaningless values and only the first failing index is kept, so the 16
// columns form one straight-line block the compiler can overlap.
template <int j>
__device__ __forceinline__ void diag_col(Frag& A, Frag& X, int m, float& rsm, int& fail, double& p64) {
  constexpr int jq = j >> 2, ji = j & 3;
  const double piv64 = bcast64(p64, j + 16 * jq);  // row j's FP64 Schur diagonal, wave-uniform
  fail = (fail == 0 && !(piv64 > 0.0)) ? j + 1 : fail;
  const float piv = (float)piv64;
  const float rs = __builtin_amdgcn_rsqf(piv), r2 = rs * rs;
  const float2 amj = shfl2(A.v[ji], m + 16 * jq);  // A[m][j]
  const float2 la = make_float2(amj.x * r2, amj.y * r2);  // l_mj / d_j
  const float2 lx = (m > j) ? la : make_float2(0.f, 0.f);
  rsm = (m == j) ? rs : rsm;
  // l_mj = A[m][j] / d_j in FP32, squared and summed in FP64 for row m
  const float lr = amj.x * rs, li = amj.y * rs;
  p64 -= (m > j) ? (double)lr * (double)lr + (double)li * (double)li : 0.0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const float2 rj = rowb2<j>(A.v[t]);  // A[j][c] = conj(A[c][j])
    const float2 yj = rowb2<j>(X.v[t]);  // Y[j][c]
    // A[m][c] -= l_mj conj(l_cj) = (A[m][j] / d_j^2) A[j][c]
    A.v[t].x = fmaf(-la.x, rj.x, fmaf(la.y, rj.y, A.v[t].x));
    A.v[t].y = fmaf(-la.x, rj.y, fmaf(-la.y, rj.x, A.v[t].y));
    X.v[t].x = fmaf(-lx.x, yj.x, fmaf(lx.y, yj.y, X.v[t].x));
    X.v[t].y = fmaf(-lx.x, yj.y, fmaf(-lx.y, yj.x, X.v[t].y));
  }
}
template <int j>
__device__ __forceinline__ void diag_cols(Frag& A, Frag& X, int m, float& rsm, int& fail, double& p64) {
  diag_col<j>(A, X, m, rsm, fail, p64);
  if constexpr (j < 15) diag_cols<j + 1>(A, X, m, rsm, fail, p64);
}

// Factor the Hermitian 16 x 16 block A (full, both triangles) as L L^H inside
// one wave and return X = L^-1 (lower triangular).  Column j: pivot
// d_j = sqrt(A[j][j]) (taken in FP64 as above, p64 the lane's starting
// value for its row: loaded diagonal minus the earlier block columns),
// l_mj = A[m][j] / d_j for m > j, then A[m][c] -= l_mj conj(l_cj) for
// m, c > j; the inverse is accumulated as X <- L_j^-1 X with L_j the
// identity carrying column j of L (row j of X divided by d_j, then row m -=
// l_mj row j), the row divisions deferred.  A[c][j] is read as conj(A[j][c])
// from row j, which lives in the same 16-lane row of the wave (a DPP
// broadcast); only l_mj crosses rows.  Returns 0 or the 1-based index of the
// first non-positive pivot.
__device__ __forceinline__ int diag_factor_inv(Frag& A, Frag& X, double p64) {
  const int l = lane_tid() & 63, m = l & 15, q = l >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) X.v[i] = make_float2(m == 4 * q + i ? 1.f : 0.f, 0.f);
  int fail = 0;
  float rsm = 1.f;
  diag_cols<0>(A, X, m, rsm, fail, p64);
#pragma unroll
  for (int i = 0; i < 4; ++i) X.v[i] = make_float2(X.v[i].x * rsm, X.v[i].y * rsm);
  return fail;
}

// The lane's own diagonal element of a block in fragment order (lane (m, q)
// holds X[m][4q + i]; the element (m, m) sits in lane q = m / 4, register
// m % 4), or 0 on the other lanes.
__device__ __forceinline__ float frag_diag(const Frag& A) {
  const int l = lane_tid() & 63, m = l & 15, q = l >> 4;
  float v = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) v = (m == 4 * q + i) ? A.v[i].x : v;
  return v;
}

// Row sums of |X|^2 of a block in fragment order, in FP64, on every lane of
// the row (lane (m, q) holds row m, columns 4q .. 4q + 3).
__device__ __forceinline__ double frag_row_norm2(const Acc& x) {
  double p = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    p += (double)x.re[i] * (double)x.re[i] + (double)x.im[i] * (double)x.im[i];
  p += __shfl_xor(p, 16);
  p += __shfl_xor(p, 32);
  return p;
}

// Static layout of one system with NB block columns of R_L and NS block rows
// of steering vectors (both run-time), NW waves, and per wave NSL register
// slots for L blocks and NSM for M blocks (compile time).  L blocks are
// numbered column by column from the diagonal down, M blocks column by
// column, each set dealt round-robin to the waves (block g -> wave g % NW,
// slot g / NW).  The blocks still active at a step are a suffix of each
// order, so every step is balanced to within one block per wave and set.
// Loops over a wave's blocks run over its slots (unrolled, so register
// indices are constants) and test the slot's block coordinates, which are
// run-time values.
template <int NSL_, int NSM_, int NW_>
struct BCfg {
  static constexpr int NSL = NSL_, NSM = NSM_, NW = NW_;
  static constexpr int NT = 64 * NW;
  // L and M slots per wave a (NB, NS) system needs
  __host__ __device__ static constexpr int lslots(int NB) { return (NB * (NB + 1) / 2 + NW - 1) / NW; }
  __host__ __device__ static constexpr int mslots(int NB, int NS) { return (NS * NB + NW - 1) / NW; }
  // LDS: exchange blocks (NB + NS + 1 for the factorisation and solves, all
  // NS NB blocks of Z for the refinement residual), the gamma partials
  // [NB][16 NS] (FP64), a flag, and the FP64 row sums of |L|^2 over the
  // finished block columns [16 NB] (for the FP64 pivots)
  __host__ __device__ static constexpr size_t xblocks(int NB, int NS) {
    return (size_t)(NB + NS + 1 > NS * NB ? NB + NS + 1 : NS * NB);
  }
  __host__ __device__ static constexpr size_t lds_bytes(int NB, int NS) {
    return xblocks(NB, NS) * 256 * 8 + (size_t)NB * 16 * NS * 8 + 16 + (size_t)NB * 16 * 8;
  }
};

// Factor diagonal block Jd held in L slot td (after its last update from the
// panel L_{Jd,Jd-1} in xb when `update`), keep Linv in the slot, publish it
// at dinv and the pivot status at sflag.  The block passes through dinv on
// its way in and out of the register slot, so the diagonal code exists once
// and every register slot is addressed by a constant index.
// The FP64 pivots start from the loaded diagonal of the block (rdg, kept
// per slot since the load) minus the FP64 row sums of |L|^2 over the earlier
// block columns (d64, LDS).
template <int NSL>
__device__ __forceinline__ void bs_factor_diag(Acc (&acc)[NSL], const float (&rdg)[NSL], int td, int Jd, bool update,
                                               const float2* xb, const double* d64, float2* dinv, int* sflag) {
  float rd = 0.f;
#pragma unroll
  for (int t = 0; t < NSL; ++t)
    if (td == t) {
      frag_store(dinv, to_frag(acc[t]));
      rd = rdg[t];
    }
  Frag A = frag_load(dinv), X;
  if (update) {
    Acc a = to_acc(A);
    const Frag P = frag_load(xb + Jd * 256);
    mma_pqh<true>(a, P, P);
    A = to_frag(a);
  }
  const int m = lane_tid() & 15;
  const double p64 = (double)rd - (Jd > 0 ? d64[16 * Jd + m] : 0.0);
  const int f = diag_factor_inv(A, X, p64);
  frag_store(dinv, X);
#pragma unroll
  for (int t = 0; t < NSL; ++t)
    if (td == t) acc[t] = to_acc(X);
  if ((lane_tid() & 63) == 0) *sflag = f ? 16 * Jd + f : 0;
}

__device__ __forceinline__ doublex4 mfma64(double a, double b, doublex4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// A global read the compiler must not merge with an earlier read of the
// same address: keeping such values live across the whole solve costs more
// registers than reading them again (they are cache hits).
__device__ __forceinline__ float2 reload(const float2* p) {
  const volatile float* v = reinterpret_cast<const volatile float*>(p);
  return make_float2(v[0], v[1]);
}

// Solve one system (D <= 16 NB, S <= 16 NS, lslots(NB) <= NSL,
// mslots(NB, NS) <= NSM).  src.lower(i, k) (k <= i < D) yields the loaded
// covariance; it must stay readable for the whole call when REFINE (the FP64
// residual reads it again).  xlds points at lds_bytes(NB, NS) of 16-byte
// aligned LDS, which may overlap the source only without REFINE (the source
// is read completely before the first write).  W is this system's [S][D]
// output, info its status word (may be null).  park (may be null) is LDS of
// at least 16 NS x 16 NB complex that is free once the last residual has
// been formed (the source, when it lives in LDS): the last refinement step
// keeps u there instead of in W.
template <class C, bool REFINE, class RSrc>
__device__ __forceinline__ void bsolve_system(const RSrc& src, const float2* __restrict__ steer,
                                              float2* __restrict__ W, int* __restrict__ info, const Dims& d,
                                              unsigned char* xlds, float2* park = nullptr) {
  constexpr int NSL = C::NSL, NSM = C::NSM, NW = C::NW;
  const int D = d.D, S = d.S;
  const int NB = (D + 15) >> 4, NS = (S + 15) >> 4;
  float2* xb = reinterpret_cast<float2*>(xlds);  // exchange blocks, 256 complex each
  double* gpart = reinterpret_cast<double*>(xlds + C::xblocks(NB, NS) * 256 * 8);
  int* sflag = reinterpret_cast<int*>(gpart + NB * 16 * NS);
  double* d64 = reinterpret_cast<double*>(reinterpret_cast<unsigned char*>(sflag) + 16);
  const int tid = lane_tid(), lane = tid & 63, m = lane & 15, q = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  float2* dinv = xb + (size_t)(NB + NS) * 256;

  // block coordinates of each slot
  bool lv[NSL], mv[NSM];
  int lr[NSL], lc[NSL], mr[NSM], mc[NSM];
#pragma unroll
  for (int t = 0; t < NSL; ++t) {
    const int g = wave + NW * t;
    lv[t] = false;
    lr[t] = 0;
    lc[t] = 0;
    int start = 0;
    for (int J = 0; J < NB; ++J) {
      const int len = NB - J;
      if (g >= start && g < start + len) {
        lv[t] = true;
        lc[t] = J;
        lr[t] = J + (g - start);
      }
      start += len;
    }
  }
#pragma unroll
  for (int t = 0; t < NSM; ++t) {
    const int g = wave + NW * t;
    mv[t] = g < NS * NB;
    mc[t] = g / NS;
    mr[t] = g - (g / NS) * NS;
  }

  Acc al[NSL], am[NSM];
  float rdg[NSL];  // loaded diagonal of the slot's block (diagonal blocks), for the FP64 pivots
  // ---- load R_L blocks (identity beyond D) and M = V^H blocks
#pragma unroll
  for (int t = 0; t < NSL; ++t) {
    Acc a = acc_zero();
    if (lv[t]) {
      const int r = 16 * lr[t] + m;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = 16 * lc[t] + 4 * q + i;
        float2 v;
        if (r < D && c < D) {
          if (c <= r) {
            v = src.lower(r, c);
          } else {
            v = src.lower(c, r);
            v.y = -v.y;
          }
        } else {
          v = make_float2(r == c ? 1.f : 0.f, 0.f);
        }
        a.re[i] = v.x;
        a.im[i] = v.y;
      }
    }
    al[t] = a;
    rdg[t] = frag_diag(to_frag(a));
  }
#pragma unroll
  for (int t = 0; t < NSM; ++t) {
    Acc a = acc_zero();
    if (mv[t]) {
      const int s = 16 * mr[t] + m;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = 16 * mc[t] + 4 * q + i;
        const float2 v = (s < S && k < D) ? steer[s * D + k] : make_float2(0.f, 0.f);
        a.re[i] = v.x;
        a.im[i] = -v.y;
      }
    }
    am[t] = a;
  }
  __syncthreads();  // without REFINE the source may be LDS that the exchange blocks reuse
  for (int r = tid; r < 16 * NB; r += C::NT) d64[r] = 0.0;  // read from step J = 0 on, after a barrier

  // ---- factorisation with the forward solve of the steering rows.  The
  // wave owning diagonal block J+1 applies its last update (from column J)
  // first and factors it right away, while the other waves finish the
  // updates of step J; step J = -1 only factors diagonal block 0.
  int fail = 0;
  for (int J = -1; J < NB; ++J) {
    if (J >= 0) {
      __syncthreads();
      fail = *sflag;
      if (fail) break;
      const Frag Q = frag_load(dinv);
#pragma unroll
      for (int t = 0; t < NSL; ++t) {
        if (lv[t] && lc[t] == J && lr[t] != J) {
          const Frag P = to_frag(al[t]);
          Acc x = acc_zero();
          mma_pqh<false>(x, P, Q);
          al[t] = x;
          frag_store(xb + lr[t] * 256, to_frag(x));
          // FP64 row sums of |L|^2 for the pivots of block row lr (one
          // panel block per block row and step: no other writer)
          const double pn = frag_row_norm2(x);
          if (q == 0) d64[16 * lr[t] + m] += pn;
        }
      }
#pragma unroll
      for (int t = 0; t < NSM; ++t) {
        if (mv[t] && mc[t] == J) {
          const Frag P = to_frag(am[t]);
          Acc x = acc_zero();
          mma_pqh<false>(x, P, Q);
          am[t] = x;
          frag_store(xb + (NB + mr[t]) * 256, to_frag(x));
        }
      }
      __syncthreads();
    }
    int tn = -1;
#pragma unroll
    for (int t = 0; t < NSL; ++t)
      if (J + 1 < NB && lv[t] && lr[t] == J + 1 && lc[t] == J + 1) tn = t;
    if (tn >= 0) bs_factor_diag<NSL>(al, rdg, tn, J + 1, J >= 0, xb, d64, dinv, sflag);
    if (J >= 0) {
#pragma unroll
      for (int t = 0; t < NSL; ++t)
        if (lv[t] && lc[t] > J && t != tn)
          mma_pqh<true>(al[t], frag_load(xb + lr[t] * 256), frag_load(xb + lc[t] * 256));
#pragma unroll
      for (int t = 0; t < NSM; ++t)
        if (mv[t] && mc[t] > J)
          mma_pqh<true>(am[t], frag_load(xb + (NB + mr[t]) * 256), frag_load(xb + mc[t] * 256));
    }
  }

  if (fail) {
    for (int e = tid; e < S * D; e += C::NT) W[e] = make_float2(0.f, 0.f);
    if (tid == 0 && info) *info = fail;
    return;
  }

  // ---- gamma_s = ||y_s||^2 (no refinement), partial per block column
  if (!REFINE || d.refine == 0) {
#pragma unroll
    for (int t = 0; t < NSM; ++t) {
      if (mv[t]) {
        float p = 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) p = fmaf(am[t].re[i], am[t].re[i], fmaf(am[t].im[i], am[t].im[i], p));
        p += __shfl_xor(p, 16);
        p += __shfl_xor(p, 32);
        if (q == 0) gpart[mc[t] * 16 * NS + 16 * mr[t] + m] = p;
      }
    }
  }

  // ---- back solve, row form Z L = Y^H (M holds Y^H on entry, Z on exit)
  auto back_solve = [&]() {
    float2* zb = xb + (size_t)NB * 256;
    for (int J = NB - 1; J >= 0; --J) {
      __syncthreads();  // previous readers of the exchange blocks are done
#pragma unroll
      for (int t = 0; t < NSL; ++t)  // L_JI^T (Linv_JJ^T at I = J)
        if (lv[t] && lr[t] == J) frag_store_t(xb + lc[t] * 256, to_frag(al[t]));
      __syncthreads();
#pragma unroll
      for (int t = 0; t < NSM; ++t) {
        if (mv[t] && mc[t] == J) {
          const Frag P = to_frag(am[t]);
          Acc x = acc_zero();
          mma_pq<false>(x, P, frag_load(xb + J * 256));
          am[t] = x;
          frag_store(zb + mr[t] * 256, to_frag(x));
        }
      }
      if (J > 0) {
        __syncthreads();
#pragma unroll
        for (int t = 0; t < NSM; ++t)
          if (mv[t] && mc[t] < J) mma_pq<true>(am[t], frag_load(zb + mr[t] * 256), frag_load(xb + mc[t] * 256));
      }
    }
  };
  back_solve();

  if (REFINE) {
    for (int it = 0; it < d.refine; ++it) {
      const bool lds_park = park != nullptr && it == d.refine - 1;
      // keep the current u = conj(Z) in W (this lane's own elements; read
      // back by the same lane after the correction), or in park
#pragma unroll
      for (int t = 0; t < NSM; ++t) {
        if (mv[t] && !lds_park) {
          const int s = 16 * mr[t] + m;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int k = 16 * mc[t] + 4 * q + i;
            if (s < S && k < D) W[s * D + k] = make_float2(am[t].re[i], -am[t].im[i]);
          }
        }
      }
      // residual in row form: conj(r) = conj(v) - Z R_L, FP64 MFMA (FP32
      // operands converted exactly).  Every Z block is published; each M
      // block's owner sums over J.  Each complex product q p takes three real
      // products (Gauss): a1 += qr pr, a2 += qi pi, a3 += (qr + qi)(pr + pi),
      // then Re = a1 - a2 and Im = a3 - a1 - a2 (the FP64 sums qr + qi and
      // pr + pi of FP32 values are exact).  Lane (m, q) register i of an
      // accumulator holds column q + 4i of the block.
      __syncthreads();
#pragma unroll
      for (int t = 0; t < NSM; ++t)
        if (mv[t]) frag_store(xb + (mr[t] * NB + mc[t]) * 256, to_frag(am[t]));
      __syncthreads();
#pragma unroll
      for (int t = 0; t < NSM; ++t) {
        if (mv[t]) {
          doublex4 a1 = {0.0, 0.0, 0.0, 0.0}, a2 = a1, a3 = a1;
          const float2* zrow = xb + (size_t)mr[t] * NB * 256 + 2 * lane;
          const int c = 16 * mc[t] + m;
          // R_L[r][c] for r = 16 J + 4 q + s4, c = 16 I + m (identity beyond D)
          auto r_elem = [&](int J, int s4) {
            const int r = 16 * J + 4 * q + s4;
            float2 rv;
            if (r < D && c < D) {
              rv = c <= r ? src.lower(r, c) : src.lower(c, r);
              rv.y = c <= r ? rv.y : -rv.y;
            } else {
              rv = make_float2(r == c ? 1.f : 0.f, 0.f);
            }
            return rv;
          };
          auto acc3 = [&](float2 rv, float2 z) {
            const double qr = rv.x, qi = rv.y, pr = z.x, pi = z.y;
            a1 = mfma64(qr, pr, a1);
            a2 = mfma64(qi, pi, a2);
            a3 = mfma64(qr + qi, pr + pi, a3);
          };
          for (int J = 0; J < NB; ++J) {
            if constexpr (kResidualLoadsAhead) {
              // the four k-steps' operands loaded before their products
              float2 zz[4], rr[4];
#pragma unroll
              for (int s4 = 0; s4 < 4; ++s4) {
                zz[s4] = zrow[J * 256 + (s4 & 2) * 64 + (s4 & 1)];  // Z_{N,J}[m][4q + s4]
                rr[s4] = r_elem(J, s4);
              }
#pragma unroll
              for (int s4 = 0; s4 < 4; ++s4) acc3(rr[s4], zz[s4]);
            } else {
#pragma unroll 1
              for (int s4 = 0; s4 < 4; ++s4) acc3(r_elem(J, s4), zrow[J * 256 + (s4 & 2) * 64 + (s4 & 1)]);
            }
          }
          const doublex4 cr = a1 - a2, ci = a3 - a1 - a2;
          const int s = 16 * mr[t] + m;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int k = 16 * mc[t] + q + 4 * i;
            const float2 v = (s < S && k < D) ? reload(steer + s * D + k) : make_float2(0.f, 0.f);
            // the slot's Z is in LDS now: its registers hold the residual,
            // column q + 4i in register i
            am[t].re[i] = (float)((double)v.x - cr[i]);
            am[t].im[i] = (float)(-(double)v.y - ci[i]);
          }
        }
      }
      __syncthreads();  // every Z block has been read
      // conj(r) rounded to FP32, back into fragment order through the
      // block's own (now free) Z position, or through its park slot, which
      // then takes the Z block itself (u for the correction)
#pragma unroll
      for (int t = 0; t < NSM; ++t) {
        if (mv[t]) {
          float2* zb = xb + (mr[t] * NB + mc[t]) * 256;
          float2* tb = lds_park ? park + (mr[t] * NB + mc[t]) * 256 : zb;
#pragma unroll
          for (int i = 0; i < 4; ++i) tb[bofs(m, q + 4 * i)] = make_float2(am[t].re[i], am[t].im[i]);
          am[t] = to_acc(frag_load(tb));
          if (lds_park) frag_store(tb, frag_load(zb));
        }
      }
      // forward solve Y^H L^H = r^H with the stored factor
      for (int J = 0; J < NB; ++J) {
        __syncthreads();
#pragma unroll
        for (int t = 0; t < NSL; ++t)  // column J of L (Linv_JJ at the diagonal)
          if (lv[t] && lc[t] == J) frag_store(xb + lr[t] * 256, to_frag(al[t]));
        __syncthreads();
#pragma unroll
        for (int t = 0; t < NSM; ++t) {
          if (mv[t] && mc[t] == J) {
            const Frag P = to_frag(am[t]);
            Acc x = acc_zero();
            mma_pqh<false>(x, P, frag_load(xb + J * 256));
            am[t] = x;
            frag_store(xb + (NB + mr[t]) * 256, to_frag(x));
          }
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < NSM; ++t)
          if (mv[t] && mc[t] > J)
            mma_pqh<true>(am[t], frag_load(xb + (NB + mr[t]) * 256), frag_load(xb + mc[t] * 256));
      }
      back_solve();
      // Z += the correction (u kept in W or park)
#pragma unroll
      for (int t = 0; t < NSM; ++t) {
        if (mv[t] && lds_park) {
          const Acc z = to_acc(frag_load(park + (mr[t] * NB + mc[t]) * 256));
          am[t].re += z.re;
          am[t].im += z.im;
        } else if (mv[t]) {
          const int s = 16 * mr[t] + m;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int k = 16 * mc[t] + 4 * q + i;
            if (s < S && k < D) {
              const float2 u = reload(W + s * D + k);
              am[t].re[i] += u.x;
              am[t].im[i] -= u.y;
            }
          }
        }
      }
    }
    if (d.refine > 0) {
      // gamma_s = Re(v_s^H u_s) in FP64 for the refined u, u = conj(Z)
#pragma unroll
      for (int t = 0; t < NSM; ++t) {
        if (mv[t]) {
          const int s = 16 * mr[t] + m;
          double p = 0.0;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int k = 16 * mc[t] + 4 * q + i;
            if (s < S && k < D) {
              const float2 v = reload(steer + s * D + k);
              p += (double)v.x * am[t].re[i] - (double)v.y * am[t].im[i];  // Re(conj(v) conj(z))
            }
          }
          p += __shfl_xor(p, 16);
          p += __shfl_xor(p, 32);
          if (q == 0) gpart[mc[t] * 16 * NS + 16 * mr[t] + m] = p;
        }
      }
    }
  }
  __syncthreads();  // gamma partials

  // ---- w_s = u_s / sqrt(gamma_s), u_s = conj(z_s)
#pragma unroll
  for (int t = 0; t < NSM; ++t) {
    if (mv[t]) {
      const int s = 16 * mr[t] + m;
      double gam = 0.0;
      for (int J = 0; J < NB; ++J) gam += gpart[J * 16 * NS + s];
      const float sc = 1.f / sqrtf((float)gam);
      if (s < S) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int k = 16 * mc[t] + 4 * q + i;
          if (k < D) W[s * D + k] = make_float2(am[t].re[i] * sc, -am[t].im[i] * sc);
        }
      }
    }
  }
  if (tid == 0 && info) *info = 0;
}

}  // namespace stap
