// Adaptive weights by Cholesky solves (textbook STAP weight solve):
//
//   R_L = L L^H,  a_s = L^-1 v_s,  gamma_s = ||a_s||^2 = v_s^H R_L^-1 v_s,
//   u_s = L^-H a_s,  w_s = u_s / sqrt(gamma_s),
//
// plus optional iterative refinement: r_s = v_s - R_L u_s formed in FP64 from
// the FP32 matrix and iterate, u_s += R_L^-1 r_s with the FP32 factor.
//
// One workgroup (256 threads = a 16 x 16 grid ty, tx) per system.  The matrix
// M = [R_L ; V^H] ((D+S) x D) lives in REGISTERS, block-cyclically: thread
// (ty, tx) owns M[ty + 16a][tx + 16b].  The L part keeps only block slots
// a >= b (lower triangle); the steering part keeps all.  Right-looking
// factorisation: at column j the owners of column j+1 publish it through a
// double-buffered LDS vector after their own update, so each column costs one
// barrier.  Appending V^H below R_L makes the factorisation produce
// conj(L^-1 V) in the steering rows (the forward solve) in the same sweep.
// The back solve runs as a backward column sweep with the same one-barrier
// protocol.  Steering rows are stored conjugated: vm = conj(work).
#include "common.h"
#include "kernels.h"

namespace stap {

namespace {

template <int NB, int NV>
struct SolveShape {
  static constexpr int DP = NB * 16;
  static constexpr int SP = NV * 16;
  static size_t dyn_lds(int refine) {
    return refine > 0 ? (size_t)DP * (DP + 1) / 2 * 8 + (size_t)SP * DP * 8 : 0;
  }
};

__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }

template <int NB, int NV, bool REFINE>
__global__ __launch_bounds__(256) void solve_kernel(const float2* __restrict__ cov,
                                                    const float2* __restrict__ steer,
                                                    float2* __restrict__ wout, int* __restrict__ info_out,
                                                    Dims d) {
  constexpr int DP = NB * 16, SP = NV * 16;
  __shared__ float2 colL[2][DP];
  __shared__ float2 colV[2][SP];
  __shared__ float invd[DP];
  __shared__ float gam[SP];
  extern __shared__ __align__(16) float2 dyn[];  // refinement: packed R_L, then u

  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int sys = blockIdx.x;
  const int D = d.D, S = d.S;
  const float2* A = cov + (long long)sys * D * D;
  const int refine = REFINE ? d.refine : 0;

  float2 lm[NB][NB];
  float2 vm[NV][NB];

  if (REFINE) {
    // stage the lower triangle packed: row i at i(i+1)/2
    float2* Rp = dyn;
    for (int i = ty; i < D; i += 16)
      for (int k = tx; k <= i; k += 16) Rp[i * (i + 1) / 2 + k] = A[(long long)i * D + k];
  }
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      const int i = ty + 16 * a, k = tx + 16 * b;
      lm[a][b] = (i < D && k <= i) ? A[(long long)i * D + k] : make_float2(0.f, 0.f);
    }
#pragma unroll
  for (int a = 0; a < NV; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int s = ty + 16 * a, k = tx + 16 * b;
      vm[a][b] = (s < S && k < D) ? conjf2(steer[s * D + k]) : make_float2(0.f, 0.f);
    }

  // publish column 0
  if (tx == 0) {
#pragma unroll
    for (int a = 0; a < NB; ++a) colL[0][ty + 16 * a] = lm[a][0];
#pragma unroll
    for (int a = 0; a < NV; ++a) colV[0][ty + 16 * a] = vm[a][0];
  }
  __syncthreads();

  int fail = 0;
  for (int j = 0; j < D; ++j) {
    const int buf = j & 1;
    const float piv = colL[buf][j].x;
    if (!(piv > 0.f)) {
      fail = j + 1;
      break;
    }
    const float dj = sqrtf(piv), inv = 1.f / dj;
    const int jb = j >> 4, jt = j & 15;
    float2 li[NB], lk[NB], lv[NV];
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      const int i = ty + 16 * a;
      const float2 c = colL[buf][i];
      li[a] = (i > j) ? make_float2(c.x * inv, c.y * inv) : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int k = tx + 16 * b;
      const float2 c = colL[buf][k];
      lk[b] = (k > j && k < D) ? make_float2(c.x * inv, c.y * inv) : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int a = 0; a < NV; ++a) {
      const float2 c = colV[buf][ty + 16 * a];
      lv[a] = make_float2(c.x * inv, c.y * inv);
    }
    if (tid == 0) invd[j] = inv;
    if (tx == jt) {  // finalise column j
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (b == jb) {
#pragma unroll
          for (int a = b; a < NB; ++a) {
            const int i = ty + 16 * a;
            if (i > j) lm[a][b] = li[a];
            else if (i == j) lm[a][b] = make_float2(dj, 0.f);
          }
#pragma unroll
          for (int a = 0; a < NV; ++a) vm[a][b] = lv[a];
        }
    }
    const int s0 = (j + 1) >> 4;
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      if (a >= s0) {
#pragma unroll
        for (int b = 0; b <= a; ++b) {
          if (b >= s0) {
            const float2 p = cmulc(li[a], lk[b]);
            lm[a][b] = csub(lm[a][b], p);
          }
        }
      }
    }
#pragma unroll
    for (int a = 0; a < NV; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (b >= s0) vm[a][b] = csub(vm[a][b], cmulc(lv[a], lk[b]));

    // publish column j+1
    const int jn = j + 1;
    if (jn < D && tx == (jn & 15)) {
      const int nb = jn >> 4;
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (b == nb) {
#pragma unroll
          for (int a = 0; a < NB; ++a) colL[buf ^ 1][ty + 16 * a] = (a >= b) ? lm[a][b] : make_float2(0.f, 0.f);
#pragma unroll
          for (int a = 0; a < NV; ++a) colV[buf ^ 1][ty + 16 * a] = vm[a][b];
        }
    }
    __syncthreads();
  }

  if (fail) {
    for (int e = tid; e < S * D; e += 256) wout[(long long)sys * S * D + e] = make_float2(0.f, 0.f);
    if (tid == 0 && info_out) info_out[sys] = fail;
    return;
  }

  // gamma_s = ||a_s||^2 from the forward-solved steering rows
  {
#pragma unroll
    for (int a = 0; a < NV; ++a) {
      float g = 0.f;
#pragma unroll
      for (int b = 0; b < NB; ++b) g += vm[a][b].x * vm[a][b].x + vm[a][b].y * vm[a][b].y;
      g += __shfl_xor(g, 8, 16);
      g += __shfl_xor(g, 4, 16);
      g += __shfl_xor(g, 2, 16);
      g += __shfl_xor(g, 1, 16);
      if (tx == 0) gam[ty + 16 * a] = g;
    }
  }

  // Backward column sweep: L^H u = a, in conjugated storage
  //   c_s = vm_s[j] / L[j][j]   (= conj(u_s[j]))
  //   vm_s[k] -= L[j][k] c_s    for k < j
  // Buffers: colL carries row j of L, colV carries c.
  auto back_solve = [&](float2 (&x)[NV][NB]) {
    __syncthreads();
    for (int j = D - 1; j >= 0; --j) {
      const int buf = j & 1;
      const int jb = j >> 4, jt = j & 15;
      if (ty == jt) {  // row j of L: slot a = jb
#pragma unroll
        for (int a = 0; a < NB; ++a)
          if (a == jb) {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
              const int k = tx + 16 * b;
              colL[buf][k] = (b <= a && k < j) ? lm[a][b] : make_float2(0.f, 0.f);
            }
          }
      }
      if (tx == jt) {
        const float iv = invd[j];
#pragma unroll
        for (int b = 0; b < NB; ++b)
          if (b == jb) {
#pragma unroll
            for (int a = 0; a < NV; ++a) {
              const float2 c = make_float2(x[a][b].x * iv, x[a][b].y * iv);
              x[a][b] = c;
              colV[buf][ty + 16 * a] = c;
            }
          }
      }
      __syncthreads();
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        if (b <= jb) {
          const float2 l = colL[buf][tx + 16 * b];
#pragma unroll
          for (int a = 0; a < NV; ++a) x[a][b] = csub(x[a][b], cmul(l, colV[buf][ty + 16 * a]));
        }
      }
    }
    __syncthreads();
  };

  // Forward column sweep L z = r in conjugated storage (used by refinement):
  //   c_s = x_s[j] / L[j][j];  x_s[k] -= conj(L[k][j]) c_s  for k > j
  auto fwd_solve = [&](float2 (&x)[NV][NB]) {
    __syncthreads();
    for (int j = 0; j < D; ++j) {
      const int buf = j & 1;
      const int jb = j >> 4, jt = j & 15;
      if (tx == jt) {
        const float iv = invd[j];
#pragma unroll
        for (int b = 0; b < NB; ++b)
          if (b == jb) {
#pragma unroll
            for (int a = 0; a < NB; ++a) {
              const int i = ty + 16 * a;
              colL[buf][i] = (a >= b && i > j) ? lm[a][b] : make_float2(0.f, 0.f);
            }
#pragma unroll
            for (int a = 0; a < NV; ++a) {
              const float2 c = make_float2(x[a][b].x * iv, x[a][b].y * iv);
              x[a][b] = c;
              colV[buf][ty + 16 * a] = c;
            }
          }
      }
      __syncthreads();
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        if (b >= jb) {
          const float2 l = colL[buf][tx + 16 * b];
#pragma unroll
          for (int a = 0; a < NV; ++a) x[a][b] = csub(x[a][b], cmulc(colV[buf][ty + 16 * a], l));
        }
      }
    }
    __syncthreads();
  };

  back_solve(vm);

  if (REFINE) {
    const float2* Rp = dyn;
    float2* ub = dyn + DP * (DP + 1) / 2;  // [SP][DP] conj(u)
    for (int it = 0; it < refine; ++it) {
#pragma unroll
      for (int a = 0; a < NV; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) ub[(ty + 16 * a) * DP + tx + 16 * b] = vm[a][b];
      __syncthreads();
      // conj(r_s[k]) = conj(v_s[k]) - sum_q conj(R[k][q]) conj(u_s[q])   (FP64)
      double accr[NV][NB], acci[NV][NB];
#pragma unroll
      for (int a = 0; a < NV; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          accr[a][b] = 0.0;
          acci[a][b] = 0.0;
        }
      for (int q = 0; q < D; ++q) {
        float2 rc[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int k = tx + 16 * b;
          if (k < D) {
            // conj(R[k][q]) : lower element (k,q) conjugated, or (q,k) as is
            rc[b] = (q <= k) ? conjf2(Rp[k * (k + 1) / 2 + q]) : Rp[q * (q + 1) / 2 + k];
          } else {
            rc[b] = make_float2(0.f, 0.f);
          }
        }
#pragma unroll
        for (int a = 0; a < NV; ++a) {
          const float2 u = ub[(ty + 16 * a) * DP + q];
          const double ur = u.x, ui = u.y;
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const double rr = rc[b].x, ri = rc[b].y;
            accr[a][b] = fma(rr, ur, fma(-ri, ui, accr[a][b]));
            acci[a][b] = fma(rr, ui, fma(ri, ur, acci[a][b]));
          }
        }
      }
      float2 rv[NV][NB];
#pragma unroll
      for (int a = 0; a < NV; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int s = ty + 16 * a, k = tx + 16 * b;
          if (s < S && k < D) {
            const float2 v = steer[s * D + k];
            rv[a][b] = make_float2((float)((double)v.x - accr[a][b]), (float)(-(double)v.y - acci[a][b]));
          } else {
            rv[a][b] = make_float2(0.f, 0.f);
          }
        }
      fwd_solve(rv);
      back_solve(rv);
#pragma unroll
      for (int a = 0; a < NV; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) vm[a][b] = cadd(vm[a][b], rv[a][b]);
    }
    // gamma_s = Re(v_s^H u_s) in FP64 for the refined u
#pragma unroll
    for (int a = 0; a < NV; ++a) {
      double g = 0.0;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int s = ty + 16 * a, k = tx + 16 * b;
        if (s < S && k < D) {
          const float2 v = steer[s * D + k];
          // Re(conj(v) * u) with u = conj(vm)
          g += (double)v.x * vm[a][b].x - (double)v.y * vm[a][b].y;
        }
      }
      g += __shfl_xor(g, 8, 16);
      g += __shfl_xor(g, 4, 16);
      g += __shfl_xor(g, 2, 16);
      g += __shfl_xor(g, 1, 16);
      if (tx == 0) gam[ty + 16 * a] = (float)g;
    }
    __syncthreads();
  }

  // w_s = u_s / sqrt(gamma_s)
  float2* W = wout + (long long)sys * S * D;
#pragma unroll
  for (int a = 0; a < NV; ++a) {
    const int s = ty + 16 * a;
    if (s < S) {
      const float sc = 1.f / sqrtf(gam[s]);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int k = tx + 16 * b;
        if (k < D) W[s * D + k] = make_float2(vm[a][b].x * sc, -vm[a][b].y * sc);
      }
    }
  }
  if (tid == 0 && info_out) info_out[sys] = 0;
}

template <int NB, int NV>
hipError_t go_solve(const Dims& d, const float2* cov, const float2* steer, float2* w, int* info,
                    hipStream_t st) {
  if (d.refine == 0) {
    hipLaunchKernelGGL((solve_kernel<NB, NV, false>), dim3(d.P * d.B), dim3(256), 0, st, cov, steer, w, info, d);
    return hipGetLastError();
  }
  const size_t dyn = SolveShape<NB, NV>::dyn_lds(d.refine);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&solve_kernel<NB, NV, true>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((solve_kernel<NB, NV, true>), dim3(d.P * d.B), dim3(256), dyn, st, cov, steer, w, info, d);
  return hipGetLastError();
}

template <int NB>
hipError_t go_solve_nv(const Dims& d, const float2* cov, const float2* steer, float2* w, int* info,
                       hipStream_t st) {
  if (d.S <= 16) return go_solve<NB, 1>(d, cov, steer, w, info, st);
  if (d.S <= 32) return go_solve<NB, 2>(d, cov, steer, w, info, st);
  if (d.S <= 48) return go_solve<NB, 3>(d, cov, steer, w, info, st);
  return go_solve<NB, 4>(d, cov, steer, w, info, st);
}

}  // namespace

hipError_t launch_solve(const Dims& d, const float2* cov, const float2* steer, float2* w, int* info,
                        hipStream_t st) {
  switch ((d.D + 15) / 16) {
    case 1: return go_solve_nv<1>(d, cov, steer, w, info, st);
    case 2: return go_solve_nv<2>(d, cov, steer, w, info, st);
    case 3: return go_solve_nv<3>(d, cov, steer, w, info, st);
    case 4: return go_solve_nv<4>(d, cov, steer, w, info, st);
    case 5: return go_solve_nv<5>(d, cov, steer, w, info, st);
    case 6: return go_solve_nv<6>(d, cov, steer, w, info, st);
    case 7: return go_solve_nv<7>(d, cov, steer, w, info, st);
    case 8: return go_solve_nv<8>(d, cov, steer, w, info, st);
  }
  return hipErrorInvalidValue;  // D > 128: not handled by the register-resident kernel
}

}  // namespace stap
