/*
 * stap.h -- C ABI of the MI355X (gfx950) STAP hot-path library (libstap.so).
 *
 * The library computes post-Doppler space-time adaptive processing (STAP) for
 * radar datacubes, the application whose kernel the paper parallelises:
 * Shirako et al., "Automatic Parallelization of Python Programs for
 * Distributed Heterogeneous Computing", arXiv 2203.06233.  Sec. 5.3 states the
 * problem: datacubes of pulses x channels x samples (range cells) per pulse.
 * Sec. 4.2 and the figure "Kernel from the STAP Signal Processing Application"
 * describe the kernel as an explicit loop (statement S), an fft along one axis
 * (statement T; Table 2, row fft_{2D,axis=1}) and a 2-D x 2-D array multiply
 * (statement U; Table 2, row dot_{2D,2D}), fused into one parallel loop over
 * independent units.  The step definitions below are textbook post-Doppler
 * STAP (Melvin 2014, the paper's STAP reference) under these readings:
 *
 *   Doppler    X[k][t*C+c][r] = sum_p h_t[p] x[c][p][r] exp(-j 2 pi k p / P),
 *              h_t[p] = h[p-t] for t <= p < t+L, L = P-T+1, h the symmetric
 *              Hann window h[n] = 1/2 - 1/2 cos(2 pi n/(L-1)); k = 0..P-1
 *              (with STAP_TAP_RELATIVE the kernel is exp(-j 2 pi k (p-t)/P)).
 *   Covariance R_hat[k][b] = (1/N) sum_{r in Omega_b} X[k][:,r] X[k][:,r]^H,
 *              Omega_b the N cells of block b (blocks of N = R/B
 *              contiguous range cells), or with STAP_TRAIN_EXCLUDE the N
 *              nearest cells outside the block and its guard cells.
 *   Loading    delta = eps * Re tr(R_hat) / D,  R_L = R_hat + delta I.
 *   Weights    R_L = L L^H (Cholesky),  u_s = R_L^-1 v_s,
 *              gamma_s = Re(v_s^H u_s),  w_s = u_s / sqrt(gamma_s); the
 *              steering vectors v_s are shared by every bin, or given per
 *              bin (steer_per_bin).
 *   Output     y[k][s][r] = w_{k,b(r),s}^H X[k][:,r],  power = |y|^2.
 *
 * Conventions for every entry point:
 *   - All array arguments are DEVICE pointers owned by the caller; the library
 *     never allocates, frees or copies to the host on these calls.  Work is
 *     enqueued on `stream` (a hipStream_t, 0 = the null stream) and the call
 *     returns without synchronising.
 *   - Complex values are stap_cf32 {re, im} (bit-compatible with
 *     std::complex<float>, numpy complex64 and torch.complex64).
 *   - Arrays are dense, row-major, last index fastest, in the layouts given
 *     with each argument.  Complex arrays must be 8-byte aligned, float and
 *     int32 arrays 4-byte aligned, the stap_run workspace 256-byte aligned
 *     (STAP_ERR_ALIGN otherwise).
 *   - Argument, shape, alignment and workspace errors are detected on the
 *     host before anything is enqueued and return a negative stap_status.
 *     A numerical failure (a pivot of the Cholesky factorisation that is not
 *     positive) is reported per system in `info` (LAPACK potrf convention:
 *     0 = success, j > 0 = 1-based index of the first bad pivot); that
 *     system's weights and output power are zero and the call still returns
 *     STAP_OK.
 *   - Limits: n_pulse P a power of two in [32, 512] or 100 (the paper's
 *     pulse count); 1 <= tdof T <= 4 and T < P; D = T*C <= 192 with C the
 *     channels after subarray summing; n_range R divisible by n_block B;
 *     1 <= S <= 64.
 *   - Subarrays (the reading used for the paper's 1000-channel cube, Sec.
 *     5.3): with subarray = n > 1 the cube holds n_chan array elements and
 *     channel c is the sum of elements c*n .. c*n + n - 1, formed by the
 *     Doppler step as it reads the cube.
 */
#ifndef STAP_H
#define STAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stap_cf32 {
  float re, im;
} stap_cf32;

typedef enum stap_status {
  STAP_OK = 0,
  STAP_ERR_ARG = -1,          /* null pointer or value out of range */
  STAP_ERR_SHAPE = -2,        /* dimensions outside the supported limits */
  STAP_ERR_ALIGN = -3,        /* a device pointer is misaligned */
  STAP_ERR_WORKSPACE = -4,    /* workspace missing or smaller than needed */
  STAP_ERR_HIP = -5,          /* a HIP runtime call failed (launch, query) */
  STAP_ERR_UNSUPPORTED = -6   /* valid request this build does not handle */
} stap_status;

typedef enum stap_precision {
  /* FP32 throughout: FP32 FFT, FP32 covariance on FP32 MFMA, FP32
   * Cholesky/solves, FP32 inner products. */
  STAP_PREC_FP32 = 0,
  /* Mixed: covariance and inner products as BF16 MFMA products with FP32
   * accumulation (each FP32 operand split exactly into three BF16 terms),
   * FP32 Cholesky/solves, FP64 refinement residual. */
  STAP_PREC_BF16 = 1,
  /* As BF16 but the covariance is one FP8 (OCP E4M3) product per element
   * with a power-of-two scale per (bin, block) and FP32 accumulation. */
  STAP_PREC_FP8 = 2
} stap_precision;

/* Which range cells train the covariance of block b (cells [bN, bN+N)). */
typedef enum stap_training {
  /* The block's own N cells (the cells under test are part of their own
   * training set). */
  STAP_TRAIN_BLOCK = 0,
  /* Standard STAP practice (Melvin 2014): the block and `guard_cells` cells
   * on each side are excluded, and the N nearest remaining cells train the
   * block -- floor(N/2) on the left and the rest on the right, moved to the
   * other side where a side runs out of cells at the edge of the cube.
   * Every block must find N such cells: R - N - 2G >= N for interior
   * blocks, R - N - G >= N at the edges (STAP_ERR_SHAPE otherwise). */
  STAP_TRAIN_EXCLUDE = 1
} stap_training;

/* Phase reference of the time-staggered taps in the Doppler DFT. */
typedef enum stap_tap_phase {
  /* Absolute pulse index: tap t's DFT kernel is exp(-j 2 pi k p / P) at
   * pulse p, so an on-bin target has the same phase in every tap. */
  STAP_TAP_ABSOLUTE = 0,
  /* Each tap referenced to its own first pulse: exp(-j 2 pi k (p - t) / P),
   * the DFT of the windowed sub-CPI itself; an on-bin target at bin k then
   * carries exp(j 2 pi k t / P) in tap t, which per-bin steering matches. */
  STAP_TAP_RELATIVE = 1
} stap_tap_phase;

/* One datacube's problem statement (Sec. 5.3: pulses x channels x samples),
 * plus the adaptive-processing parameters. */
typedef struct stap_problem {
  int32_t n_chan;        /* C: receive channels */
  int32_t n_pulse;       /* P: pulses per CPI = FFT length = Doppler bins */
  int32_t n_range;       /* R: range cells (samples per pulse) */
  int32_t tdof;          /* T: time-staggered taps (temporal DOF); D = T*C */
  int32_t n_block;       /* B: training blocks along range, N = R/B cells */
  int32_t n_steer;       /* S: steering vectors */
  float load_eps;        /* eps >= 0: loading delta = eps * tr(R_hat) / D */
  int32_t precision;     /* stap_precision */
  int32_t refine_steps;  /* FP64 iterative-refinement steps, 0..4 */
  int32_t training;      /* stap_training */
  int64_t cube_stride_chan;   /* elements between channels of `cube`; 0 = P*R */
  int64_t cube_stride_pulse;  /* elements between pulses of `cube`; 0 = R.
                                 The range stride is always 1. */
  int32_t guard_cells;   /* G >= 0 guard cells per side (STAP_TRAIN_EXCLUDE;
                            must be 0 with STAP_TRAIN_BLOCK) */
  int32_t tap_phase;     /* stap_tap_phase */
  int32_t steer_per_bin; /* 0: one steering set V[S][D] for every Doppler
                            bin; 1: a set per bin, V[P][S][D] */
  int32_t subarray;      /* array elements summed into each channel: n_chan
                            counts elements, the processing sees
                            C = n_chan / subarray channels (0 or 1: none) */
} stap_problem;

/* Doppler filtering with time-staggered DOF (statements S and T of the
 * paper's kernel, Sec. 4.2; Table 2 row fft_{2D,axis=1}).
 *   cube  in : x[n_chan][P][R] complex, strides from `prob` (range stride
 *              1; channels outermost, or pulses outermost as in the paper's
 *              pulses x channels x samples cube).
 *   snap  out: X[P][D][R] complex, D = T*C, d = t*C + c, bins k = 0..P-1.
 * FP32 arithmetic for every precision. */
stap_status stap_doppler(const stap_problem* prob, const stap_cf32* cube,
                         stap_cf32* snap, void* stream);

/* Sample covariance per (Doppler bin, training block) with diagonal loading
 * (statement U, Sec. 4.2; Table 2 row dot_{2D,2D}).
 *   snap  in : X[P][D][R] as written by stap_doppler.
 *   cov   out: R_L[P][B][D][D], full Hermitian (both triangles; the upper is
 *              the conjugate of the lower, bit for bit), loading included.
 *   delta out: delta[P][B] float, may be NULL.
 * Arithmetic per prob->precision (FP32 MFMA, split-BF16 MFMA or scaled FP8
 * MFMA, FP32 accumulation); the trace for the loading is summed in FP64. */
stap_status stap_covariance(const stap_problem* prob, const stap_cf32* snap,
                            stap_cf32* cov, float* delta, void* stream);

/* Adaptive weights by Cholesky solves (the textbook STAP weight solve).
 *   cov   in : R_L[P][B][D][D] Hermitian; only the lower triangle is read.
 *   steer in : V[S][D] steering vectors, or V[P][S][D] with steer_per_bin.
 *   w     out: W[P][B][S][D], w_s = R_L^-1 v_s / sqrt(v_s^H R_L^-1 v_s).
 *   info  out: info[P][B] int32 (0 = ok, j = first non-positive pivot).
 * FP32 factorisation and triangular solves; prob->refine_steps steps of
 * iterative refinement whose residual v - R_L u is formed in FP64. */
stap_status stap_solve_weights(const stap_problem* prob, const stap_cf32* cov,
                               const stap_cf32* steer, stap_cf32* w,
                               int32_t* info, void* stream);

/* Covariance, loading, Cholesky and solves fused per system (the path
 * stap_run takes): the loaded covariance stays on chip.  Same definitions,
 * arithmetic and outputs as stap_covariance followed by stap_solve_weights
 * (weights and info; the covariance itself is not written).
 *   snap  in : X[P][D][R];  steer in: V[S][D] (V[P][S][D] with steer_per_bin).
 *   w     out: W[P][B][S][D];  info out: info[P][B].
 * STAP_ERR_UNSUPPORTED for D > 128 or FP8 (use the two stage calls). */
stap_status stap_covariance_solve(const stap_problem* prob, const stap_cf32* snap,
                                  const stap_cf32* steer, stap_cf32* w,
                                  int32_t* info, void* stream);

/* Weight x snapshot inner products and output power (statement U applied to
 * the weights; the adaptive filter output).
 *   w     in : W[P][B][S][D];  snap in: X[P][D][R].
 *   power out: |y|^2 as float [P][S][R].
 *   y     out: y[P][S][R] complex, may be NULL. */
stap_status stap_inner_products(const stap_problem* prob, const stap_cf32* w,
                                const stap_cf32* snap, float* power,
                                stap_cf32* y, void* stream);

/* The whole chain (Doppler -> covariance -> weights -> output) for n_probs
 * independent cubes of possibly different shapes, enqueued as one batch
 * (the paper's fused parallel loop over independent units, Sec. 4.2).
 *   cubes[i]   in : x_i as for stap_doppler.
 *   steers[i]  in : V_i[S_i][D_i] (V_i[P_i][S_i][D_i] with steer_per_bin).
 *   powers[i]  out: power_i[P_i][S_i][R_i].
 *   weights    out: NULL, or weights[i] = W_i[P_i][B_i][S_i][D_i] (each may be
 *                   NULL).
 *   info       out: NULL, or info[i] = info_i[P_i][B_i] (each may be NULL).
 *   workspace  scratch device memory of at least stap_workspace_size() bytes,
 *              256-byte aligned; its contents on entry are ignored.
 * All problems must share precision and refine_steps.  With n_probs > 1 and
 * every cube fused-eligible (D <= 128, FP32 or BF16) the batch runs as one
 * Doppler launch per pulse count, then per shape class (DOF class x
 * steering class, largest first) one persistent covariance->solve launch
 * sized for the class, whose workgroups take the class's (cube, bin, block)
 * systems, most expensive first, from a device work queue, and one
 * inner-product launch per class; the problem table (136 bytes per cube,
 * then 24 queue counters of 8 bytes) is written into the
 * workspace by a kernel that carries it in its arguments, and the launch
 * chain is replayed from a cached hipGraph (a stream that is being captured
 * gets the launches directly, table kernel included).  Batches with a cube
 * that is not fused-eligible run cube by cube.  A single cube runs Doppler, the fused covariance->solve
 * (or, where the tuning table selects kind-0 variant 1 or the shape is not
 * fused-eligible, the stage covariance and a stage solve), and the inner
 * products.  Calls that overlap on one workspace race. */
stap_status stap_run(const stap_problem* probs, int32_t n_probs,
                     const stap_cf32* const* cubes,
                     const stap_cf32* const* steers, float* const* powers,
                     stap_cf32* const* weights, int32_t* const* info,
                     void* workspace, size_t workspace_bytes, void* stream);

/* Cell-averaging CFAR parameters (detection on the output power). */
typedef struct stap_cfar_params {
  int32_t n_ref;    /* reference cells per side, 1..64 */
  int32_t n_guard;  /* guard cells per side between the cell and its
                       reference cells, 0..64 */
  double alpha;     /* threshold factor > 0; for N = 2 n_ref reference cells
                       of exponential noise, alpha = N (Pfa^(-1/N) - 1) gives
                       false-alarm probability Pfa */
} stap_cfar_params;

/* Cell-averaging CFAR detection along range on the output power (the
 * textbook CA-CFAR detector, Finn and Johnson 1968, applied to each
 * (Doppler bin, steering vector) row; the step after the paper's kernel).
 * For cell r the reference cells are r-g-n .. r-g-1 and r+g+1 .. r+g+n
 * (n = n_ref, g = n_guard); cells outside [0, R) are left out and n_used
 * counts the rest.  The reference cells are added in FP64 one at a time in
 * that order and the cell is a detection when
 *   (double) power[r] * n_used  >  alpha * sum
 * (FP64, no fused multiply-add), so the mask is reproducible bit for bit.
 *   power  in : power[P][S][R] float as written by stap_run or
 *               stap_inner_products (only P, S and R of prob are used).
 *   detect out: detect[P][S][R] uint8, 1 = detection, 0 = none.
 * STAP_ERR_ARG for a null pointer or parameters out of range. */
stap_status stap_cfar(const stap_problem* prob, const stap_cfar_params* cfar,
                      const float* power, uint8_t* detect, void* stream);

/* Maximum stap_workspace_size() of a stap_run_noalloc call (256 MiB). */
#define STAP_NOALLOC_MAX_BYTES ((size_t)256 << 20)

/* stap_run for callers that cannot allocate device memory: code under graph
 * capture, tight serving loops, hosts whose rules forbid hipMalloc.  Same
 * arguments, layouts, ownership, results and errors as stap_run, without the
 * workspace: the scratch memory (snapshots, and where stap_run would put
 * them the covariance, weights and status) is a fixed array of
 * STAP_NOALLOC_MAX_BYTES in the library's device code, one copy per GPU,
 * held until the process ends.  The call allocates and frees nothing, does
 * not create streams or graphs, and launches the kernels directly on
 * `stream` (several cubes: the batched launch chain, never the cached graph).
 *   Errors: STAP_ERR_WORKSPACE when stap_workspace_size(probs, n_probs)
 *   exceeds STAP_NOALLOC_MAX_BYTES; otherwise as stap_run.
 * Every call on one GPU uses that GPU's one array and leaves its contents
 * behind; nothing in it needs to start at zero.  Calls that overlap in time
 * on the same GPU (several streams or host threads) race on the array and
 * must be serialised by the caller. */
stap_status stap_run_noalloc(const stap_problem* probs, int32_t n_probs,
                             const stap_cf32* const* cubes,
                             const stap_cf32* const* steers,
                             float* const* powers, stap_cf32* const* weights,
                             int32_t* const* info, void* stream);

/* Kernel-variant selection, written by the autotuner (tune.py) and read by
 * stap_run and stap_covariance_solve (kind 0, the fused covariance->solve
 * kernel), by stap_solve_weights and the stage path of stap_run (kind 1),
 * by stap_covariance and the stage path of stap_run (kind 2: waves per
 * system, 4, 8 or 16 where the DOF class offers them, every choice giving
 * the same covariance bit for bit) and by stap_inner_products and the
 * single-cube stap_run (kind 3: 1, 2 or 4 range tiles of 16 cells per wave
 * step, at most 2 on the split-BF16 form; the same output bit for bit).
 * An entry applies to the shape class containing (dof, n_steer): dof classes
 * end at 16, 32, 48, 64, 96, 128, 160, 192 and steering classes at 16, 32, 64.
 * variant: 0 = built-in default;
 *          16 or 32 = column-sweep solve with 16 or 32 rows per register
 *                     slot (a 16 x 16 or 32 x 16 thread grid per system);
 *          4 or 8   = blocked solve on the FP32 matrix cores with 4 or 8
 *                     waves per system (8 runs D > 128 on 16 waves);
 *          1        = one wave per system with every block of the solve in
 *                     its registers (D <= 96, S <= 32): the stage solve
 *                     (kind 1), and for kind 0 a route of single-cube
 *                     stap_run calls through the stage covariance and that
 *                     solve (stap_covariance_solve then takes variant 8).
 *          Requests a variant does not cover take the default. 
 * Not thread-safe with respect to concurrent stap_run calls.  Returns
 * STAP_ERR_ARG for values out of range. */
stap_status stap_tune_set(int32_t kind, int32_t dof, int32_t n_steer, int32_t precision, int32_t refine,
                          int32_t variant);
/* The variant stored for that class (0 = default), or -1 for invalid input. */
int32_t stap_tune_get(int32_t kind, int32_t dof, int32_t n_steer, int32_t precision, int32_t refine);

/* Whether stap_run replays a cached hipGraph of its batched launch chain
 * (n_probs > 1; default on).  Off: the same kernels are launched directly.
 * When the caller's stream is itself being captured the kernels are always
 * launched directly into that capture. */
void stap_use_graphs(int32_t enable);

/* Bytes of device workspace stap_run needs for these problems (per cube:
 * snapshots, weights and info, plus the covariance and delta for D > 128,
 * FP8, or D <= 96 with S <= 32); 0 on invalid
 * arguments. */
size_t stap_workspace_size(const stap_problem* probs, int32_t n_probs);

/* Validate one problem without touching the GPU (host-only check). */
stap_status stap_check_problem(const stap_problem* prob);

/* Static description of a status code. */
const char* stap_status_string(stap_status status);

/* Library version, "major.minor.patch". */
const char* stap_version(void);

#ifdef __cplusplus
}
#endif

#endif /* STAP_H */
