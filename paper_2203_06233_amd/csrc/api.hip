// C ABI of libstap.so: host-side validation, workspace layout and the launch
// sequence of the STAP hot path.  Every argument check happens before the
// first HIP call, so invalid requests return an error without touching the
// device.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "kernels.h"

using stap::Dims;

namespace {

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// Pulse counts with a Doppler kernel: the powers of two 32..512 and the
// paper's 100.
bool valid_pulse(int p) {
  return p == 32 || p == 64 || p == 100 || p == 128 || p == 256 || p == 512;
}
// Array elements per processing channel (0 and 1 both mean none).
int sub_of(const stap_problem* q) { return q->subarray > 1 ? q->subarray : 1; }

stap_status check(const stap_problem* q) {
  if (!q) return STAP_ERR_ARG;
  if (q->subarray < 0) return STAP_ERR_ARG;
  if (q->training != STAP_TRAIN_BLOCK && q->training != STAP_TRAIN_EXCLUDE) return STAP_ERR_ARG;
  if (q->guard_cells < 0 || (q->training == STAP_TRAIN_BLOCK && q->guard_cells != 0)) return STAP_ERR_ARG;
  if (q->tap_phase != STAP_TAP_ABSOLUTE && q->tap_phase != STAP_TAP_RELATIVE) return STAP_ERR_ARG;
  if (q->steer_per_bin != 0 && q->steer_per_bin != 1) return STAP_ERR_ARG;
  if (!(q->load_eps >= 0.f) || !isfinite(q->load_eps)) return STAP_ERR_ARG;
  if (q->precision < STAP_PREC_FP32 || q->precision > STAP_PREC_FP8) return STAP_ERR_ARG;
  if (q->refine_steps < 0 || q->refine_steps > 4) return STAP_ERR_ARG;
  if (q->n_chan < 1 || q->n_range < 1 || q->n_block < 1 || q->n_steer < 1 || q->tdof < 1)
    return STAP_ERR_SHAPE;
  if (!valid_pulse(q->n_pulse)) return STAP_ERR_SHAPE;
  if (q->tdof > stap::kMaxTdof || q->tdof >= q->n_pulse) return STAP_ERR_SHAPE;
  if (q->n_chan % sub_of(q) != 0) return STAP_ERR_SHAPE;
  if ((long long)q->tdof * (q->n_chan / sub_of(q)) > stap::kMaxDof) return STAP_ERR_SHAPE;
  if (q->n_steer > stap::kMaxSteer) return STAP_ERR_SHAPE;
  if (q->n_range % q->n_block != 0) return STAP_ERR_SHAPE;
  if ((long long)q->n_pulse * q->n_block > 0x7fffffffLL) return STAP_ERR_SHAPE;
  // The range rows of the cube must not overlap: channels outermost
  // ([C][P][R], the default) or pulses outermost ([P][C][R], the paper's
  // pulses x channels x samples), each with rows of at least R elements.
  const long long sp = q->cube_stride_pulse ? q->cube_stride_pulse : q->n_range;
  const long long sc = q->cube_stride_chan ? q->cube_stride_chan : (long long)q->n_pulse * sp;
  const bool chan_outer = sp >= q->n_range && (q->n_chan == 1 || sc >= (long long)(q->n_pulse - 1) * sp + q->n_range);
  const bool pulse_outer = sc >= q->n_range && sp >= (long long)(q->n_chan - 1) * sc + q->n_range;
  if (!chan_outer && !pulse_outer) return STAP_ERR_SHAPE;
  if (q->training == STAP_TRAIN_EXCLUDE) {
    // every block needs N training cells outside itself and its guard cells
    const long long N = q->n_range / q->n_block;
    for (long long b = 0; b < q->n_block; ++b) {
      const long long lo = b * N - q->guard_cells, hi = b * N + N + q->guard_cells;
      const long long avail = (lo > 0 ? lo : 0) + (q->n_range - hi > 0 ? q->n_range - hi : 0);
      if (avail < N) return STAP_ERR_SHAPE;
    }
  }
  return STAP_OK;
}

Dims dims_of(const stap_problem* q) {
  Dims d;
  d.sub = sub_of(q);
  d.C = q->n_chan / d.sub;
  d.P = q->n_pulse;
  d.R = q->n_range;
  d.T = q->tdof;
  d.B = q->n_block;
  d.S = q->n_steer;
  d.D = d.T * d.C;
  d.N = d.R / d.B;
  d.L = d.P - d.T + 1;
  d.eps = q->load_eps;
  d.prec = q->precision;
  d.refine = q->refine_steps;
  d.sp = q->cube_stride_pulse ? q->cube_stride_pulse : d.R;
  d.sc = q->cube_stride_chan ? q->cube_stride_chan : (long long)d.P * d.sp;
  d.train = q->training;
  d.guard = q->guard_cells;
  d.tap_rel = q->tap_phase;
  d.steer_bin = q->steer_per_bin;
  return d;
}

// Every validated shape is solvable: D <= 128 on a 16 x 16 thread grid,
// D <= 192 on a 32 x 16 grid.
stap_status check_solvable(const stap_problem* q) {
  return (q->tdof * (q->n_chan / sub_of(q)) > stap::kMaxDof) ? STAP_ERR_UNSUPPORTED : STAP_OK;
}

stap_status hip_status(hipError_t e) { return e == hipSuccess ? STAP_OK : STAP_ERR_HIP; }

// Kernel-variant table written by the autotuner: [kind][dof class][steer
// class][precision][refine] -> variant (0 = built-in default).  Kind 0 is
// the fused covariance -> solve of stap_run, kind 1 the stage weight solve,
// kind 2 the stage covariance (waves per system), kind 3 the inner products
// (range tiles per wave step).
constexpr int kDofClass[] = {16, 32, 48, 64, 96, 128, 160, 192};
constexpr int kSteerClass[] = {16, 32, 64};
constexpr int kKinds = 4;
int8_t g_tune[kKinds][8][3][3][2];
bool valid_variant(int kind, int v) {
  if (kind == 2) return v == 0 || v == 4 || v == 8 || v == 16;
  if (kind == 3) return v == 0 || v == 1 || v == 2 || v == 4;
  return v == 0 || v == 1 || v == 4 || v == 8 || v == 16 || v == 32;
}

int dof_class(int d) {
  for (int i = 0; i < 8; ++i)
    if (d <= kDofClass[i]) return i;
  return -1;
}
int steer_class(int s) {
  for (int i = 0; i < 3; ++i)
    if (s <= kSteerClass[i]) return i;
  return -1;
}
int tuned(int kind, const Dims& d) {
  const int dc = dof_class(d.D), sc = steer_class(d.S);
  if (dc < 0 || sc < 0) return 0;
  return g_tune[kind][dc][sc][d.prec][d.refine > 0 ? 1 : 0];
}
// Variant of the fused covariance -> solve kernel; variant 1 of kind 0 is
// not a fused kernel but stap_run's stage route (one_wave_route()), so the
// fused entry point takes the blocked 8-wave kernel for it.
int fused_variant(const Dims& d) {
  const int v = tuned(0, d);
  return v == 0 ? 16 : v == 1 ? 8 : v;
}
// stap_run on one cube: the stage covariance and the one-wave solve instead
// of the fused kernel, where the table asks for it (kind 0, variant 1) and
// the shape allows.
bool one_wave_route(const Dims& d) { return tuned(0, d) == 1 && stap::wsolve_supported(d); }
// Stage solve: the one-wave register-resident solve (variant 1) or the
// blocked matrix-core solve (variant 4 or 8 waves) where the table asks for
// it and the shape allows, else the column-sweep solve.
hipError_t stage_solve(const Dims& d, const float2* cov, const float2* steer, float2* w, int* info,
                       hipStream_t st) {
  const int v = tuned(1, d);
  if (v == 1 && stap::wsolve_supported(d)) return stap::launch_wsolve(d, cov, steer, w, info, st);
  if ((v == 4 || v == 8) && stap::bsolve_supported(d, v)) return stap::launch_bsolve(d, cov, steer, w, info, st, v);
  return stap::launch_solve(d, cov, steer, w, info, st);
}

constexpr size_t kAlign = 256;
size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Workspace of one cube: snapshots, weights and info (when the caller passes
// none), and the covariance and delta where the fused kernel does not apply
// (D > 128 or FP8) or the one-wave stage route may (D <= 96, S <= 32).
struct Parts {
  size_t snap, cov, delta, w, info;
  size_t total() const { return snap + cov + delta + w + info; }
};
Parts parts_of(const stap_problem* q) {
  const size_t P = q->n_pulse, D = (size_t)q->tdof * (q->n_chan / sub_of(q)), R = q->n_range, B = q->n_block,
               S = q->n_steer;
  const Dims d = dims_of(q);
  const bool fused = stap::fused_supported(d) && !stap::wsolve_supported(d);
  Parts p;
  p.snap = up(P * D * R * 8);
  p.cov = fused ? 0 : up(P * B * D * D * 8);
  p.delta = fused ? 0 : up(P * B * 4);
  p.w = up(P * B * S * D * 8);
  p.info = up(P * B * 4);
  return p;
}
// A batch is split into shape classes (DOF class x steering class), each
// with its own persistent covariance -> solve launch and inner-product
// launch sized for it.  The workspace starts with the problem table, then
// one 8-byte work-queue counter per class.
constexpr int kMaxClasses = 8 * 3;
int shape_class(const Dims& d) { return dof_class(d.D) * 3 + steer_class(d.S); }
size_t table_bytes(int n) {
  return up((size_t)n * sizeof(stap::ProbDesc) + kMaxClasses * sizeof(unsigned long long));
}

// Per-system cost used to order a batch (largest first).
double system_cost(const Dims& d) {
  const double D = d.D, S = d.S, N = d.N;
  return D * D * D / 3.0 + D * D * S + D * D * N / 2.0 + S * D * N;
}

bool g_use_graphs = true;

// hipGraph cache of the batched chain, keyed by device, workspace address
// and every launch parameter.  The graph's kernels read the problem table
// from the workspace, so one graph serves every call with the same shapes.
struct GraphCache {
  std::mutex mu;
  std::map<std::string, hipGraphExec_t> exec;
  std::map<int, hipStream_t> capture_stream;
};
GraphCache& graphs() {
  static GraphCache* g = new GraphCache();  // lives until the process ends
  return *g;
}

// Arguments of a stap_run call, checked on the host before any HIP call.
stap_status check_run(const stap_problem* probs, int32_t n_probs, const stap_cf32* const* cubes,
                      const stap_cf32* const* steers, float* const* powers, stap_cf32* const* weights,
                      int32_t* const* info) {
  if (!probs || n_probs < 1 || !cubes || !steers || !powers) return STAP_ERR_ARG;
  for (int i = 0; i < n_probs; ++i) {
    stap_status s = check(&probs[i]);
    if (s != STAP_OK) return s;
    if ((s = check_solvable(&probs[i])) != STAP_OK) return s;
    if (probs[i].precision != probs[0].precision || probs[i].refine_steps != probs[0].refine_steps)
      return STAP_ERR_ARG;
    if (!cubes[i] || !steers[i] || !powers[i]) return STAP_ERR_ARG;
    if (!aligned(cubes[i], 8) || !aligned(steers[i], 8) || !aligned(powers[i], 4)) return STAP_ERR_ALIGN;
    if (weights && !aligned(weights[i], 8)) return STAP_ERR_ALIGN;
    if (info && !aligned(info[i], 4)) return STAP_ERR_ALIGN;
  }
  return STAP_OK;
}

// The batched problem table reaches the device as kernel arguments (by
// value), so a launch recorded into a graph carries its own copy of the
// table and nothing on the host has to outlive the call.
constexpr int kTableChunk = 3072 / (int)sizeof(stap::ProbDesc);
struct TableChunk {
  int first, n;
  stap::ProbDesc d[kTableChunk];
};
static_assert(sizeof(stap::ProbDesc) % 8 == 0, "table entries are copied as 8-byte words");

// The first chunk's launch also resets the work-queue counters (kernel
// stores, so a captured graph resets them on every replay).
__global__ void table_kernel(stap::ProbDesc* __restrict__ table, TableChunk c, unsigned long long* queue) {
  const int words = c.n * (int)(sizeof(stap::ProbDesc) / 8);
  const unsigned long long* src = reinterpret_cast<const unsigned long long*>(c.d);
  unsigned long long* dst = reinterpret_cast<unsigned long long*>(table + c.first);
  for (int i = threadIdx.x; i < words; i += blockDim.x) dst[i] = src[i];
  if (c.first == 0 && threadIdx.x < kMaxClasses) queue[threadIdx.x] = 0ULL;
}

hipError_t upload_table(stap::ProbDesc* table, const std::vector<stap::ProbDesc>& desc, unsigned long long* queue,
                        hipStream_t st) {
  for (int first = 0; first < (int)desc.size(); first += kTableChunk) {
    TableChunk c;
    c.first = first;
    c.n = std::min(kTableChunk, (int)desc.size() - first);
    for (int i = 0; i < c.n; ++i) c.d[i] = desc[first + i];
    hipLaunchKernelGGL(table_kernel, dim3(1), dim3(256), 0, st, table, c, queue);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Scratch memory of stap_run_noalloc: a fixed-size array in the library's
// device code object, one copy per GPU, held until the process ends.  Host
// code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol); it uses the device address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = STAP_NOALLOC_MAX_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices];

stap_status scratch_of_current_device(char** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return STAP_ERR_HIP;
  if (dev < 0 || dev >= kMaxDevices) return STAP_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return STAP_ERR_HIP;
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return STAP_OK;
}

// stap_run after argument checks: ws0 is a workspace of at least
// stap_workspace_size() bytes.  `graphs_ok` allows the batched chain to be
// replayed from the graph cache (instantiating a graph and creating its
// capture stream allocate, so the no-allocation entry point passes false).
stap_status run_impl(const stap_problem* probs, int32_t n_probs, const stap_cf32* const* cubes,
                     const stap_cf32* const* steers, float* const* powers, stap_cf32* const* weights,
                     int32_t* const* info, char* const ws0, hipStream_t st, bool graphs_ok) {
  stap::ProbDesc* table = reinterpret_cast<stap::ProbDesc*>(ws0);
  unsigned long long* queue = reinterpret_cast<unsigned long long*>(ws0 + (size_t)n_probs * sizeof(stap::ProbDesc));
  char* ws = ws0 + table_bytes(n_probs);
  std::vector<stap::ProbDesc> desc(n_probs);
  bool all_fused = true;
  for (int i = 0; i < n_probs; ++i) {
    const Dims d = dims_of(&probs[i]);
    const Parts p = parts_of(&probs[i]);
    stap::ProbDesc& pd = desc[i];
    pd.d = d;
    pd.cube = reinterpret_cast<const float2*>(cubes[i]);
    pd.steer = reinterpret_cast<const float2*>(steers[i]);
    pd.power = powers[i];
    pd.snap = reinterpret_cast<float2*>(ws);
    pd.w = reinterpret_cast<float2*>(ws + p.snap + p.cov + p.delta);
    pd.info = reinterpret_cast<int*>(ws + p.snap + p.cov + p.delta + p.w);
    ws += p.total();
    if (weights && weights[i]) pd.w = reinterpret_cast<float2*>(weights[i]);
    if (info && info[i]) pd.info = info[i];
    pd.sys_begin = 0;
    all_fused = all_fused && stap::fused_supported(d);
  }

  if (n_probs == 1 || !all_fused) {
    char* wsp = ws0 + table_bytes(n_probs);
    for (int i = 0; i < n_probs; ++i) {
      const stap::ProbDesc& pd = desc[i];
      const Dims& d = pd.d;
      const Parts p = parts_of(&probs[i]);
      float2* cov = reinterpret_cast<float2*>(wsp + p.snap);
      float* delta = reinterpret_cast<float*>(wsp + p.snap + p.cov);
      wsp += p.total();
      hipError_t e = stap::launch_doppler(d, pd.cube, pd.snap, st);
      if (one_wave_route(d)) {
        if (e == hipSuccess) e = stap::launch_covariance(d, pd.snap, cov, delta, st, tuned(2, d));
        if (e == hipSuccess) e = stap::launch_wsolve(d, cov, pd.steer, pd.w, pd.info, st);
      } else if (stap::fused_supported(d)) {
        if (e == hipSuccess) e = stap::launch_fused(d, pd.snap, pd.steer, pd.w, pd.info, st, fused_variant(d));
      } else {
        if (e == hipSuccess) e = stap::launch_covariance(d, pd.snap, cov, delta, st, tuned(2, d));
        if (e == hipSuccess) e = stage_solve(d, cov, pd.steer, pd.w, pd.info, st);
      }
      if (e == hipSuccess) e = stap::launch_inner(d, pd.w, pd.snap, pd.power, nullptr, st, tuned(3, d));
      if (e != hipSuccess) return STAP_ERR_HIP;
    }
    return STAP_OK;
  }

  // Batched: group the cubes by shape class (largest class first), order
  // each class by per-system cost, number its systems, upload the table.
  std::stable_sort(desc.begin(), desc.end(), [](const stap::ProbDesc& a, const stap::ProbDesc& b) {
    const int ka = shape_class(a.d), kb = shape_class(b.d);
    if (ka != kb) return ka > kb;
    return system_cost(a.d) > system_cost(b.d);
  });
  struct Group {
    int lo, n, key;
    long long total;
    int max_dof, max_steer, ty;
  };
  std::vector<Group> groups;
  for (int i = 0; i < n_probs; ++i) {
    stap::ProbDesc& pd = desc[i];
    const int key = shape_class(pd.d);
    if (groups.empty() || groups.back().key != key) groups.push_back(Group{i, 0, key, 0, 0, 0, 0});
    Group& g = groups.back();
    pd.sys_begin = g.total;
    g.total += (long long)pd.d.P * pd.d.B;
    g.max_dof = std::max(g.max_dof, pd.d.D);
    g.max_steer = std::max(g.max_steer, pd.d.S);
    ++g.n;
  }
  for (Group& g : groups) {
    Dims cls = desc[g.lo].d;
    cls.D = g.max_dof;
    cls.S = g.max_steer;
    g.ty = fused_variant(cls);
  }
  const int prec = probs[0].precision, refine = probs[0].refine_steps;

  // Doppler launches, one per pulse count (at most kMaxBatchArg cubes each).
  std::vector<std::pair<stap::BatchIndex, int>> dop;
  for (int P : {32, 64, 100, 128, 256, 512}) {
    stap::BatchIndex bi;
    bi.n = 0;
    int tiles = 0;
    for (int i = 0; i < n_probs; ++i) {
      if (desc[i].d.P != P) continue;
      if (bi.n == stap::kMaxBatchArg) {
        bi.tile_begin[bi.n] = tiles;
        dop.push_back({bi, P});
        bi.n = 0;
        tiles = 0;
      }
      bi.prob[bi.n] = i;
      bi.tile_begin[bi.n] = tiles;
      tiles += stap::doppler_tiles(desc[i].d);
      ++bi.n;
    }
    if (bi.n > 0) {
      bi.tile_begin[bi.n] = tiles;
      dop.push_back({bi, P});
    }
  }
  auto enqueue = [&](hipStream_t s) -> hipError_t {
    for (auto& x : dop) {
      hipError_t e = stap::launch_doppler_batched(x.second, table, x.first, x.first.tile_begin[x.first.n], s);
      if (e != hipSuccess) return e;
    }
    for (size_t i = 0; i < groups.size(); ++i) {
      const Group& g = groups[i];
      const hipError_t e = stap::launch_fused_batched(table + g.lo, g.n, g.total, g.max_dof, g.max_steer, prec, refine,
                                                      g.ty, s, queue + i);
      if (e != hipSuccess) return e;
    }
    for (const Group& g : groups) {
      const hipError_t e = stap::launch_inner_batched(table + g.lo, g.n, g.total, g.max_dof, g.max_steer, prec, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };

  if (upload_table(table, desc, queue, st) != hipSuccess) return STAP_ERR_HIP;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cap) != hipSuccess) return STAP_ERR_HIP;
  if (!graphs_ok || !g_use_graphs || cap != hipStreamCaptureStatusNone) return hip_status(enqueue(st));

  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return STAP_ERR_HIP;
  std::string key = std::to_string(dev) + "|" + std::to_string((uintptr_t)ws0) + "|" +
                    std::to_string(prec) + "|" + std::to_string(refine);
  for (const Group& g : groups) key += "|v" + std::to_string(g.ty);
  for (auto& pd : desc) {
    key += "|" + std::to_string(pd.d.C) + "," + std::to_string(pd.d.P) + "," + std::to_string(pd.d.R) + "," +
           std::to_string(pd.d.T) + "," + std::to_string(pd.d.B) + "," + std::to_string(pd.d.S);
  }
  GraphCache& gc = graphs();
  std::lock_guard<std::mutex> lock(gc.mu);
  auto it = gc.exec.find(key);
  if (it == gc.exec.end()) {
    hipStream_t cs;
    auto sit = gc.capture_stream.find(dev);
    if (sit == gc.capture_stream.end()) {
      if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return STAP_ERR_HIP;
      gc.capture_stream[dev] = cs;
    } else {
      cs = sit->second;
    }
    hipGraph_t graph;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return STAP_ERR_HIP;
    const hipError_t e = enqueue(cs);
    const hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (e != hipSuccess || e2 != hipSuccess) return STAP_ERR_HIP;
    hipGraphExec_t ge;
    const hipError_t e3 = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e3 != hipSuccess) return STAP_ERR_HIP;
    it = gc.exec.emplace(key, ge).first;
  }
  return hip_status(hipGraphLaunch(it->second, st));
}

}  // namespace

extern "C" {

stap_status stap_check_problem(const stap_problem* prob) { return check(prob); }

stap_status stap_doppler(const stap_problem* prob, const stap_cf32* cube, stap_cf32* snap, void* stream) {
  stap_status s = check(prob);
  if (s != STAP_OK) return s;
  if (!cube || !snap) return STAP_ERR_ARG;
  if (!aligned(cube, 8) || !aligned(snap, 8)) return STAP_ERR_ALIGN;
  const Dims d = dims_of(prob);
  return hip_status(stap::launch_doppler(d, reinterpret_cast<const float2*>(cube),
                                         reinterpret_cast<float2*>(snap), (hipStream_t)stream));
}

stap_status stap_covariance(const stap_problem* prob, const stap_cf32* snap, stap_cf32* cov, float* delta,
                            void* stream) {
  stap_status s = check(prob);
  if (s != STAP_OK) return s;
  if (!snap || !cov) return STAP_ERR_ARG;
  if (!aligned(snap, 8) || !aligned(cov, 8) || !aligned(delta, 4)) return STAP_ERR_ALIGN;
  const Dims d = dims_of(prob);
  return hip_status(stap::launch_covariance(d, reinterpret_cast<const float2*>(snap),
                                            reinterpret_cast<float2*>(cov), delta, (hipStream_t)stream,
                                            tuned(2, d)));
}

stap_status stap_solve_weights(const stap_problem* prob, const stap_cf32* cov, const stap_cf32* steer,
                               stap_cf32* w, int32_t* info, void* stream) {
  stap_status s = check(prob);
  if (s != STAP_OK) return s;
  if (!cov || !steer || !w || !info) return STAP_ERR_ARG;
  if (!aligned(cov, 8) || !aligned(steer, 8) || !aligned(w, 8) || !aligned(info, 4)) return STAP_ERR_ALIGN;
  if ((s = check_solvable(prob)) != STAP_OK) return s;
  const Dims d = dims_of(prob);
  return hip_status(stage_solve(d, reinterpret_cast<const float2*>(cov), reinterpret_cast<const float2*>(steer),
                                 reinterpret_cast<float2*>(w), info, (hipStream_t)stream));
}

stap_status stap_covariance_solve(const stap_problem* prob, const stap_cf32* snap, const stap_cf32* steer,
                                  stap_cf32* w, int32_t* info, void* stream) {
  stap_status s = check(prob);
  if (s != STAP_OK) return s;
  if (!snap || !steer || !w || !info) return STAP_ERR_ARG;
  if (!aligned(snap, 8) || !aligned(steer, 8) || !aligned(w, 8) || !aligned(info, 4)) return STAP_ERR_ALIGN;
  const Dims d = dims_of(prob);
  if (!stap::fused_supported(d)) return STAP_ERR_UNSUPPORTED;
  return hip_status(stap::launch_fused(d, reinterpret_cast<const float2*>(snap), reinterpret_cast<const float2*>(steer),
                                       reinterpret_cast<float2*>(w), info, (hipStream_t)stream, fused_variant(d)));
}

stap_status stap_inner_products(const stap_problem* prob, const stap_cf32* w, const stap_cf32* snap,
                                float* power, stap_cf32* y, void* stream) {
  stap_status s = check(prob);
  if (s != STAP_OK) return s;
  if (!w || !snap || !power) return STAP_ERR_ARG;
  if (!aligned(w, 8) || !aligned(snap, 8) || !aligned(power, 4) || !aligned(y, 8)) return STAP_ERR_ALIGN;
  const Dims d = dims_of(prob);
  return hip_status(stap::launch_inner(d, reinterpret_cast<const float2*>(w),
                                       reinterpret_cast<const float2*>(snap), power,
                                       reinterpret_cast<float2*>(y), (hipStream_t)stream, tuned(3, d)));
}

stap_status stap_cfar(const stap_problem* prob, const stap_cfar_params* cfar, const float* power, uint8_t* detect,
                      void* stream) {
  stap_status s = check(prob);
  if (s != STAP_OK) return s;
  if (!cfar || !power || !detect) return STAP_ERR_ARG;
  if (cfar->n_ref < 1 || cfar->n_ref > stap::kMaxCfarRef || cfar->n_guard < 0 || cfar->n_guard > stap::kMaxCfarGuard)
    return STAP_ERR_ARG;
  if (!(cfar->alpha > 0.0) || !isfinite(cfar->alpha)) return STAP_ERR_ARG;
  if (!aligned(power, 4)) return STAP_ERR_ALIGN;
  const Dims d = dims_of(prob);
  return hip_status(stap::launch_cfar(d, cfar->n_ref, cfar->n_guard, cfar->alpha, power, detect, (hipStream_t)stream));
}

size_t stap_workspace_size(const stap_problem* probs, int32_t n_probs) {
  if (!probs || n_probs < 1) return 0;
  size_t total = table_bytes(n_probs);
  for (int i = 0; i < n_probs; ++i) {
    if (check(&probs[i]) != STAP_OK) return 0;
    total += parts_of(&probs[i]).total();
  }
  return total;
}

stap_status stap_run(const stap_problem* probs, int32_t n_probs, const stap_cf32* const* cubes,
                     const stap_cf32* const* steers, float* const* powers, stap_cf32* const* weights,
                     int32_t* const* info, void* workspace, size_t workspace_bytes, void* stream) {
  stap_status s = check_run(probs, n_probs, cubes, steers, powers, weights, info);
  if (s != STAP_OK) return s;
  const size_t need = stap_workspace_size(probs, n_probs);
  if (!workspace || workspace_bytes < need) return STAP_ERR_WORKSPACE;
  if (!aligned(workspace, kAlign)) return STAP_ERR_ALIGN;
  return run_impl(probs, n_probs, cubes, steers, powers, weights, info, static_cast<char*>(workspace),
                  (hipStream_t)stream, true);
}

stap_status stap_run_noalloc(const stap_problem* probs, int32_t n_probs, const stap_cf32* const* cubes,
                             const stap_cf32* const* steers, float* const* powers, stap_cf32* const* weights,
                             int32_t* const* info, void* stream) {
  stap_status s = check_run(probs, n_probs, cubes, steers, powers, weights, info);
  if (s != STAP_OK) return s;
  if (stap_workspace_size(probs, n_probs) > kScratchBytes) return STAP_ERR_WORKSPACE;
  char* ws = nullptr;
  if ((s = scratch_of_current_device(&ws)) != STAP_OK) return s;
  return run_impl(probs, n_probs, cubes, steers, powers, weights, info, ws, (hipStream_t)stream, false);
}

void stap_use_graphs(int32_t enable) { g_use_graphs = enable != 0; }

const char* stap_status_string(stap_status status) {
  switch (status) {
    case STAP_OK: return "ok";
    case STAP_ERR_ARG: return "invalid argument (null pointer or value out of range)";
    case STAP_ERR_SHAPE: return "dimensions outside the supported limits";
    case STAP_ERR_ALIGN: return "misaligned device pointer";
    case STAP_ERR_WORKSPACE: return "workspace missing or too small";
    case STAP_ERR_HIP: return "HIP runtime error";
    case STAP_ERR_UNSUPPORTED: return "request not supported by the library";
  }
  return "unknown status";
}

stap_status stap_tune_set(int32_t kind, int32_t dof, int32_t n_steer, int32_t precision, int32_t refine,
                          int32_t variant) {
  const int dc = dof_class(dof), sc = steer_class(n_steer);
  if (kind < 0 || kind >= kKinds || dc < 0 || sc < 0 || precision < 0 || precision > 2 || refine < 0)
    return STAP_ERR_ARG;
  if (!valid_variant(kind, variant)) return STAP_ERR_ARG;
  g_tune[kind][dc][sc][precision][refine > 0 ? 1 : 0] = (int8_t)variant;
  return STAP_OK;
}

int32_t stap_tune_get(int32_t kind, int32_t dof, int32_t n_steer, int32_t precision, int32_t refine) {
  const int dc = dof_class(dof), sc = steer_class(n_steer);
  if (kind < 0 || kind >= kKinds || dc < 0 || sc < 0 || precision < 0 || precision > 2 || refine < 0) return -1;
  return g_tune[kind][dc][sc][precision][refine > 0 ? 1 : 0];
}

const char* stap_version(void) { return "0.2.0"; }

}  // extern "C"
