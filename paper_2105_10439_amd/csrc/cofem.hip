// Host driver of the CoFEM hot path and its C ABI (include/cofem.h).
//
// One context = one problem shape on one device and one stream.  The driver
// runs Algorithm 1 on the host side of the boundary and keeps every vector,
// every CG scalar and the stop decision on the device: the host only enqueues
// fixed chunks of CG steps and reads back one small state record per chunk;
// steps enqueued after the stop rule fired are no-ops on the device.
#include "cofem.h"
#include "kernels.h"
#include "mt_batch.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#define COFEM_API extern "C" __attribute__((visibility("default")))

using namespace cofem;

namespace {

thread_local std::string g_err;

cofem_status fail(cofem_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

}  // namespace

void cofem::set_error(const std::string& msg) { g_err = msg; }

namespace {

#define HIP_TRY(expr)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return fail(COFEM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

inline int64_t round_up(int64_t x, int64_t m) { return ((x + m - 1) / m) * m; }

uint64_t mix64_host(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct TimedLaunch {
  hipEvent_t a, b;
  int which;      // 0 = FP32 operator, 1 = bf16 operator
  int step;       // CG step index within the chunk
};

}  // namespace

struct cofem_ctx {
  cofem_params p{};
  hipStream_t stream = nullptr;
  int device = 0;
  int64_t Np = 0, Dp = 0;
  int Q = 0, Qp = 0;
  bool need32 = false, need16 = false;
  bool dict_loaded = false;
  bool fitted = false;
  // dictionary layouts
  float* phi32 = nullptr;
  float* phi32T = nullptr;
  uint16_t* phi16 = nullptr;
  uint16_t* phi16T = nullptr;
  // convolutional dictionary: padded taps (FP32 and bfloat16)
  float* hp32 = nullptr;
  uint16_t* hp16 = nullptr;
  // subsampled DCT dictionary: transform tables, mask, kept samples, scratch signal
  float2 *dct_tw = nullptr, *dct_w2 = nullptr, *dct_mz = nullptr;
  float2 *dct_mzt = nullptr, *dct_y1 = nullptr, *dct_y2 = nullptr;  // split operator (null: one workgroup per column)
  int probe_mode = COFEM_PROBES_HASH;
  int estep_prev = 0;  // CG steps of the running E-step already harvested
  int32_t* dct_rows = nullptr;
  float* dct_u = nullptr;
  // D- and N-vectors
  float *theta = nullptr, *alpha = nullptr, *alpha_hook = nullptr, *b32 = nullptr, *b16 = nullptr;
  float* minv = nullptr;
  float *mu = nullptr, *s = nullptr, *yv = nullptr;
  // post-fit variance: running sum, one batch's estimate and mean
  float *var_sum = nullptr, *var_s = nullptr, *var_mu = nullptr;
  // CG blocks
  float *X = nullptr, *R = nullptr, *Pd = nullptr, *Psi = nullptr, *V = nullptr;
  uint16_t *PdH = nullptr, *PdL = nullptr, *VH = nullptr, *VL = nullptr;
  uint16_t *PdX = nullptr, *VX = nullptr;  // third slices of Pd and V for the FP32 dense operator
  float* Ypart = nullptr;
  double* part = nullptr;    // em_init partials and CG-update partials
  double* pipart = nullptr;  // pi partials
  CGState* st = nullptr;
  CGState* h_st = nullptr;  // pinned host mirror
  GemmCfg g1_16{}, g2_16{}, g1_32{}, g2_32{};
  int chunk = 8;
  // A chunk of CG steps captured once as a graph per operator phase (bf16 or FP32) and
  // alpha buffer, replayed on `stream` (launch latency dominates small problems).  The
  // capture runs on cap_stream: the caller's stream may be the legacy default stream,
  // which cannot be captured.  Not used while operator timing is on.
  struct ChunkGraph {
    hipGraphExec_t exec = nullptr;
    const float* alpha = nullptr;
  } graphs[2];
  hipStream_t cap_stream = nullptr;
  bool graph_off = false;  // a capture failed: eager launches from then on
  cofem_stats stats{};
  // operator timing
  bool timing = false;
  double t_ms[2] = {0, 0};
  int64_t t_n[2] = {0, 0};
  std::vector<hipEvent_t> ev_pool;
  std::vector<TimedLaunch> pending;
  std::vector<void*> allocs;
};

namespace {

template <class T>
cofem_status dalloc(cofem_ctx* c, T** out, size_t n) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(COFEM_ENOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed: " +
                                  hipGetErrorString(e));
  }
  c->allocs.push_back(p);
  *out = static_cast<T*>(p);
  return COFEM_OK;
}

void free_all(cofem_ctx* c) {
  for (auto& g : c->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
  }
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  c->cap_stream = nullptr;
  for (void* p : c->allocs) (void)hipFree(p);
  c->allocs.clear();
  if (c->h_st) (void)hipHostFree(c->h_st);
  c->h_st = nullptr;
  for (auto& t : c->pending) {
    c->ev_pool.push_back(t.a);
    c->ev_pool.push_back(t.b);
  }
  c->pending.clear();
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  c->ev_pool.clear();
}

cofem_status validate(const cofem_params* p) {
  if (!p) return fail(COFEM_EINVAL, "params is NULL");
  if (p->N < 1 || p->D < 1) return fail(COFEM_EINVAL, "N and D must be >= 1");
  if (p->N > (int64_t(1) << 31) || p->D > (int64_t(1) << 31)) return fail(COFEM_EINVAL, "N or D too large");
  if (!(p->beta > 0.0) || !std::isfinite(p->beta)) return fail(COFEM_EINVAL, "beta must be finite and > 0");
  if (p->K < 1 || p->K > COFEM_MAX_K) return fail(COFEM_EINVAL, "K must be in [1, COFEM_MAX_K]");
  if (p->T < 1 || p->T > COFEM_MAX_T) return fail(COFEM_EINVAL, "T must be in [1, COFEM_MAX_T]");
  if (p->U < 1) return fail(COFEM_EINVAL, "U must be >= 1");
  if (!(p->tol >= 0.0) || !std::isfinite(p->tol)) return fail(COFEM_EINVAL, "tol must be finite and >= 0");
  if (p->theta_mode != COFEM_THETA_ONES && p->theta_mode != COFEM_THETA_JACOBI)
    return fail(COFEM_EINVAL, "bad theta_mode");
  if (p->stop_mode != COFEM_STOP_JOINT && p->stop_mode != COFEM_STOP_COLUMN)
    return fail(COFEM_EINVAL, "bad stop_mode");
  if (p->phi_dtype != COFEM_PHI_FP32 && p->phi_dtype != COFEM_PHI_BF16) return fail(COFEM_EINVAL, "bad phi_dtype");
  if (p->refine_last < 0 || p->refine_last > p->T) return fail(COFEM_EINVAL, "refine_last must be in [0, T]");
  if (!(p->alpha_floor > 0.0) || !std::isfinite(p->alpha_floor))
    return fail(COFEM_EINVAL, "alpha_floor must be finite and > 0");
  if (p->mstep_mode != COFEM_MSTEP_GAUSSIAN && p->mstep_mode != COFEM_MSTEP_NONNEG)
    return fail(COFEM_EINVAL, "bad mstep_mode");
  if (p->op_kind == COFEM_OP_CONV) {
    if (p->N != p->D) return fail(COFEM_EINVAL, "COFEM_OP_CONV needs N == D");
    if (p->conv_taps < 1 || p->conv_taps > CONV_MAX_TAPS)
      return fail(COFEM_EINVAL, "conv_taps must be in [1, " + std::to_string(CONV_MAX_TAPS) + "]");
  } else if (p->op_kind == COFEM_OP_DCT) {
    if (!dct_size_ok(p->D))
      return fail(COFEM_EINVAL, "COFEM_OP_DCT needs D a power of two in [" + std::to_string(DCT_MIN_D) + ", " +
                                    std::to_string(DCT_MAX_D) + "]");
    if (p->N > p->D) return fail(COFEM_EINVAL, "COFEM_OP_DCT needs N <= D");
    if (p->phi_dtype != COFEM_PHI_FP32) return fail(COFEM_EINVAL, "COFEM_OP_DCT runs in FP32 (phi_dtype)");
  } else if (p->op_kind != COFEM_OP_DENSE) {
    return fail(COFEM_EINVAL, "bad op_kind");
  }
  return COFEM_OK;
}

SolveCfg solve_cfg(const cofem_ctx* c) {
  SolveCfg s;
  s.Q = c->Q;
  s.Qp = c->Qp;
  s.K = c->p.K;
  s.U = c->p.U;
  s.stop_mode = c->p.stop_mode;
  s.nonneg = c->p.mstep_mode == COFEM_MSTEP_NONNEG ? 1 : 0;
  s.tol = c->p.tol;
  s.beta = c->p.beta;
  s.hadamard = c->probe_mode;
  s.sigblk = c->p.op_kind == COFEM_OP_CONV ? 1 : 0;
  s.nt_store = c->p.op_kind == COFEM_OP_DCT ? 0 : 1;
  return s;
}

cofem_status timed_begin(cofem_ctx* c, int which, int step, TimedLaunch* t) {
  t->which = which;
  t->step = step;
  for (int i = 0; i < 2; ++i) {
    hipEvent_t e;
    if (!c->ev_pool.empty()) {
      e = c->ev_pool.back();
      c->ev_pool.pop_back();
    } else {
      HIP_TRY(hipEventCreate(&e));
    }
    (i == 0 ? t->a : t->b) = e;
  }
  HIP_TRY(hipEventRecord(t->a, c->stream));
  return COFEM_OK;
}

cofem_status timed_end(cofem_ctx* c, TimedLaunch* t) {
  HIP_TRY(hipEventRecord(t->b, c->stream));
  c->pending.push_back(*t);
  return COFEM_OK;
}

// Called after a stream sync: accumulate the launches of the first `real_steps`
// steps of the chunk (later ones were no-ops after the stop rule fired).
cofem_status harvest(cofem_ctx* c, int real_steps) {
  for (auto& t : c->pending) {
    if (t.step < real_steps) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, t.a, t.b));
      c->t_ms[t.which] += ms;
      c->t_n[t.which] += 1;
    }
    c->ev_pool.push_back(t.a);
    c->ev_pool.push_back(t.b);
  }
  c->pending.clear();
  return COFEM_OK;
}

// Psi = A Pd into c->Psi and pi into the state, for the given alpha buffer.
// The two filter passes of the convolutional dictionary (pass 2 fuses the finish).
DctArgs dct_args(const cofem_ctx* c) {
  DctArgs a{};
  a.D = c->p.D;
  a.Dp = c->Dp;
  a.nbx = (int)((c->Dp + 1023) / 1024);
  a.s0 = (float)std::sqrt(1.0 / (double)c->p.D);
  a.s1 = (float)std::sqrt(2.0 / (double)c->p.D);
  a.tw = c->dct_tw;
  a.mz = c->dct_mz;
  a.w2 = c->dct_w2;
  a.mzt = c->dct_mzt;
  a.y1 = c->dct_y1;
  a.y2 = c->dct_y2;
  a.beta = c->p.beta;
  return a;
}

// The DCT operator: three launches over several workgroups per column where the split
// form exists, else one launch with one workgroup per column (the transforms in LDS).
cofem_status apply_dct(cofem_ctx* c, const float* alpha, const SolveCfg& sc, int step) {
  DctArgs a = dct_args(c);
  a.in = c->Pd;
  a.out = c->Psi;
  a.alpha = alpha;
  a.pipart = c->pipart;
  a.done = &c->st->done;
  TimedLaunch t;
  cofem_status rc;
  if (c->timing && (rc = timed_begin(c, 0, step, &t)) != COFEM_OK) return rc;
  launch_dct_operator(a, sc.Q, c->stream);
  if (c->timing && (rc = timed_end(c, &t)) != COFEM_OK) return rc;
  return COFEM_OK;
}

// The FIR operator: bf16, both filters in one launch with V kept in registers; FP32,
// the two filter passes with V through memory (conv.hip).
cofem_status apply_conv(cofem_ctx* c, bool use16, const float* alpha, const SolveCfg& sc, int step) {
  ConvArgs a{};
  a.hp32 = c->hp32;
  a.hp16 = c->hp16;
  a.L = c->p.conv_taps;
  a.D = c->p.D;
  a.Dp = c->Dp;
  a.Q = sc.Q;
  a.nct = (sc.Q + 15) / 16;
  a.nbx = (int)((c->Dp + 1023) / 1024);
  a.beta = sc.beta;
  a.done = &c->st->done;
  a.out32 = c->Psi;
  a.alpha = alpha;
  a.pipart = c->pipart;
  TimedLaunch t;
  cofem_status rc;
  if (use16) {  // the bf16 form carries Pd as its hi/lo pair
    a.xclear = &c->st->xpend;
    a.inH = c->PdH;
    a.inL = c->PdL;
    if (c->timing && (rc = timed_begin(c, 1, step, &t)) != COFEM_OK) return rc;
    launch_conv_op_bf16(a, c->stream);
    if (c->timing && (rc = timed_end(c, &t)) != COFEM_OK) return rc;
    return COFEM_OK;
  }
  ConvArgs p1 = a;
  p1.in32 = c->Pd;
  p1.out32 = c->V;
  a.in32 = c->V;
  a.Pd = c->Pd;
  if (c->timing && (rc = timed_begin(c, 0, step, &t)) != COFEM_OK) return rc;
  launch_conv_pass(p1, 0, c->stream);
  if (c->timing && (rc = timed_end(c, &t)) != COFEM_OK) return rc;
  if (c->timing && (rc = timed_begin(c, 0, step, &t)) != COFEM_OK) return rc;
  launch_conv_pass(a, 1, c->stream);
  if (c->timing && (rc = timed_end(c, &t)) != COFEM_OK) return rc;
  return COFEM_OK;
}

cofem_status apply_operator(cofem_ctx* c, bool use16, const float* alpha, const SolveCfg& sc, int step) {
  if (c->p.op_kind == COFEM_OP_CONV) return apply_conv(c, use16, alpha, sc, step);
  if (c->p.op_kind == COFEM_OP_DCT) return apply_dct(c, alpha, sc, step);
  TimedLaunch t;
  cofem_status rc;
  if (use16) {
    if (c->timing && (rc = timed_begin(c, 1, step, &t)) != COFEM_OK) return rc;
    launch_gemm_bf16(c->g1_16, c->phi16, c->g1_16.kchunk, c->Np * c->g1_16.kchunk, c->Np, c->Dp, c->PdH, c->PdL, sc.Q,
                     c->Qp, c->Ypart, c->st, c->stream);
    if (c->timing && (rc = timed_end(c, &t)) != COFEM_OK) return rc;
    launch_finish_pass1(c->Ypart, c->g1_16.splits, sc.Q, c->Qp, c->Np, nullptr, c->VH, c->VL, c->st, c->stream);
    if (c->timing && (rc = timed_begin(c, 1, step, &t)) != COFEM_OK) return rc;
    launch_gemm_bf16(c->g2_16, c->phi16T, dict_ld(c->Np, 2), 0, c->Dp, c->Np, c->VH, c->VL, sc.Q, c->Qp, c->Ypart,
                     c->st, c->stream);
    if (c->timing && (rc = timed_end(c, &t)) != COFEM_OK) return rc;
    launch_finish_pass2(sc, c->Ypart, c->g2_16.splits, c->Dp, alpha, c->Pd, c->Psi, c->pipart, c->st, c->stream);
  } else {
    if (c->timing && (rc = timed_begin(c, 0, step, &t)) != COFEM_OK) return rc;
    launch_gemm_f32(c->g1_32, c->phi32, c->Np, c->Dp, c->PdH, c->PdL, c->PdX, sc.Q, c->Qp, c->Ypart, c->st,
                    c->stream);
    if (c->timing && (rc = timed_end(c, &t)) != COFEM_OK) return rc;
    launch_finish_pass1(c->Ypart, c->g1_32.splits, sc.Q, c->Qp, c->Np, nullptr, c->VH, c->VL, c->st, c->stream,
                        c->VX);
    if (c->timing && (rc = timed_begin(c, 0, step, &t)) != COFEM_OK) return rc;
    launch_gemm_f32(c->g2_32, c->phi32T, c->Dp, c->Np, c->VH, c->VL, c->VX, sc.Q, c->Qp, c->Ypart, c->st,
                    c->stream);
    if (c->timing && (rc = timed_end(c, &t)) != COFEM_OK) return rc;
    launch_finish_pass2(sc, c->Ypart, c->g2_32.splits, c->Dp, alpha, c->Pd, c->Psi, c->pipart, c->st, c->stream);
  }
  return COFEM_OK;
}

cofem_status sync_state(cofem_ctx* c) {
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(c->h_st, c->st, sizeof(CGState), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return COFEM_OK;
}

uint64_t estep_key(const cofem_ctx* c, int t) { return mix64_host(c->p.seed + (uint64_t)t * GOLDEN_GAMMA); }

// Start of a fit: stats, CG state, y padded, and b = beta Phi^T y for each phase's operator.
void begin_fit(cofem_ctx* c, const float* y) {
  const cofem_params& p = c->p;
  const double ms_setup = c->stats.ms_setup;
  std::memset(&c->stats, 0, sizeof(c->stats));
  c->stats.ms_setup = ms_setup;
  c->fitted = false;
  launch_state_reset(c->st, c->Q, c->stream);
  launch_copy_pad(y, p.N, c->Np, 0.0f, c->yv, c->stream);
  launch_count_nonfinite(y, p.N, &c->st->nonfinite, c->stream);
  // b = beta Phi^T y, formed with the same dictionary as the operator of each phase: the
  // rounding residual of an FP32 b is not in the range of the bf16 Phi^T, and EM would
  // amplify it through the directions that only diag(alpha) constrains.
  if (p.op_kind == COFEM_OP_DCT) {
    DctArgs a = dct_args(c);
    a.out = c->b32;
    launch_dct_rhs(a, c->yv, c->dct_rows, p.N, c->dct_u, c->stream);
  } else if (p.op_kind == COFEM_OP_CONV) {
    if (c->need32) launch_conv_rhs(c->hp32, nullptr, p.conv_taps, p.D, c->Dp, c->yv, p.beta, c->b32, c->stream);
    if (c->need16) launch_conv_rhs(c->hp32, c->hp16, p.conv_taps, p.D, c->Dp, c->yv, p.beta, c->b16, c->stream);
  } else {
    if (c->need32) launch_rhs(c->phi32T, nullptr, dict_ld(c->Np, 4), c->Np, c->Dp, c->yv, p.beta, c->b32, c->stream);
    if (c->need16) launch_rhs(nullptr, c->phi16T, dict_ld(c->Np, 2), c->Np, c->Dp, c->yv, p.beta, c->b16, c->stream);
  }
}

// After an input was counted into the state (begin_fit, set_dictionary): COFEM_EINVAL if
// it holds a NaN or an infinity, before any EM work uses it.
cofem_status check_finite(cofem_ctx* c, const char* what) {
  cofem_status rc = sync_state(c);
  if (rc != COFEM_OK) return rc;
  if (c->h_st->nonfinite > 0)
    return fail(COFEM_EINVAL, std::string(what) + " has " + std::to_string(c->h_st->nonfinite) +
                                  " non-finite entries (NaN or infinity)");
  return COFEM_OK;
}

// Slices of Pd the producers write: hi/lo for the bf16 operator, hi/lo and the third
// slice for the dense FP32 one (which takes its right-hand sides as three bf16 slices).
struct PdSlices {
  uint16_t *H, *L, *X;
};
PdSlices pd_slices(const cofem_ctx* c, bool use16) {
  const bool sliced32 = !use16 && c->PdX;
  return PdSlices{(use16 || sliced32) ? c->PdH : nullptr, (use16 || sliced32) ? c->PdL : nullptr,
                  sliced32 ? c->PdX : nullptr};
}

// One E-step (Algorithm 1) in three parts, so that several contexts can interleave:
// estep_begin draws the probes of iteration key `key` and sets up B and the PCG of
// Algorithm 2 at the given alpha; estep_chunk enqueues c->chunk CG steps (those past the
// device-side stop rule return at once); estep_poll waits for them and reports whether
// the stop rule has fired.
void estep_begin(cofem_ctx* c, uint64_t key, bool use16, const float* alpha) {
  const SolveCfg sc = solve_cfg(c);
  const PdSlices sl = pd_slices(c, use16);
  launch_em_init(sc, key, c->p.D, c->Dp, use16 ? c->b16 : c->b32, c->theta, alpha, c->minv, c->X, c->R, c->Pd, sl.H,
                 sl.L, c->part, c->st, c->stream, sl.X);
  c->estep_prev = 0;
}
cofem_status estep_chunk_launches(cofem_ctx* c, bool use16, const float* alpha) {
  const SolveCfg sc = solve_cfg(c);
  const PdSlices sl = pd_slices(c, use16);
  for (int i = 0; i < c->chunk; ++i) {
    cofem_status rc = apply_operator(c, use16, alpha, sc, i);
    if (rc != COFEM_OK) return rc;
    // FIR dictionary, bf16 form: X += gamma P moves from the update to the direction kernel
    const bool xdir = sc.sigblk && sl.H;
    const bool fused = cg_direction_fuses_scalars(sc, sl.H);
    launch_cg_update(sc, c->Dp, c->minv, c->X, c->R, c->Pd, c->Psi, c->pipart, c->part, c->st, c->stream, xdir,
                     !fused);
    launch_cg_direction(sc, c->Dp, c->minv, c->R, c->Pd, sl.H, sl.L, c->st, c->stream, sl.X,
                        xdir ? c->X : nullptr, c->part);
  }
  return COFEM_OK;
}
// Capture the chunk's launches (every argument is fixed for the context, use16 and alpha;
// the per-step state lives on the device) into g.
cofem_status capture_chunk(cofem_ctx* c, bool use16, const float* alpha, cofem_ctx::ChunkGraph& g) {
  if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  hipStream_t caller = c->stream;
  HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  c->stream = c->cap_stream;
  const cofem_status rc = estep_chunk_launches(c, use16, alpha);
  c->stream = caller;
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
  if (rc != COFEM_OK || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc != COFEM_OK ? rc : fail(COFEM_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  }
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  g.exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) {
    g.exec = nullptr;
    return fail(COFEM_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
  }
  g.alpha = alpha;
  return COFEM_OK;
}
cofem_status estep_chunk(cofem_ctx* c, bool use16, const float* alpha) {
  // per-launch events (timing) stay eager, and so does a context whose capture failed
  if (c->timing || c->graph_off) return estep_chunk_launches(c, use16, alpha);
  cofem_ctx::ChunkGraph& g = c->graphs[use16 ? 1 : 0];
  if (!g.exec || g.alpha != alpha) {
    if (capture_chunk(c, use16, alpha, g) != COFEM_OK) {
      (void)hipGetLastError();
      c->graph_off = true;
      return estep_chunk_launches(c, use16, alpha);
    }
  }
  HIP_TRY(hipGraphLaunch(g.exec, c->stream));
  return COFEM_OK;
}
cofem_status estep_poll(cofem_ctx* c, bool* done) {
  cofem_status rc = sync_state(c);
  if (rc != COFEM_OK) return rc;
  if (c->timing && (rc = harvest(c, c->h_st->steps - c->estep_prev)) != COFEM_OK) return rc;
  c->estep_prev = c->h_st->steps;
  *done = c->h_st->done != 0;
  return COFEM_OK;
}

// One E-step on its own: reports the steps taken and the final ratio.
cofem_status solve_estep(cofem_ctx* c, uint64_t key, bool use16, const float* alpha, int* steps, double* delta) {
  estep_begin(c, key, use16, alpha);
  for (bool done = false; !done;) {
    cofem_status rc = estep_chunk(c, use16, alpha);
    if (rc == COFEM_OK) rc = estep_poll(c, &done);
    if (rc != COFEM_OK) return rc;
  }
  *steps = c->h_st->steps;
  *delta = c->h_st->delta;
  return COFEM_OK;
}

bool estep_use16(const cofem_ctx* c, int t) { return c->need16 && (t <= c->p.T - c->p.refine_last); }

// The fit's record of EM iteration t.
void record_estep(cofem_ctx* c, int t, bool use16) {
  c->stats.cg_steps[t - 1] = c->h_st->steps;
  c->stats.rel_resid[t - 1] = c->h_st->delta;
  c->stats.used_bf16[t - 1] = use16 ? 1 : 0;
  c->stats.total_cg_steps += c->h_st->steps;
}

// The E-step of EM iteration t at the given alpha, recorded in the fit's stats.
cofem_status run_estep(cofem_ctx* c, int t, const float* alpha) {
  const bool use16 = estep_use16(c, t);
  int steps = 0;
  double delta = 0.0;
  cofem_status rc = solve_estep(c, estep_key(c, t), use16, alpha, &steps, &delta);
  if (rc != COFEM_OK) return rc;
  record_estep(c, t, use16);
  return COFEM_OK;
}

// The E-steps of EM iteration t of several contexts, each on its own stream, at one
// alpha: the host enqueues a chunk of CG steps for every context still iterating before
// it waits on any of them, so small problems overlap on the device.
cofem_status run_esteps(const std::vector<cofem_ctx*>& cs, int t, const float* alpha) {
  const int n = (int)cs.size();
  std::vector<char> live(n, 1);
  for (cofem_ctx* c : cs) estep_begin(c, estep_key(c, t), estep_use16(c, t), alpha);
  for (int left = n; left > 0;) {
    for (int l = 0; l < n; ++l) {
      if (!live[l]) continue;
      cofem_status rc = estep_chunk(cs[l], estep_use16(cs[l], t), alpha);
      if (rc != COFEM_OK) return rc;
    }
    for (int l = 0; l < n; ++l) {
      if (!live[l]) continue;
      bool done = false;
      cofem_status rc = estep_poll(cs[l], &done);
      if (rc != COFEM_OK) return rc;
      if (done) {
        record_estep(cs[l], t, estep_use16(cs[l], t));
        live[l] = 0;
        --left;
      }
    }
  }
  return COFEM_OK;
}

// End of a fit: the record, and the breakdown error if the mu column broke down.
cofem_status end_fit(cofem_ctx* c, double t0) {
  cofem_status rc = sync_state(c);
  if (rc != COFEM_OK) return rc;
  c->stats.T = c->p.T;
  c->stats.clamped = c->h_st->clamped;
  c->stats.breakdown = c->h_st->breakdown;
  c->stats.ms_fit = now_ms() - t0;
  c->fitted = true;
  if (c->h_st->active[0] == 0 && c->h_st->breakdown > 0 && c->p.stop_mode == COFEM_STOP_JOINT) {
    // the mu column can only be inactive in joint mode through a breakdown
    return fail(COFEM_EBREAKDOWN, "CG breakdown in the mu column");
  }
  return COFEM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
COFEM_API int32_t cofem_abi_version(void) { return COFEM_ABI_VERSION; }

COFEM_API const char* cofem_last_error(void) { return g_err.c_str(); }

COFEM_API cofem_status cofem_create(const cofem_params* p, void* stream, cofem_ctx** out) {
  if (!out) return fail(COFEM_EINVAL, "out is NULL");
  *out = nullptr;
  cofem_status rc = validate(p);
  if (rc != COFEM_OK) return rc;
  cofem_ctx* c = new (std::nothrow) cofem_ctx();
  if (!c) return fail(COFEM_ENOMEM, "host allocation failed");
  c->p = *p;
  c->stream = static_cast<hipStream_t>(stream);
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return fail(COFEM_EDEVICE, "hipGetDevice failed");
  }
  const bool conv = p->op_kind == COFEM_OP_CONV;
  const bool dct = p->op_kind == COFEM_OP_DCT;
  const bool matrix_free = conv || dct;
  c->Np = round_up(p->N, 256);
  c->Dp = round_up(p->D, 256);
  c->Q = p->K + 1;
  c->Qp = (int)round_up(c->Q, 16);
  c->need16 = p->phi_dtype == COFEM_PHI_BF16;
  c->need32 = p->phi_dtype == COFEM_PHI_FP32 || p->refine_last > 0;
  c->g1_16 = choose_gemm(c->Np, c->Dp, 1);
  c->g2_16 = choose_gemm(c->Dp, c->Np, 1);
  c->g1_32 = choose_gemm(c->Np, c->Dp, 0);
  c->g2_32 = choose_gemm(c->Dp, c->Np, 0);
  const int64_t Np = c->Np, Dp = c->Dp, Qp = c->Qp;
  const int64_t ysplit = matrix_free ? 0
                              : std::max<int64_t>(std::max<int64_t>(c->g1_16.splits, c->g1_32.splits) * Np,
                                                  std::max<int64_t>(c->g2_16.splits, c->g2_32.splits) * Dp);
  // dictionary layouts: rows padded to dict_ld (row-major Np rows, transposed Dp rows)
  const size_t nd32 = matrix_free ? 0 : (size_t)Np * (size_t)dict_ld(Dp, 4);
  const size_t nd32T = matrix_free ? 0 : (size_t)Dp * (size_t)dict_ld(Np, 4);
  const size_t nd16 = matrix_free ? 0 : (size_t)c->g1_16.splits * (size_t)Np * (size_t)c->g1_16.kchunk;
  const size_t nd16T = matrix_free ? 0 : (size_t)Dp * (size_t)dict_ld(Np, 2);
#define TRY(x)                   \
  do {                           \
    cofem_status r_ = (x);       \
    if (r_ != COFEM_OK) {        \
      free_all(c);               \
      delete c;                  \
      return r_;                 \
    }                            \
  } while (0)
  if (conv) {
    TRY(dalloc(c, &c->hp32, CONV_HPAD));
    TRY(dalloc(c, &c->hp16, CONV_HPAD));
  }
  if (dct) {
    const size_t L = (size_t)(p->D / 2);
    TRY(dalloc(c, &c->dct_tw, L));
    TRY(dalloc(c, &c->dct_w2, (size_t)DCT_W2_SIZE));
    TRY(dalloc(c, &c->dct_mz, L));
    TRY(dalloc(c, &c->dct_rows, (size_t)p->N));
    TRY(dalloc(c, &c->dct_u, (size_t)Dp));
    if (dct_split_ok(p->D)) {
      TRY(dalloc(c, &c->dct_mzt, L));
      TRY(dalloc(c, &c->dct_y1, (size_t)Qp * L));
      TRY(dalloc(c, &c->dct_y2, (size_t)Qp * L));
    }
  }
  if (c->need32) {
    if (!matrix_free) {
      TRY(dalloc(c, &c->phi32, nd32));
      TRY(dalloc(c, &c->phi32T, nd32T));
    }
    if (conv) TRY(dalloc(c, &c->V, (size_t)Qp * Np));
  }
  if (c->need16) {
    if (!matrix_free) {
      TRY(dalloc(c, &c->phi16, nd16));
      TRY(dalloc(c, &c->phi16T, nd16T));
    }
  }
  // hi/lo slices of Pd and V: the bf16 operators; with the third slices also the dense
  // FP32 operator (the bf16 FIR operator keeps V in registers and needs no V slices)
  const bool dense32 = c->need32 && !matrix_free;
  if (c->need16 || dense32) {
    TRY(dalloc(c, &c->PdH, (size_t)Qp * Dp));
    TRY(dalloc(c, &c->PdL, (size_t)Qp * Dp));
    if (!conv) {
      TRY(dalloc(c, &c->VH, (size_t)Qp * Np));
      TRY(dalloc(c, &c->VL, (size_t)Qp * Np));
    }
  }
  if (dense32) {
    TRY(dalloc(c, &c->PdX, (size_t)Qp * Dp));
    TRY(dalloc(c, &c->VX, (size_t)Qp * Np));
  }
  TRY(dalloc(c, &c->theta, Dp));
  TRY(dalloc(c, &c->alpha, Dp));
  TRY(dalloc(c, &c->alpha_hook, Dp));
  TRY(dalloc(c, &c->b32, Dp));
  TRY(dalloc(c, &c->b16, Dp));
  TRY(dalloc(c, &c->minv, Dp));
  TRY(dalloc(c, &c->mu, Dp));
  TRY(dalloc(c, &c->s, Dp));
  TRY(dalloc(c, &c->yv, Np));
  TRY(dalloc(c, &c->var_sum, Dp));
  TRY(dalloc(c, &c->var_s, Dp));
  TRY(dalloc(c, &c->var_mu, Dp));
  TRY(dalloc(c, &c->X, (size_t)Qp * Dp));
  TRY(dalloc(c, &c->R, (size_t)Qp * Dp));
  TRY(dalloc(c, &c->Pd, (size_t)Qp * Dp));
  TRY(dalloc(c, &c->Psi, (size_t)Qp * Dp));
  TRY(dalloc(c, &c->Ypart, (size_t)Qp * (size_t)ysplit));
  TRY(dalloc(c, &c->part, (size_t)(Dp / VPART + 1) * 2 * QMAX));
  TRY(dalloc(c, &c->pipart, (size_t)(Dp / VPART + 1) * QMAX));
  TRY(dalloc(c, &c->st, 1));
  if (hipHostMalloc((void**)&c->h_st, sizeof(CGState), hipHostMallocDefault) != hipSuccess) {
    c->h_st = nullptr;
    free_all(c);
    delete c;
    return fail(COFEM_ENOMEM, "pinned host allocation failed");
  }
#undef TRY
  launch_state_reset(c->st, c->Q, c->stream);
  // columns of V past the real ones are never written by the passes: keep them zero
  bool zero_ok = true;
  if (c->V) zero_ok &= hipMemsetAsync(c->V, 0, (size_t)Qp * Np * sizeof(float), c->stream) == hipSuccess;
  if (c->VH) zero_ok &= hipMemsetAsync(c->VH, 0, (size_t)Qp * Np * sizeof(uint16_t), c->stream) == hipSuccess;
  if (c->VL) zero_ok &= hipMemsetAsync(c->VL, 0, (size_t)Qp * Np * sizeof(uint16_t), c->stream) == hipSuccess;
  if (c->VX) zero_ok &= hipMemsetAsync(c->VX, 0, (size_t)Qp * Np * sizeof(uint16_t), c->stream) == hipSuccess;
  if (!zero_ok || hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) {
    free_all(c);
    delete c;
    return fail(COFEM_EDEVICE, "workspace initialisation failed");
  }
  *out = c;
  return COFEM_OK;
}

COFEM_API void cofem_destroy(cofem_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  free_all(c);
  delete c;
}

COFEM_API cofem_status cofem_set_dictionary(cofem_ctx* c, const float* phi) {
  if (!c || !phi) return fail(COFEM_EINVAL, "NULL argument");
  if (c->p.op_kind == COFEM_OP_DCT) return fail(COFEM_EINVAL, "a DCT dictionary is loaded by cofem_set_dct_samples");
  const double t0 = now_ms();
  c->dict_loaded = false;
  launch_state_reset(c->st, c->Q, c->stream);
  if (c->p.op_kind == COFEM_OP_CONV) {
    launch_count_nonfinite(phi, c->p.conv_taps, &c->st->nonfinite, c->stream);
    launch_conv_setup(phi, c->p.conv_taps, c->p.D, c->Dp, c->p.theta_mode == COFEM_THETA_JACOBI, c->hp32, c->hp16,
                      c->theta, c->stream);
    HIP_TRY(hipGetLastError());
    cofem_status rc = check_finite(c, "the filter taps");
    if (rc != COFEM_OK) return rc;
    c->dict_loaded = true;
    c->stats.ms_setup = now_ms() - t0;
    return COFEM_OK;
  }
  launch_count_nonfinite(phi, c->p.N * c->p.D, &c->st->nonfinite, c->stream);
  launch_dict_layouts(phi, c->p.N, c->p.D, c->Np, c->Dp, c->g1_16.kchunk, c->phi32, c->phi32T, c->phi16, c->phi16T,
                      c->stream);
  // theta from the caller's FP32 matrix (b is formed per fit from the library's copies)
  launch_theta(phi, c->p.N, c->p.D, c->Dp, c->p.theta_mode == COFEM_THETA_JACOBI, c->theta, c->stream);
  HIP_TRY(hipGetLastError());
  cofem_status rc = check_finite(c, "the dictionary");
  if (rc != COFEM_OK) return rc;
  c->dict_loaded = true;
  c->stats.ms_setup = now_ms() - t0;
  return COFEM_OK;
}

COFEM_API cofem_status cofem_set_dct_samples(cofem_ctx* c, const int32_t* rows) {
  if (!c || !rows) return fail(COFEM_EINVAL, "NULL argument");
  if (c->p.op_kind != COFEM_OP_DCT) return fail(COFEM_EINVAL, "cofem_set_dct_samples needs op_kind COFEM_OP_DCT");
  const double t0 = now_ms();
  const int64_t N = c->p.N, D = c->p.D;
  // the kept samples must be distinct indices in [0, D): checked on the host
  std::vector<int32_t> h(N);
  HIP_TRY(hipMemcpyAsync(h.data(), rows, sizeof(int32_t) * N, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  std::vector<char> seen(D, 0);
  for (int64_t i = 0; i < N; ++i) {
    if (h[i] < 0 || h[i] >= D) return fail(COFEM_EINVAL, "sample index " + std::to_string(h[i]) + " outside [0, D)");
    if (seen[h[i]]) return fail(COFEM_EINVAL, "sample index " + std::to_string(h[i]) + " repeated");
    seen[h[i]] = 1;
  }
  HIP_TRY(hipMemcpyAsync(c->dct_rows, h.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, c->stream));
  launch_dct_setup(c->dct_rows, N, D, c->Dp, c->p.theta_mode == COFEM_THETA_JACOBI, c->dct_tw, c->dct_w2,
                   c->dct_mz, c->dct_mzt, c->dct_u, c->theta, c->stream);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->dict_loaded = true;
  c->stats.ms_setup = now_ms() - t0;
  return COFEM_OK;
}

COFEM_API cofem_status cofem_fit(cofem_ctx* c, const float* y) {
  if (!c || !y) return fail(COFEM_EINVAL, "NULL argument");
  if (!c->dict_loaded) return fail(COFEM_ESTATE, "cofem_fit before cofem_set_dictionary");
  const double t0 = now_ms();
  const cofem_params& p = c->p;
  begin_fit(c, y);
  cofem_status rc0 = check_finite(c, "y");
  if (rc0 != COFEM_OK) return rc0;
  launch_fill(c->alpha, 1.0f, c->Dp, c->stream);
  for (int t = 1; t <= p.T; ++t) {
    cofem_status rc = run_estep(c, t, c->alpha);
    if (rc != COFEM_OK) return rc;
    launch_mstep(solve_cfg(c), estep_key(c, t), p.D, c->Dp, c->X, c->mu, c->s, c->alpha, p.alpha_floor,
                 t < p.T ? 1 : 0, c->st, c->stream);
  }
  return end_fit(c, t0);
}

COFEM_API cofem_status cofem_posterior(cofem_ctx* c, float* mu, float* s, float* alpha, cofem_stats* st) {
  if (!c) return fail(COFEM_EINVAL, "NULL context");
  if (!c->fitted) return fail(COFEM_ESTATE, "cofem_posterior before a successful cofem_fit");
  const size_t bytes = (size_t)c->p.D * sizeof(float);
  if (mu) HIP_TRY(hipMemcpyAsync(mu, c->mu, bytes, hipMemcpyDeviceToDevice, c->stream));
  if (s) HIP_TRY(hipMemcpyAsync(s, c->s, bytes, hipMemcpyDeviceToDevice, c->stream));
  if (alpha) HIP_TRY(hipMemcpyAsync(alpha, c->alpha, bytes, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (st) *st = c->stats;
  return COFEM_OK;
}

COFEM_API cofem_status cofem_variance(cofem_ctx* c, const float* alpha, int32_t batches, uint64_t seed, float* s_out,
                                      float* mu_out, cofem_stats* st) {
  if (!c || !s_out) return fail(COFEM_EINVAL, "NULL argument");
  if (batches < 1 || batches > COFEM_MAX_T) return fail(COFEM_EINVAL, "batches must be in [1, COFEM_MAX_T]");
  if (!c->fitted) return fail(COFEM_ESTATE, "cofem_variance before a successful cofem_fit");
  const cofem_params& p = c->p;
  const double t0 = now_ms();
  const float* a = c->alpha;
  if (alpha) {
    launch_copy_pad(alpha, p.D, c->Dp, 1.0f, c->alpha_hook, c->stream);
    a = c->alpha_hook;
  }
  const bool use16 = !c->need32;  // the FP32 operator whenever the context holds it
  cofem_stats vs{};
  vs.T = batches;
  launch_fill(c->var_sum, 0.0f, c->Dp, c->stream);
  for (int b = 1; b <= batches; ++b) {
    const uint64_t key = mix64_host(seed + (uint64_t)b * GOLDEN_GAMMA);
    int steps = 0;
    double delta = 0.0;
    cofem_status rc = solve_estep(c, key, use16, a, &steps, &delta);
    if (rc != COFEM_OK) return rc;
    vs.cg_steps[b - 1] = steps;
    vs.rel_resid[b - 1] = delta;
    vs.used_bf16[b - 1] = use16 ? 1 : 0;
    vs.total_cg_steps += steps;
    launch_mstep(solve_cfg(c), key, p.D, c->Dp, c->X, c->var_mu, c->var_s, c->alpha_hook, p.alpha_floor, 0, c->st,
                 c->stream);
    launch_axpy(c->var_sum, c->var_s, (float)(1.0 / batches), c->Dp, c->stream);
  }
  const size_t bytes = (size_t)p.D * sizeof(float);
  HIP_TRY(hipMemcpyAsync(s_out, c->var_sum, bytes, hipMemcpyDeviceToDevice, c->stream));
  if (mu_out) HIP_TRY(hipMemcpyAsync(mu_out, c->var_mu, bytes, hipMemcpyDeviceToDevice, c->stream));
  cofem_status rc = sync_state(c);
  if (rc != COFEM_OK) return rc;
  vs.breakdown = c->h_st->breakdown;
  vs.ms_fit = now_ms() - t0;
  if (st) *st = vs;
  if (c->h_st->active[0] == 0 && c->h_st->breakdown > 0 && p.stop_mode == COFEM_STOP_JOINT)
    return fail(COFEM_EBREAKDOWN, "CG breakdown in the mu column");
  return COFEM_OK;
}

COFEM_API cofem_status cofem_apply_A(cofem_ctx* c, const float* alpha, const float* P, float* Psi, int32_t ncols,
                                     int32_t use_bf16, double* pi) {
  if (!c || !alpha || !P || !Psi) return fail(COFEM_EINVAL, "NULL argument");
  if (!c->dict_loaded) return fail(COFEM_ESTATE, "cofem_apply_A before cofem_set_dictionary");
  if (ncols < 1 || ncols > c->Qp) return fail(COFEM_EINVAL, "ncols must be in [1, padded K+1]");
  if (use_bf16 && !c->need16) return fail(COFEM_EINVAL, "bfloat16 operator needs phi_dtype = COFEM_PHI_BF16");
  if (!use_bf16 && !c->need32) return fail(COFEM_EINVAL, "FP32 operator needs phi_dtype = FP32 or refine_last > 0");
  SolveCfg sc = solve_cfg(c);
  sc.Q = ncols;
  launch_copy_pad(alpha, c->p.D, c->Dp, 1.0f, c->alpha_hook, c->stream);
  const bool sliced32 = !use_bf16 && c->PdX;
  launch_pack_block(P, ncols, c->p.D, c->Qp, c->Dp, c->Pd, (use_bf16 || sliced32) ? c->PdH : nullptr,
                    (use_bf16 || sliced32) ? c->PdL : nullptr, c->stream, sliced32 ? c->PdX : nullptr,
                    c->p.op_kind == COFEM_OP_CONV ? 1 : 0);
  launch_state_reset(c->st, c->Q, c->stream);
  cofem_status rc = apply_operator(c, use_bf16 != 0, c->alpha_hook, sc, 0);
  if (rc != COFEM_OK) return rc;
  launch_reduce_pi(ncols, c->Dp, c->pipart, c->st->pi, c->stream);
  launch_unpack_block(c->Psi, ncols, c->p.D, c->Dp, Psi, c->stream);
  if (pi) HIP_TRY(hipMemcpyAsync(pi, c->st->pi, sizeof(double) * ncols, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (c->timing && (rc = harvest(c, 1)) != COFEM_OK) return rc;
  return COFEM_OK;
}

COFEM_API cofem_status cofem_set_probe_mode(cofem_ctx* c, int32_t mode) {
  if (!c) return fail(COFEM_EINVAL, "NULL context");
  if (mode != COFEM_PROBES_HASH && mode != COFEM_PROBES_HADAMARD) return fail(COFEM_EINVAL, "bad probe mode");
  if (mode == COFEM_PROBES_HADAMARD) {
    const int64_t D = c->p.D;
    if ((D & (D - 1)) != 0) return fail(COFEM_EINVAL, "Hadamard probes need D a power of two");
    if (c->p.K > D) return fail(COFEM_EINVAL, "Hadamard probes need K <= D");
  }
  c->probe_mode = mode;
  return COFEM_OK;
}

COFEM_API cofem_status cofem_set_timing(cofem_ctx* c, int32_t enable) {
  if (!c) return fail(COFEM_EINVAL, "NULL context");
  HIP_TRY(hipStreamSynchronize(c->stream));
  cofem_status rc = harvest(c, 0);
  if (rc != COFEM_OK) return rc;
  c->timing = enable != 0;
  c->t_ms[0] = c->t_ms[1] = 0.0;
  c->t_n[0] = c->t_n[1] = 0;
  return COFEM_OK;
}

COFEM_API cofem_status cofem_get_timing(cofem_ctx* c, int32_t which, double* total_ms, int64_t* launches) {
  if (!c || which < 0 || which > 1) return fail(COFEM_EINVAL, "bad argument");
  if (total_ms) *total_ms = c->t_ms[which];
  if (launches) *launches = c->t_n[which];
  return COFEM_OK;
}

// ---------------------------------------------------------------------------
// Multi-task CoFEM, in one of two forms: batched (every task a slot of one alpha group
// of the serving kernels, mt_batch.h), or one context per task on its own stream with
// alpha shared (the buffer of task 0).
// ---------------------------------------------------------------------------
struct cofem_mt {
  cofem::MtBatch* batch = nullptr;  // the batched form; the fields below are then unused
  std::vector<cofem_ctx*> tasks;
  // task 0 runs on the caller's stream, task l > 0 on streams[l - 1] (created here, default
  // priority); ev[l] orders the tasks' streams around the shared alpha
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> ev;
  const float** d_mus = nullptr;  // device arrays of the tasks' mu and s pointers
  const float** d_ss = nullptr;
  bool fitted = false;
};

namespace {

void mt_free(cofem_mt* m) {
  cofem::mtb_destroy(m->batch);
  m->batch = nullptr;
  for (cofem_ctx* c : m->tasks) cofem_destroy(c);
  m->tasks.clear();
  for (hipStream_t s : m->streams) (void)hipStreamDestroy(s);
  m->streams.clear();
  for (hipEvent_t e : m->ev) (void)hipEventDestroy(e);
  m->ev.clear();
  if (m->d_mus) (void)hipFree(m->d_mus);
  if (m->d_ss) (void)hipFree(m->d_ss);
  m->d_mus = m->d_ss = nullptr;
}

}  // namespace

COFEM_API cofem_status cofem_mt_create(const cofem_params* p, int32_t L, void* stream, cofem_mt** out) {
  return cofem_mt_create_mode(p, L, COFEM_MT_AUTO, stream, out);
}

COFEM_API cofem_status cofem_mt_create_mode(const cofem_params* p, int32_t L, int32_t mode, void* stream,
                                           cofem_mt** out) {
  if (!out) return fail(COFEM_EINVAL, "out is NULL");
  *out = nullptr;
  if (L < 1 || L > COFEM_MAX_TASKS) return fail(COFEM_EINVAL, "L must be in [1, COFEM_MAX_TASKS]");
  if (mode != COFEM_MT_AUTO && mode != COFEM_MT_STREAMS && mode != COFEM_MT_BATCHED)
    return fail(COFEM_EINVAL, "bad multi-task mode");
  cofem_status rc = validate(p);
  if (rc != COFEM_OK) return rc;
  if (p->mstep_mode != COFEM_MSTEP_GAUSSIAN) return fail(COFEM_EINVAL, "multi-task fits use the Gaussian M-step");
  const bool eligible = cofem::mtb_eligible(*p);
  if (mode == COFEM_MT_BATCHED && !eligible)
    return fail(COFEM_EINVAL, "the batched multi-task fit takes dense FP32 dictionaries, no refinement, K <= 31");
  cofem_mt* m = new (std::nothrow) cofem_mt();
  if (!m) return fail(COFEM_ENOMEM, "host allocation failed");
  // the streams form overlaps the tasks only as far as the device's hardware queues go (4
  // per process by default): batched beyond that
  if (mode == COFEM_MT_BATCHED || (mode == COFEM_MT_AUTO && eligible && L > COFEM_MT_AUTO_STREAMS_MAX)) {
    rc = cofem::mtb_create(*p, L, static_cast<hipStream_t>(stream), &m->batch);
    if (rc != COFEM_OK) {
      delete m;
      return rc;
    }
    *out = m;
    return COFEM_OK;
  }
  std::vector<const float*> mus(L), ss(L);
  for (int l = 0; l < L; ++l) {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      mt_free(m);
      delete m;
      return fail(COFEM_EDEVICE, "hipEventCreateWithFlags failed");
    }
    m->ev.push_back(e);
    void* task_stream = stream;
    if (l > 0) {
      hipStream_t s = nullptr;
      if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        mt_free(m);
        delete m;
        return fail(COFEM_EDEVICE, "hipStreamCreateWithFlags failed");
      }
      m->streams.push_back(s);
      task_stream = s;
    }
    cofem_params q = *p;
    q.seed = p->seed + (uint64_t)l;  // task l's probes
    cofem_ctx* c = nullptr;
    rc = cofem_create(&q, task_stream, &c);
    if (rc != COFEM_OK) {
      mt_free(m);
      delete m;
      return rc;
    }
    m->tasks.push_back(c);
    mus[l] = c->mu;
    ss[l] = c->s;
  }
  hipStream_t st = m->tasks[0]->stream;
  if (hipMalloc((void**)&m->d_mus, sizeof(float*) * L) != hipSuccess ||
      hipMalloc((void**)&m->d_ss, sizeof(float*) * L) != hipSuccess ||
      hipMemcpyAsync(m->d_mus, mus.data(), sizeof(float*) * L, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(m->d_ss, ss.data(), sizeof(float*) * L, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    (void)hipGetLastError();
    mt_free(m);
    delete m;
    return fail(COFEM_ENOMEM, "task table allocation failed");
  }
  *out = m;
  return COFEM_OK;
}

COFEM_API void cofem_mt_destroy(cofem_mt* m) {
  if (!m) return;
  mt_free(m);
  delete m;
}

COFEM_API int32_t cofem_mt_batched(const cofem_mt* m) { return (m && m->batch) ? 1 : 0; }

// Task `task`'s stream after the caller's stream (task 0's), so that the task reads
// caller data only once the caller's stream has produced it.
static cofem_status mt_after_caller(cofem_mt* m, int task) {
  if (task == 0) return COFEM_OK;
  HIP_TRY(hipEventRecord(m->ev[0], m->tasks[0]->stream));
  HIP_TRY(hipStreamWaitEvent(m->tasks[task]->stream, m->ev[0], 0));
  return COFEM_OK;
}

COFEM_API cofem_status cofem_mt_set_dictionary(cofem_mt* m, int32_t task, const float* phi) {
  if (m && m->batch) return cofem::mtb_set_dictionary(m->batch, task, phi);
  if (!m || task < 0 || task >= (int32_t)m->tasks.size()) return fail(COFEM_EINVAL, "bad task");
  cofem_status rc = mt_after_caller(m, task);
  if (rc != COFEM_OK) return rc;
  return cofem_set_dictionary(m->tasks[task], phi);
}

COFEM_API cofem_status cofem_mt_set_dct_samples(cofem_mt* m, int32_t task, const int32_t* rows) {
  if (m && m->batch) return fail(COFEM_EINVAL, "the batched multi-task fit takes dense dictionaries");
  if (!m || task < 0 || task >= (int32_t)m->tasks.size()) return fail(COFEM_EINVAL, "bad task");
  cofem_status rc = mt_after_caller(m, task);
  if (rc != COFEM_OK) return rc;
  return cofem_set_dct_samples(m->tasks[task], rows);
}

COFEM_API cofem_status cofem_mt_fit(cofem_mt* m, const float* const* ys) {
  if (!m || !ys) return fail(COFEM_EINVAL, "NULL argument");
  if (m->batch) return cofem::mtb_fit(m->batch, ys);
  const int L = (int)m->tasks.size();
  for (int l = 0; l < L; ++l) {
    if (!ys[l]) return fail(COFEM_EINVAL, "NULL observation");
    if (!m->tasks[l]->dict_loaded) return fail(COFEM_ESTATE, "cofem_mt_fit before every task has a dictionary");
  }
  const double t0 = now_ms();
  m->fitted = false;
  cofem_ctx* c0 = m->tasks[0];
  const cofem_params& p = c0->p;
  float* alpha = c0->alpha;  // the shared alpha
  // every task stream after the caller's stream (the observations, then alpha)
  auto fork = [&]() -> cofem_status {
    HIP_TRY(hipEventRecord(m->ev[0], c0->stream));
    for (int l = 1; l < L; ++l) HIP_TRY(hipStreamWaitEvent(m->tasks[l]->stream, m->ev[0], 0));
    return COFEM_OK;
  };
  // the caller's stream after every task stream
  auto join = [&]() -> cofem_status {
    for (int l = 1; l < L; ++l) {
      HIP_TRY(hipEventRecord(m->ev[l], m->tasks[l]->stream));
      HIP_TRY(hipStreamWaitEvent(c0->stream, m->ev[l], 0));
    }
    return COFEM_OK;
  };
  cofem_status rc = fork();
  if (rc != COFEM_OK) return rc;
  for (int l = 0; l < L; ++l) begin_fit(m->tasks[l], ys[l]);
  for (int l = 0; l < L; ++l) {
    const std::string what = "ys[" + std::to_string(l) + "]";
    if ((rc = check_finite(m->tasks[l], what.c_str())) != COFEM_OK) return rc;
  }
  launch_fill(alpha, 1.0f, c0->Dp, c0->stream);
  for (int t = 1; t <= p.T; ++t) {
    // the L E-steps run concurrently, one stream each, at the shared alpha
    if ((rc = fork()) != COFEM_OK) return rc;
    if ((rc = run_esteps(m->tasks, t, alpha)) != COFEM_OK) return rc;
    for (int l = 0; l < L; ++l) {
      cofem_ctx* c = m->tasks[l];
      // mu_l and s_l only; the joint M-step follows
      launch_mstep(solve_cfg(c), estep_key(c, t), p.D, c->Dp, c->X, c->mu, c->s, nullptr, p.alpha_floor, 0, c->st,
                   c->stream);
    }
    if ((rc = join()) != COFEM_OK) return rc;
    if (t < p.T) launch_mt_mstep(m->d_mus, m->d_ss, L, p.D, alpha, p.alpha_floor, &c0->st->clamped, c0->stream);
  }
  cofem_status worst = COFEM_OK;
  for (int l = 0; l < L; ++l) {
    const cofem_status r = end_fit(m->tasks[l], t0);
    if (r == COFEM_EBREAKDOWN) worst = r;
    else if (r != COFEM_OK) return r;
  }
  m->fitted = true;
  return worst;
}

COFEM_API cofem_status cofem_mt_posterior(cofem_mt* m, int32_t task, float* mu, float* s, float* alpha,
                                          cofem_stats* st) {
  if (m && m->batch) return cofem::mtb_posterior(m->batch, task, mu, s, alpha, st);
  if (!m || task < 0 || task >= (int32_t)m->tasks.size()) return fail(COFEM_EINVAL, "bad task");
  if (!m->fitted) return fail(COFEM_ESTATE, "cofem_mt_posterior before a successful cofem_mt_fit");
  cofem_ctx* c = m->tasks[task];
  cofem_status rc = cofem_posterior(c, mu, s, nullptr, st);
  if (rc != COFEM_OK) return rc;
  if (alpha) {
    cofem_ctx* c0 = m->tasks[0];
    HIP_TRY(hipMemcpyAsync(alpha, c0->alpha, (size_t)c0->p.D * sizeof(float), hipMemcpyDeviceToDevice, c0->stream));
    HIP_TRY(hipStreamSynchronize(c0->stream));
  }
  return COFEM_OK;
}

