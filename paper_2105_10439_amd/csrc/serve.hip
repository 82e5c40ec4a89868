// Serving: continuous batching of independent CoFEM fits (include/cofem.h), and the
// batched multi-task fit (Sec. III-E.1) on the same kernels.
//
// Every admitted request owns a slot: a region of one device arena holding its
// dictionary (row-major and transposed, FP32), its CG blocks and its state.  A
// tick is a fixed sequence of persistent kernels, captured once as a hipGraph:
// E-step initialisation, steps_per_tick CG steps, M-step and EM advance.  Each
// kernel has a fixed grid that strides over a tile table covering all running
// slots (rebuilt by the host only when slots are admitted or retired), and each
// slot moves through its own EM iterations on the device.  The per-tile work is
// the same code as the single-problem path (tiles.h).
//
// A group of slots shares one alpha (multi-task CoFEM): its members run their own
// E-steps (own dictionary, observation, probes and stop rule), each computes its mu and
// s when its E-step ends and then waits; once every member has finished E-step t, one
// kernel forms the joint M-step alpha_j = L / sum_l (mu_lj^2 + s_lj) and the members
// move to E-step t + 1 together.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

#include "cofem.h"
#include "kernels.h"
#include "mt_batch.h"
#include "tiles.h"

#define COFEM_API extern "C" __attribute__((visibility("default")))

namespace cofem {

constexpr int SRV_MAXSLOTS = 128;
constexpr int SRV_QP = 32;              // padded right-hand sides of a serving fit (K <= 31)
constexpr int SRV_RT = 2;               // row tiles of 16 per wave in the serving contractions
constexpr int64_t SRV_KCHUNK = 2048;    // reduction length per split
constexpr int SRV_GEMM_GRID = 512;      // persistent grids (multiples of 8: tile L stays on XCD L % 8)
constexpr int SRV_VEC_GRID = 1024;

enum { PH_IDLE = 0, PH_INIT = 1, PH_CG = 2, PH_DONE = 3 };

// Immutable description of one running fit (device copy in the slot array).
struct SlotDev {
  SolveCfg c;
  int64_t N, D, Np, Dp;
  int T;
  uint64_t seed;
  double floor;
  int nrb1, splits1, nrb2, splits2;
  int64_t kchunk1, kchunk2;
  int nbx, nbn;  // vector tiles per column over Dp and Np
  int x1;        // Q = 17: one MFMA column tile plus the 17th column on the vector ALU
  const float* phi;
  const float* phiT;
  float *V, *Ypart, *X, *R, *Pd, *Psi, *minv, *alpha, *b, *theta, *mu, *s;
  double *part, *pipart;
  CGState* st;
  int* steps_log;       // CG steps of each E-step (T ints)
  double* resid_log;    // ||R||_F / ||B||_F at the end of each E-step (T doubles)
  int grp_first, grp_n;  // alpha group: slots grp_first .. grp_first + grp_n - 1 (grp_n = 0: none)
};

// Tile table of the running slots: for every kind of tile, a prefix sum of the
// per-slot tile counts, each slot's range starting at a multiple of 8.
struct SrvTable {
  int n;
  int slot[SRV_MAXSLOTS];
  int em[SRV_MAXSLOTS + 1];   // E-step init / M-step blocks: Dp / 256
  int g1[SRV_MAXSLOTS + 1];   // pass-1 contraction tiles: nrb1 * splits1
  int g2[SRV_MAXSLOTS + 1];   // pass-2 contraction tiles: nrb2 * splits2
  int f1[SRV_MAXSLOTS + 1];   // pass-1 finish tiles: nbn * Qp
  int vq[SRV_MAXSLOTS + 1];   // per-column vector tiles: nbx * Q
};

__device__ __forceinline__ int find_slot(const int* start, int n, int t) {
  int lo = 0, hi = n - 1;  // largest i with start[i] <= t
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ---- tick kernels -----------------------------------------------------------
__global__ __launch_bounds__(VBLOCK) void ks_em_init(const SlotDev* __restrict__ slots,
                                                     const SrvTable* __restrict__ tab) {
  const int n = tab->n, total = tab->em[n];
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    const int i = find_slot(tab->em, n, t);
    const SlotDev& sd = slots[tab->slot[i]];
    const int local = t - tab->em[i];
    if (sd.st->phase != PH_INIT || local >= (int)(sd.Dp / VBLOCK)) continue;
    em_init_block(sd.c, iteration_key(sd.seed, sd.st->t), sd.D, sd.Dp, local, sd.b, sd.theta, sd.alpha, sd.minv,
                  sd.X, sd.R, sd.Pd, nullptr, nullptr, nullptr, sd.part);
  }
}

__global__ __launch_bounds__(VBLOCK) void ks_em_scalars(const SlotDev* __restrict__ slots,
                                                        const SrvTable* __restrict__ tab) {
  for (int i = blockIdx.x; i < tab->n; i += gridDim.x) {
    const SlotDev& sd = slots[tab->slot[i]];
    if (sd.st->phase != PH_INIT) continue;
    em_scalars_block(sd.c, sd.D, (int)(sd.Dp / VBLOCK), sd.part, sd.st);
    if (threadIdx.x == 0) sd.st->phase = PH_CG;
    __syncthreads();
  }
}

__device__ __forceinline__ bool in_cg(const SlotDev& sd) { return sd.st->phase == PH_CG && !sd.st->done; }

// Contraction tiles of all running slots, claimed one at a time from a counter (tiles of
// different requests differ in length, so a static stride leaves blocks idle at the end).
// Each tile writes its own partial, so the result does not depend on which block ran it.
// Every block leaves once the counter has passed the last tile.
__global__ __launch_bounds__(64 * GEMM_WAVES, 2) void ks_gemm(const SlotDev* __restrict__ slots, const SrvTable* __restrict__ tab,
                                                  int pass, int* __restrict__ ctr) {
  const int n = tab->n;
  const int* start = pass == 1 ? tab->g1 : tab->g2;
  const int total = start[n];
  __shared__ int s_t;
  for (;;) {
    if (threadIdx.x == 0) s_t = atomicAdd(ctr, 1);
    __syncthreads();
    const int t = s_t;
    __syncthreads();  // every wave has read s_t before the next claim overwrites it
    if (t >= total) break;
    const int i = find_slot(start, n, t);
    const SlotDev& sd = slots[tab->slot[i]];
    const int local = t - start[i];
    const int ntile = pass == 1 ? sd.nrb1 * sd.splits1 : sd.nrb2 * sd.splits2;
    if (!in_cg(sd) || local >= ntile) continue;
    const float* M = pass == 1 ? sd.phi : sd.phiT;
    const float* Z = pass == 1 ? sd.Pd : sd.V;
    const int64_t kdim = pass == 1 ? sd.Dp : sd.Np, rows = pass == 1 ? sd.Np : sd.Dp;
    const int64_t kchunk = pass == 1 ? sd.kchunk1 : sd.kchunk2;
    const int nrb = pass == 1 ? sd.nrb1 : sd.nrb2, splits = pass == 1 ? sd.splits1 : sd.splits2;
    if (sd.x1)
      gemm_f32_tile<SRV_RT, 1, 4, true>(local, M, kdim, Z, kdim, sd.Ypart, rows, SRV_QP, kchunk, kdim, nrb, splits);
    else
      gemm_f32_tile<SRV_RT, SRV_QP / 16, 4, false>(local, M, kdim, Z, kdim, sd.Ypart, rows, SRV_QP, kchunk, kdim, nrb,
                                                   splits);
    __syncthreads();  // the next tile reuses the LDS staging buffers
  }
}

// Zero the tile counters of one tick (a kernel, not a memset node, inside the captured graph).
__global__ void ks_reset_ctr(int* __restrict__ ctr, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) ctr[i] = 0;
}

__global__ __launch_bounds__(VBLOCK) void ks_finish1(const SlotDev* __restrict__ slots,
                                                     const SrvTable* __restrict__ tab) {
  const int n = tab->n, total = tab->f1[n];
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    const int i = find_slot(tab->f1, n, t);
    const SlotDev& sd = slots[tab->slot[i]];
    const int local = t - tab->f1[i];
    if (!in_cg(sd) || local >= sd.nbn * (sd.x1 ? sd.c.Q : SRV_QP)) continue;  // X1 leaves columns > Q unwritten
    finish1_tile(local % sd.nbn, local / sd.nbn, sd.Ypart, sd.splits1, sd.Np, sd.V, nullptr, nullptr, SRV_QP);
  }
}

__global__ __launch_bounds__(VBLOCK) void ks_finish2(const SlotDev* __restrict__ slots,
                                                     const SrvTable* __restrict__ tab) {
  const int n = tab->n, total = tab->vq[n];
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    const int i = find_slot(tab->vq, n, t);
    const SlotDev& sd = slots[tab->slot[i]];
    const int local = t - tab->vq[i];
    if (!in_cg(sd) || local >= sd.nbx * sd.c.Q) continue;
    finish2_tile(sd.c, local % sd.nbx, local / sd.nbx, sd.nbx, sd.Ypart, sd.splits2, sd.Dp, sd.alpha, sd.Pd, sd.Psi,
                 sd.pipart);
  }
}

__global__ __launch_bounds__(VBLOCK) void ks_update(const SlotDev* __restrict__ slots,
                                                    const SrvTable* __restrict__ tab) {
  const int n = tab->n, total = tab->vq[n];
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    const int i = find_slot(tab->vq, n, t);
    const SlotDev& sd = slots[tab->slot[i]];
    const int local = t - tab->vq[i];
    if (!in_cg(sd) || local >= sd.nbx * sd.c.Q) continue;
    cg_update_tile<false>(sd.c, local % sd.nbx, local / sd.nbx, sd.nbx, sd.Dp, sd.minv, sd.X, sd.R, sd.Pd, sd.Psi,
                   sd.pipart, sd.part, sd.st);
  }
}

// The CG scalars and the direction of every running slot in one launch (as the
// single-problem k_cg_scalars_direction): a tile reduces its column's rho' partials for
// eta with the old rho from rho_prev, and the slot's first tile also runs the slot's
// scalars (norms, stop rule, step count, done).
__global__ __launch_bounds__(VBLOCK) void ks_scalars_direction(const SlotDev* __restrict__ slots,
                                                               const SrvTable* __restrict__ tab) {
  __shared__ double s_eta;
  __shared__ int s_run;
  const int n = tab->n, total = tab->vq[n];
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    const int i = find_slot(tab->vq, n, t);
    const SlotDev& sd = slots[tab->slot[i]];
    const int local = t - tab->vq[i];
    // the slot's first tile sets done during this launch: one reading of the flag for the
    // whole block, so its waves agree on which tiles they run (and so on their barriers)
    if (threadIdx.x == 0) s_run = in_cg(sd) && local < sd.nbx * sd.c.Q;
    __syncthreads();
    const int run = s_run;
    __syncthreads();  // s_run is written again for the next tile
    if (!run) continue;
    const int bx = local % sd.nbx, q = local / sd.nbx;
    const DirTile dt = cg_direction_load(bx, q, sd.Dp, sd.minv, sd.R, sd.Pd);  // in flight during eta's reduction
    if (threadIdx.x < 64) {
      const double old = sd.st->rho_prev[q];  // loaded with the partials, not after them
      const double2* pq = reinterpret_cast<const double2*>(sd.part + (int64_t)q * sd.nbx * 2);
      double b = 0.0;
#pragma unroll 8
      for (int k = threadIdx.x; k < sd.nbx; k += 64) b += pq[k].y;
      b = wave_sum(b);
      if (threadIdx.x == 0) s_eta = (old != 0.0) ? b / old : 0.0;
    }
    __syncthreads();
    cg_direction_store(dt, bx, q, sd.Dp, s_eta, sd.Pd, nullptr, nullptr, nullptr);
    if (local == 0) cg_scalars_block(sd.c, sd.nbx, sd.part, sd.st);
    __syncthreads();  // s_eta and the scalars' shared arrays are reused by the next tile
  }
}

__global__ __launch_bounds__(VBLOCK) void ks_mstep(const SlotDev* __restrict__ slots, const SrvTable* __restrict__ tab) {
  const int n = tab->n, total = tab->em[n];
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    const int i = find_slot(tab->em, n, t);
    const SlotDev& sd = slots[tab->slot[i]];
    const int local = t - tab->em[i];
    if (sd.st->phase != PH_CG || !sd.st->done || local >= (int)((sd.D + VBLOCK - 1) / VBLOCK)) continue;
    const int tt = sd.st->t;
    // a group member takes mu and s only (recomputed unchanged while it waits for the group)
    mstep_block(sd.c, iteration_key(sd.seed, tt), sd.D, sd.Dp, local, sd.X, sd.mu, sd.s, sd.alpha, sd.floor,
                (tt < sd.T && sd.grp_n == 0) ? 1 : 0, sd.st);
  }
}

__device__ __forceinline__ bool estep_over(const CGState* st) { return st->phase == PH_CG && st->done; }

// Joint M-step of an alpha group once every member has finished the same E-step t < T:
// alpha_j = 1 / max((1/L) sum_l (mu_lj^2 + s_lj), floor), the members summed in slot
// order in FP64, floor events counted on the first member.  The group's first slot's
// E-step blocks cover D.
__global__ __launch_bounds__(VBLOCK) void ks_group_alpha(const SlotDev* __restrict__ slots,
                                                         const SrvTable* __restrict__ tab) {
  const int n = tab->n, total = tab->em[n];
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    const int i = find_slot(tab->em, n, t);
    const int si = tab->slot[i];
    const SlotDev& sd = slots[si];
    const int local = t - tab->em[i];
    if (sd.grp_n == 0 || si != sd.grp_first || local >= (int)((sd.D + VBLOCK - 1) / VBLOCK)) continue;
    bool ready = true;
    for (int m = 0; m < sd.grp_n; ++m) {
      const CGState* st = slots[si + m].st;
      ready = ready && estep_over(st) && st->t == sd.st->t;
    }
    if (!ready || sd.st->t >= sd.T) continue;
    const int64_t j = (int64_t)local * VBLOCK + threadIdx.x;
    int low = 0;
    if (j < sd.D) {
      double acc = 0.0;
      for (int m = 0; m < sd.grp_n; ++m) {
        const double mu = (double)slots[si + m].mu[j];
        acc += mu * mu + (double)slots[si + m].s[j];
      }
      double den = acc / (double)sd.grp_n;
      if (den < sd.floor) {
        den = sd.floor;
        low = 1;
      }
      sd.alpha[j] = (float)(1.0 / den);
    }
    low = wave_sum_int(low);
    if ((threadIdx.x & 63) == 0 && low) atomicAdd(&sd.st->clamped, low);
  }
}

// One block, one thread per listed slot: record the finished E-step and move to the
// next EM iteration or to DONE (a group member only once every member has finished the
// same E-step); publish every listed slot's phase.  Every thread decides from the
// states as they were at entry before any thread changes one.
__global__ void ks_advance(const SlotDev* __restrict__ slots, const SrvTable* __restrict__ tab,
                           int* __restrict__ phase_out) {
  __shared__ unsigned char over[SRV_MAXSLOTS];  // by slot index
  const int n = tab->n, i = threadIdx.x;
  for (int k = i; k < SRV_MAXSLOTS; k += blockDim.x) over[k] = 0;
  __syncthreads();
  if (i < n) over[tab->slot[i]] = estep_over(slots[tab->slot[i]].st) ? 1 : 0;
  __syncthreads();
  if (i >= n) return;
  const SlotDev& sd = slots[tab->slot[i]];
  CGState* st = sd.st;
  bool go = over[tab->slot[i]] != 0;
  for (int m = 0; go && m < sd.grp_n; ++m) go = over[sd.grp_first + m] != 0;
  if (go) {
    sd.steps_log[st->t - 1] = st->steps;
    sd.resid_log[st->t - 1] = st->delta;
    st->total_steps += st->steps;
    if (st->t < sd.T) {
      st->t += 1;
      st->phase = PH_INIT;
    } else {
      st->phase = PH_DONE;
    }
  }
  phase_out[i] = st->phase;
}

// ---- admission kernels ---------------------------------------------------------
__global__ void ks_zero(float* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

// phiT (Dp x Np) from phi (Np x Dp), 64 x 64 tiles through LDS.
__global__ __launch_bounds__(256) void ks_transpose(const float* __restrict__ phi, int64_t Np, int64_t Dp,
                                                    float* __restrict__ phiT) {
  __shared__ float tile[64][65];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t j0 = (int64_t)blockIdx.x * 64, i0 = (int64_t)blockIdx.y * 64;
  for (int r = ty; r < 64; r += 4) tile[r][tx] = phi[(i0 + r) * Dp + j0 + tx];
  __syncthreads();
  for (int r = ty; r < 64; r += 4) phiT[(j0 + r) * Np + i0 + tx] = tile[tx][r];
}

// theta_j = sum_i Phi_ij^2 (Jacobi) or 1 over the padded row-major copy; padding 1.
__global__ void ks_theta(const float* __restrict__ phi, int64_t Np, int64_t D, int64_t Dp, int jacobi,
                         float* __restrict__ theta) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= Dp) return;
  if (!jacobi || j >= D) {
    theta[j] = 1.0f;
    return;
  }
  double sq = 0.0;
  for (int64_t i = 0; i < Np; ++i) {
    const double v = (double)phi[i * Dp + j];
    sq += v * v;
  }
  theta[j] = (float)sq;
}

__global__ void ks_slot_start(CGState* st, float* alpha, int64_t Dp) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < Dp; j += (int64_t)gridDim.x * blockDim.x)
    alpha[j] = 1.0f;
  if (blockIdx.x == 0) {
    int* w = reinterpret_cast<int*>(st);
    for (int i = threadIdx.x; i < (int)(sizeof(CGState) / sizeof(int)); i += blockDim.x) w[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
      st->t = 1;
      st->phase = PH_INIT;
    }
  }
}

}  // namespace cofem

using namespace cofem;

namespace {

cofem_status sfail(cofem_status s, const std::string& m) {
  set_error(m);
  return s;
}
#define SRV_TRY(expr)                                                                                   \
  do {                                                                                                 \
    hipError_t e_ = (expr);                                                                            \
    if (e_ != hipSuccess) return sfail(COFEM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

inline int64_t rup(int64_t x, int64_t m) { return ((x + m - 1) / m) * m; }
inline int cdivi(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

double wall_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Byte layout of one slot's workspace inside the arena.
struct SlotLayout {
  int64_t Np, Dp;
  int nrb1, splits1, nrb2, splits2;
  int64_t kchunk1, kchunk2;
  size_t off_phi, off_phiT, off_V, off_Yp, off_X, off_R, off_Pd, off_Psi, off_vec, off_y, off_part, off_pipart,
      off_st, off_log, off_rlog, total;
};

// kchunk: reduction length per split of both contractions (a multiple of 256).
SlotLayout layout_of(const cofem_params& p, int64_t kchunk = SRV_KCHUNK) {
  SlotLayout L{};
  L.Np = rup(p.N, 256);
  L.Dp = rup(p.D, 256);
  L.nrb1 = (int)(L.Np / (64 * SRV_RT));
  L.kchunk1 = std::min<int64_t>(kchunk, L.Dp);
  L.splits1 = cdivi(L.Dp, L.kchunk1);
  L.nrb2 = (int)(L.Dp / (64 * SRV_RT));
  L.kchunk2 = std::min<int64_t>(kchunk, L.Np);
  L.splits2 = cdivi(L.Np, L.kchunk2);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += (size_t)rup((int64_t)bytes, 256);
    return at;
  };
  const size_t nd = (size_t)L.Np * (size_t)L.Dp * sizeof(float);
  L.off_phi = take(nd);
  L.off_phiT = take(nd);
  L.off_V = take((size_t)SRV_QP * L.Np * sizeof(float));
  L.off_Yp = take((size_t)SRV_QP * std::max<int64_t>(L.splits1 * L.Np, L.splits2 * L.Dp) * sizeof(float));
  L.off_X = take((size_t)SRV_QP * L.Dp * sizeof(float));
  L.off_R = take((size_t)SRV_QP * L.Dp * sizeof(float));
  L.off_Pd = take((size_t)SRV_QP * L.Dp * sizeof(float));
  L.off_Psi = take((size_t)SRV_QP * L.Dp * sizeof(float));
  L.off_vec = take((size_t)6 * L.Dp * sizeof(float));  // minv, alpha, b, theta, mu, s
  L.off_y = take((size_t)L.Np * sizeof(float));
  L.off_part = take((size_t)(L.Dp / VPART + 1) * 2 * QMAX * sizeof(double));
  L.off_pipart = take((size_t)(L.Dp / VPART + 1) * QMAX * sizeof(double));
  L.off_st = take(sizeof(CGState));
  L.off_log = take((size_t)p.T * sizeof(int));
  L.off_rlog = take((size_t)p.T * sizeof(double));
  L.total = o;
  return L;
}

// First-fit allocator over [0, size) with coalescing.
struct Arena {
  size_t size = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  void init(size_t n) {
    size = n;
    free_.clear();
    free_[0] = n;
  }
  bool alloc(size_t n, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n, at = it->first + n;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct Request {
  cofem_params p;
  const float* phi = nullptr;
  const float* y = nullptr;
  int state = COFEM_REQ_PENDING;
  double t_submit = 0, t_admit = 0, t_finish = 0;
  size_t bytes = 0, off = 0;
  int slot = -1;
  int total_steps = 0;
  std::vector<float> mu, s, alpha;
};

}  // namespace

struct cofem_server {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int max_slots = 0, steps = 1;
  char* arena_base = nullptr;
  Arena arena;
  SlotDev* d_slots = nullptr;
  SrvTable* d_table = nullptr;
  int* d_phase = nullptr;
  int* d_ctr = nullptr;  // tile counters: two per CG step of a tick
  // Ticks are pipelined: a step launches the next tick and then reads the previous one's
  // phases, so the host's work overlaps a running tick.  Per tick buffer b: the phases
  // (pinned), the events around the graph and after the phase copy, and the table
  // positions' slots and requests at launch.
  int* h_phase[2] = {nullptr, nullptr};
  SrvTable* h_table_up[2] = {nullptr, nullptr};  // pinned staging of the table uploads
  int table_buf = 0;
  struct Tick {
    int n = 0;
    int slot[SRV_MAXSLOTS];
    int64_t rid[SRV_MAXSLOTS];
  } tick[2];
  int tick_buf = 0;       // buffer of the next launch
  int tick_pending = -1;  // buffer of the launched tick whose phases are not read yet
  hipEvent_t ev_ph[2] = {nullptr, nullptr};
  SrvTable h_table{};
  std::vector<SlotDev> slot_dev;
  std::vector<int64_t> slot_req;  // request id per slot, -1 = free
  std::deque<int64_t> pending;
  std::unordered_map<int64_t, Request> reqs;
  int64_t next_id = 1;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  hipEvent_t ev_tick[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // around each tick's graph
  bool table_dirty = true;
  double t0 = 0;
  cofem_server_stats stats{};
};

namespace {

cofem_status validate_request(const cofem_params* p) {
  if (!p) return sfail(COFEM_EINVAL, "params is NULL");
  if (p->N < 1 || p->D < 1 || p->N > (int64_t(1) << 28) || p->D > (int64_t(1) << 28))
    return sfail(COFEM_EINVAL, "bad N or D");
  if (!(p->beta > 0.0) || !std::isfinite(p->beta)) return sfail(COFEM_EINVAL, "beta must be finite and > 0");
  if (p->K < 1 || p->K > SRV_QP - 1) return sfail(COFEM_EINVAL, "serving requests need 1 <= K <= 31");
  if (p->T < 1 || p->T > COFEM_MAX_T) return sfail(COFEM_EINVAL, "T must be in [1, COFEM_MAX_T]");
  if (p->U < 1) return sfail(COFEM_EINVAL, "U must be >= 1");
  if (!(p->tol >= 0.0) || !std::isfinite(p->tol)) return sfail(COFEM_EINVAL, "tol must be finite and >= 0");
  if (p->theta_mode != COFEM_THETA_ONES && p->theta_mode != COFEM_THETA_JACOBI)
    return sfail(COFEM_EINVAL, "bad theta_mode");
  if (p->stop_mode != COFEM_STOP_JOINT && p->stop_mode != COFEM_STOP_COLUMN) return sfail(COFEM_EINVAL, "bad stop_mode");
  if (p->op_kind != COFEM_OP_DENSE || p->phi_dtype != COFEM_PHI_FP32 || p->refine_last != 0)
    return sfail(COFEM_EINVAL, "serving requests are dense FP32 without refinement");
  if (!(p->alpha_floor > 0.0) || !std::isfinite(p->alpha_floor))
    return sfail(COFEM_EINVAL, "alpha_floor must be finite and > 0");
  if (p->mstep_mode != COFEM_MSTEP_GAUSSIAN && p->mstep_mode != COFEM_MSTEP_NONNEG)
    return sfail(COFEM_EINVAL, "bad mstep_mode");
  return COFEM_OK;
}

// One tick as a graph: E-step initialisation, `steps` CG steps, M-step, the alpha groups'
// joint M-step, EM advance.  ctr holds 2 * steps tile counters.
cofem_status capture_tick_graph(hipStream_t st, int steps, const SlotDev* slots, const SrvTable* tab, int* ctr,
                                int* phase, hipGraph_t* graph, hipGraphExec_t* exec) {
  SRV_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  hipLaunchKernelGGL(ks_reset_ctr, dim3(1), dim3(128), 0, st, ctr, 2 * steps);
  hipLaunchKernelGGL(ks_em_init, dim3(SRV_VEC_GRID), dim3(VBLOCK), 0, st, slots, tab);
  hipLaunchKernelGGL(ks_em_scalars, dim3(SRV_MAXSLOTS), dim3(VBLOCK), 0, st, slots, tab);
  for (int k = 0; k < steps; ++k) {
    hipLaunchKernelGGL(ks_gemm, dim3(SRV_GEMM_GRID), dim3(64 * GEMM_WAVES), 0, st, slots, tab, 1, ctr + 2 * k);
    hipLaunchKernelGGL(ks_finish1, dim3(SRV_VEC_GRID), dim3(VBLOCK), 0, st, slots, tab);
    hipLaunchKernelGGL(ks_gemm, dim3(SRV_GEMM_GRID), dim3(64 * GEMM_WAVES), 0, st, slots, tab, 2, ctr + 2 * k + 1);
    hipLaunchKernelGGL(ks_finish2, dim3(SRV_VEC_GRID), dim3(VBLOCK), 0, st, slots, tab);
    hipLaunchKernelGGL(ks_update, dim3(SRV_VEC_GRID), dim3(VBLOCK), 0, st, slots, tab);
    hipLaunchKernelGGL(ks_scalars_direction, dim3(SRV_VEC_GRID), dim3(VBLOCK), 0, st, slots, tab);
  }
  hipLaunchKernelGGL(ks_mstep, dim3(SRV_VEC_GRID), dim3(VBLOCK), 0, st, slots, tab);
  hipLaunchKernelGGL(ks_group_alpha, dim3(SRV_VEC_GRID), dim3(VBLOCK), 0, st, slots, tab);
  hipLaunchKernelGGL(ks_advance, dim3(1), dim3(SRV_MAXSLOTS), 0, st, slots, tab, phase);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(st, &g);
  if (e != hipSuccess) return sfail(COFEM_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  *graph = g;
  SRV_TRY(hipGraphInstantiate(exec, g, nullptr, nullptr, 0));
  return COFEM_OK;
}

cofem_status capture_tick(cofem_server* s) {
  return capture_tick_graph(s->stream, s->steps, s->d_slots, s->d_table, s->d_ctr, s->d_phase, &s->graph, &s->exec);
}

void destroy_server(cofem_server* s) {
  if (!s) return;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  if (s->exec) (void)hipGraphExecDestroy(s->exec);
  if (s->graph) (void)hipGraphDestroy(s->graph);
  if (s->arena_base) (void)hipFree(s->arena_base);
  if (s->d_slots) (void)hipFree(s->d_slots);
  if (s->d_table) (void)hipFree(s->d_table);
  if (s->d_phase) (void)hipFree(s->d_phase);
  if (s->d_ctr) (void)hipFree(s->d_ctr);
  for (int b = 0; b < 2; ++b) {
    if (s->h_phase[b]) (void)hipHostFree(s->h_phase[b]);
    if (s->h_table_up[b]) (void)hipHostFree(s->h_table_up[b]);
    for (hipEvent_t e : s->ev_tick[b])
      if (e) (void)hipEventDestroy(e);
    if (s->ev_ph[b]) (void)hipEventDestroy(s->ev_ph[b]);
  }
  if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

// The device description of a fit whose workspace (layout_of(p, kchunk)) starts at base.
SlotDev make_slot(const cofem_params& p, char* base, int64_t kchunk = SRV_KCHUNK) {
  const SlotLayout L = layout_of(p, kchunk);
  SlotDev sd{};
  sd.c.Q = p.K + 1;
  sd.c.Qp = SRV_QP;
  sd.x1 = sd.c.Q == 17 ? 1 : 0;
  sd.c.nonneg = p.mstep_mode == COFEM_MSTEP_NONNEG ? 1 : 0;
  sd.c.K = p.K;
  sd.c.U = p.U;
  sd.c.stop_mode = p.stop_mode;
  sd.c.tol = p.tol;
  sd.c.beta = p.beta;
  sd.N = p.N;
  sd.D = p.D;
  sd.Np = L.Np;
  sd.Dp = L.Dp;
  sd.T = p.T;
  sd.seed = p.seed;
  sd.floor = p.alpha_floor;
  sd.nrb1 = L.nrb1;
  sd.splits1 = L.splits1;
  sd.kchunk1 = L.kchunk1;
  sd.nrb2 = L.nrb2;
  sd.splits2 = L.splits2;
  sd.kchunk2 = L.kchunk2;
  sd.nbx = cdivi(L.Dp, VCHUNK);
  sd.nbn = cdivi(L.Np, VCHUNK);
  sd.phi = reinterpret_cast<float*>(base + L.off_phi);
  sd.phiT = reinterpret_cast<float*>(base + L.off_phiT);
  sd.V = reinterpret_cast<float*>(base + L.off_V);
  sd.Ypart = reinterpret_cast<float*>(base + L.off_Yp);
  sd.X = reinterpret_cast<float*>(base + L.off_X);
  sd.R = reinterpret_cast<float*>(base + L.off_R);
  sd.Pd = reinterpret_cast<float*>(base + L.off_Pd);
  sd.Psi = reinterpret_cast<float*>(base + L.off_Psi);
  float* vec = reinterpret_cast<float*>(base + L.off_vec);
  sd.minv = vec;
  sd.alpha = vec + L.Dp;
  sd.b = vec + 2 * L.Dp;
  sd.theta = vec + 3 * L.Dp;
  sd.mu = vec + 4 * L.Dp;
  sd.s = vec + 5 * L.Dp;
  sd.part = reinterpret_cast<double*>(base + L.off_part);
  sd.pipart = reinterpret_cast<double*>(base + L.off_pipart);
  sd.st = reinterpret_cast<CGState*>(base + L.off_st);
  sd.steps_log = reinterpret_cast<int*>(base + L.off_log);
  sd.resid_log = reinterpret_cast<double*>(base + L.off_rlog);
  sd.grp_first = 0;
  sd.grp_n = 0;
  return sd;
}

// Copy the request's inputs into its slot and prepare its first E-step.
cofem_status admit(cofem_server* s, int slot, Request& r) {
  const cofem_params& p = r.p;
  const SlotLayout L = layout_of(p);
  char* base = s->arena_base + r.off;
  const SlotDev sd = make_slot(p, base);
  float* phi = reinterpret_cast<float*>(base + L.off_phi);
  float* phiT = reinterpret_cast<float*>(base + L.off_phiT);
  float* yv = reinterpret_cast<float*>(base + L.off_y);
  const int64_t nd = L.Np * L.Dp;
  // zero the padded buffers the copies do not cover (V's padded rows and columns stay zero)
  hipLaunchKernelGGL(ks_zero, dim3(1024), dim3(256), 0, s->stream, phi, nd);
  hipLaunchKernelGGL(ks_zero, dim3(64), dim3(256), 0, s->stream, yv, L.Np);
  hipLaunchKernelGGL(ks_zero, dim3(256), dim3(256), 0, s->stream, sd.V, (int64_t)SRV_QP * L.Np);
  SRV_TRY(hipMemcpy2DAsync(phi, (size_t)L.Dp * sizeof(float), r.phi, (size_t)p.D * sizeof(float),
                           (size_t)p.D * sizeof(float), (size_t)p.N, hipMemcpyHostToDevice, s->stream));
  SRV_TRY(hipMemcpyAsync(yv, r.y, (size_t)p.N * sizeof(float), hipMemcpyHostToDevice, s->stream));
  hipLaunchKernelGGL(ks_transpose, dim3((unsigned)(L.Dp / 64), (unsigned)(L.Np / 64)), dim3(256), 0, s->stream, phi,
                     L.Np, L.Dp, phiT);
  hipLaunchKernelGGL(ks_theta, dim3((unsigned)cdivi(L.Dp, 256)), dim3(256), 0, s->stream, phi, L.Np, p.D, L.Dp,
                     p.theta_mode == COFEM_THETA_JACOBI ? 1 : 0, sd.theta);
  launch_rhs(phiT, nullptr, L.Np, L.Np, L.Dp, yv, p.beta, sd.b, s->stream);
  hipLaunchKernelGGL(ks_slot_start, dim3(64), dim3(256), 0, s->stream, sd.st, sd.alpha, L.Dp);
  SRV_TRY(hipGetLastError());
  // the caller's host buffers have been consumed once the copies above are done
  SRV_TRY(hipStreamSynchronize(s->stream));
  s->slot_dev[slot] = sd;
  SRV_TRY(hipMemcpyAsync(s->d_slots + slot, &s->slot_dev[slot], sizeof(SlotDev), hipMemcpyHostToDevice, s->stream));
  return COFEM_OK;
}

// Append slot i (described by sd) to the tile table.
void table_add(SrvTable& t, int i, const SlotDev& sd) {
  auto pad8 = [](int x) { return (x + 7) & ~7; };
  const int k = t.n++;
  t.slot[k] = i;
  t.em[k + 1] = t.em[k] + pad8((int)(sd.Dp / VBLOCK));
  t.g1[k + 1] = t.g1[k] + pad8(sd.nrb1 * sd.splits1);
  t.g2[k + 1] = t.g2[k] + pad8(sd.nrb2 * sd.splits2);
  t.f1[k + 1] = t.f1[k] + pad8(sd.nbn * SRV_QP);
  t.vq[k + 1] = t.vq[k] + pad8(sd.nbx * sd.c.Q);
}

void table_clear(SrvTable& t) {
  t.n = 0;
  t.em[0] = t.g1[0] = t.g2[0] = t.f1[0] = t.vq[0] = 0;
}

void rebuild_table(cofem_server* s) {
  table_clear(s->h_table);
  for (int i = 0; i < s->max_slots; ++i)
    if (s->slot_req[i] >= 0) table_add(s->h_table, i, s->slot_dev[i]);
}

}  // namespace

COFEM_API cofem_status cofem_server_create(size_t hbm_budget, int32_t max_slots, int32_t steps_per_tick, void* stream,
                                           cofem_server** out) {
  if (!out) return sfail(COFEM_EINVAL, "out is NULL");
  *out = nullptr;
  if (hbm_budget < (size_t(1) << 20)) return sfail(COFEM_EINVAL, "hbm_budget must be at least 1 MiB");
  if (max_slots < 1 || max_slots > SRV_MAXSLOTS) return sfail(COFEM_EINVAL, "max_slots must be in [1, 128]");
  if (steps_per_tick < 1 || steps_per_tick > 64) return sfail(COFEM_EINVAL, "steps_per_tick must be in [1, 64]");
  cofem_server* s = new (std::nothrow) cofem_server();
  if (!s) return sfail(COFEM_ENOMEM, "host allocation failed");
  s->max_slots = max_slots;
  s->steps = steps_per_tick;
  s->slot_dev.assign(SRV_MAXSLOTS, SlotDev{});
  s->slot_req.assign(SRV_MAXSLOTS, -1);
  s->t0 = wall_ms();
  auto bail = [&](cofem_status st, const char* what) {
    (void)hipGetLastError();
    destroy_server(s);
    return sfail(st, what);
  };
  if (stream) {
    s->stream = static_cast<hipStream_t>(stream);
  } else {
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess)
      return bail(COFEM_EDEVICE, "hipStreamCreate failed");
    s->own_stream = true;
  }
  if (hipMalloc((void**)&s->arena_base, hbm_budget) != hipSuccess) return bail(COFEM_ENOMEM, "arena allocation failed");
  s->arena.init(hbm_budget);
  if (hipMalloc((void**)&s->d_slots, sizeof(SlotDev) * SRV_MAXSLOTS) != hipSuccess ||
      hipMalloc((void**)&s->d_table, sizeof(SrvTable)) != hipSuccess ||
      hipMalloc((void**)&s->d_phase, sizeof(int) * SRV_MAXSLOTS) != hipSuccess ||
      hipMalloc((void**)&s->d_ctr, sizeof(int) * 2 * 64) != hipSuccess)  // steps_per_tick <= 64
    return bail(COFEM_ENOMEM, "server tables allocation failed");
  for (int b = 0; b < 2; ++b) {
    if (hipHostMalloc((void**)&s->h_phase[b], sizeof(int) * SRV_MAXSLOTS, hipHostMallocDefault) != hipSuccess) {
      s->h_phase[b] = nullptr;
      return bail(COFEM_ENOMEM, "pinned allocation failed");
    }
    if (hipHostMalloc((void**)&s->h_table_up[b], sizeof(SrvTable), hipHostMallocDefault) != hipSuccess) {
      s->h_table_up[b] = nullptr;
      return bail(COFEM_ENOMEM, "pinned allocation failed");
    }
    for (hipEvent_t& e : s->ev_tick[b])
      if (hipEventCreate(&e) != hipSuccess) {
        e = nullptr;
        return bail(COFEM_EDEVICE, "event creation failed");
      }
    if (hipEventCreateWithFlags(&s->ev_ph[b], hipEventDisableTiming) != hipSuccess) {
      s->ev_ph[b] = nullptr;
      return bail(COFEM_EDEVICE, "event creation failed");
    }
  }
  rebuild_table(s);
  if (hipMemcpyAsync(s->d_table, &s->h_table, sizeof(SrvTable), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
      hipStreamSynchronize(s->stream) != hipSuccess)
    return bail(COFEM_EDEVICE, "server table upload failed");
  s->table_dirty = false;
  cofem_status rc = capture_tick(s);
  if (rc != COFEM_OK) {
    destroy_server(s);
    return rc;
  }
  s->stats.budget = (int64_t)hbm_budget;
  *out = s;
  return COFEM_OK;
}

COFEM_API void cofem_server_destroy(cofem_server* s) { destroy_server(s); }

COFEM_API cofem_status cofem_server_submit(cofem_server* s, const cofem_params* p, const float* phi, const float* y,
                                           int64_t* id) {
  if (!s || !phi || !y || !id) return sfail(COFEM_EINVAL, "NULL argument");
  cofem_status rc = validate_request(p);
  if (rc != COFEM_OK) {
    s->stats.rejected++;
    return rc;
  }
  for (int64_t i = 0; i < p->N; ++i)
    if (!std::isfinite(y[i])) {
      s->stats.rejected++;
      return sfail(COFEM_EINVAL, "y[" + std::to_string(i) + "] is not finite");
    }
  const SlotLayout L = layout_of(*p);
  if (L.total > s->arena.size) {
    s->stats.rejected++;
    return sfail(COFEM_EBUDGET, "request workspace (" + std::to_string(L.total) + " bytes) exceeds the budget");
  }
  Request r;
  r.p = *p;
  r.phi = phi;
  r.y = y;
  r.bytes = L.total;
  r.t_submit = wall_ms() - s->t0;
  const int64_t rid = s->next_id++;
  s->reqs.emplace(rid, std::move(r));
  s->pending.push_back(rid);
  s->stats.submitted++;
  *id = rid;
  return COFEM_OK;
}

namespace {

// Read the phases of the launched tick in buffer b (waiting for it) and retire the
// requests it finished.  A slot whose request changed since the launch (cancelled, then
// perhaps re-admitted) is skipped.
cofem_status harvest_tick(cofem_server* s, int b) {
  SRV_TRY(hipEventSynchronize(s->ev_ph[b]));
  float tick_ms = 0.0f;
  SRV_TRY(hipEventElapsedTime(&tick_ms, s->ev_tick[b][0], s->ev_tick[b][1]));
  s->stats.tick_ms += tick_ms;
  s->stats.ticks++;
  const cofem_server::Tick& t = s->tick[b];
  for (int k = 0; k < t.n; ++k) {
    if (s->h_phase[b][k] != PH_DONE) continue;
    const int slot = t.slot[k];
    const int64_t rid = t.rid[k];
    if (s->slot_req[slot] != rid) continue;
    Request& r = s->reqs[rid];
    const SlotDev& sd = s->slot_dev[slot];
    r.mu.resize((size_t)r.p.D);
    r.s.resize((size_t)r.p.D);
    r.alpha.resize((size_t)r.p.D);
    const size_t bytes = (size_t)r.p.D * sizeof(float);
    CGState st;
    // a finished slot is left alone by every kernel, so its results are final; the copies
    // queue behind the tick launched since, which this waits for
    SRV_TRY(hipMemcpyAsync(r.mu.data(), sd.mu, bytes, hipMemcpyDeviceToHost, s->stream));
    SRV_TRY(hipMemcpyAsync(r.s.data(), sd.s, bytes, hipMemcpyDeviceToHost, s->stream));
    SRV_TRY(hipMemcpyAsync(r.alpha.data(), sd.alpha, bytes, hipMemcpyDeviceToHost, s->stream));
    SRV_TRY(hipMemcpyAsync(&st, sd.st, sizeof(CGState), hipMemcpyDeviceToHost, s->stream));
    SRV_TRY(hipStreamSynchronize(s->stream));
    r.total_steps = st.total_steps;
    s->stats.dict_bytes += (double)st.total_steps * 2.0 * (double)r.p.N * (double)r.p.D * sizeof(float);
    r.state = COFEM_REQ_DONE;
    r.t_finish = wall_ms() - s->t0;
    s->arena.release(r.off, r.bytes);
    s->stats.bytes_in_use -= (int64_t)r.bytes;
    s->slot_req[slot] = -1;
    s->stats.completed++;
    s->table_dirty = true;
  }
  return COFEM_OK;
}

}  // namespace

COFEM_API cofem_status cofem_server_step(cofem_server* s, int32_t* n_running, int32_t* n_pending) {
  if (!s) return sfail(COFEM_EINVAL, "NULL server");
  // admission, first in first out (each admission waits for the stream: the copies of the
  // caller's host buffers must be done when it returns)
  while (!s->pending.empty()) {
    int slot = -1;
    for (int i = 0; i < s->max_slots; ++i)
      if (s->slot_req[i] < 0) {
        slot = i;
        break;
      }
    if (slot < 0) break;
    const int64_t rid = s->pending.front();
    Request& r = s->reqs[rid];
    size_t off = 0;
    if (!s->arena.alloc(r.bytes, &off)) break;
    r.off = off;
    cofem_status rc = admit(s, slot, r);
    if (rc != COFEM_OK) return rc;
    s->slot_req[slot] = rid;
    r.slot = slot;
    r.state = COFEM_REQ_RUNNING;
    r.phi = nullptr;
    r.y = nullptr;
    r.t_admit = wall_ms() - s->t0;
    s->pending.pop_front();
    s->stats.admitted++;
    s->stats.bytes_in_use += (int64_t)r.bytes;
    s->stats.bytes_peak = std::max(s->stats.bytes_peak, s->stats.bytes_in_use);
    s->table_dirty = true;
  }
  if (s->table_dirty) {
    rebuild_table(s);
    // staged in pinned memory: the upload runs behind the tick in flight, and the staging
    // buffer is not written again before that tick's phases have been read
    SrvTable* up = s->h_table_up[s->table_buf];
    s->table_buf ^= 1;
    std::memcpy(up, &s->h_table, sizeof(SrvTable));
    SRV_TRY(hipMemcpyAsync(s->d_table, up, sizeof(SrvTable), hipMemcpyHostToDevice, s->stream));
    s->table_dirty = false;
  }
  const int n = s->h_table.n;
  s->stats.active = n;
  s->stats.max_active = std::max(s->stats.max_active, n);
  int launched = -1;
  if (n > 0) {
    const int b = s->tick_buf;
    s->tick_buf ^= 1;
    SRV_TRY(hipEventRecord(s->ev_tick[b][0], s->stream));
    SRV_TRY(hipGraphLaunch(s->exec, s->stream));
    SRV_TRY(hipEventRecord(s->ev_tick[b][1], s->stream));
    SRV_TRY(hipMemcpyAsync(s->h_phase[b], s->d_phase, sizeof(int) * n, hipMemcpyDeviceToHost, s->stream));
    SRV_TRY(hipEventRecord(s->ev_ph[b], s->stream));
    cofem_server::Tick& t = s->tick[b];
    t.n = n;
    for (int k = 0; k < n; ++k) {
      t.slot[k] = s->h_table.slot[k];
      t.rid[k] = s->slot_req[t.slot[k]];
    }
    launched = b;
  }
  // the tick launched by the previous step (this one's, when the server went idle)
  const int prev = s->tick_pending;
  s->tick_pending = launched;
  if (prev >= 0) {
    cofem_status rc = harvest_tick(s, prev);
    if (rc != COFEM_OK) return rc;
  }
  int running = 0;
  for (int i = 0; i < s->max_slots; ++i) running += s->slot_req[i] >= 0;
  s->stats.active = running;
  if (n_running) *n_running = running;
  if (n_pending) *n_pending = (int32_t)s->pending.size();
  return COFEM_OK;
}

COFEM_API cofem_status cofem_server_poll(cofem_server* s, int64_t id, float* mu, float* s_out, float* alpha,
                                         cofem_request_info* info) {
  if (!s) return sfail(COFEM_EINVAL, "NULL server");
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) {
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->state = COFEM_REQ_UNKNOWN;
    }
    return sfail(COFEM_EINVAL, "unknown request id");
  }
  Request& r = it->second;
  if (info) {
    info->state = r.state;
    info->T = r.p.T;
    info->total_cg_steps = r.total_steps;
    info->pad_ = 0;
    info->t_submit_ms = r.t_submit;
    info->t_admit_ms = r.t_admit;
    info->t_finish_ms = r.t_finish;
    info->bytes = (int64_t)r.bytes;
  }
  if (r.state == COFEM_REQ_DONE) {
    const size_t bytes = (size_t)r.p.D * sizeof(float);
    if (mu) std::memcpy(mu, r.mu.data(), bytes);
    if (s_out) std::memcpy(s_out, r.s.data(), bytes);
    if (alpha) std::memcpy(alpha, r.alpha.data(), bytes);
    if (mu) s->reqs.erase(it);
  }
  return COFEM_OK;
}

COFEM_API cofem_status cofem_server_cancel(cofem_server* s, int64_t id) {
  if (!s) return sfail(COFEM_EINVAL, "NULL server");
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return sfail(COFEM_EINVAL, "unknown request id");
  Request& r = it->second;
  if (r.state == COFEM_REQ_PENDING) {
    s->pending.erase(std::find(s->pending.begin(), s->pending.end(), id));
  } else if (r.state == COFEM_REQ_RUNNING) {
    // its slot and arena bytes are handed back at once: a tick still in flight may run
    // this request's tiles, but everything that reuses the bytes (a later admission's
    // copies and kernels, the next table) is queued behind that tick on the server's
    // stream, and the tick's phases are not read for a slot whose request changed
    s->arena.release(r.off, r.bytes);
    s->stats.bytes_in_use -= (int64_t)r.bytes;
    s->slot_req[r.slot] = -1;
    s->table_dirty = true;
  }
  s->reqs.erase(it);
  return COFEM_OK;
}

COFEM_API cofem_status cofem_server_get_stats(cofem_server* s, cofem_server_stats* out) {
  if (!s || !out) return sfail(COFEM_EINVAL, "NULL argument");
  *out = s->stats;
  return COFEM_OK;
}

// ---------------------------------------------------------------------------
// Batched multi-task fit (Sec. III-E.1): the L tasks are the slots 0 .. L - 1 of one
// alpha group, so every CG step of all L(K + 1) systems is one launch per phase
// (two contraction launches over every task's tiles, the vector kernels over every
// task's columns), each task keeping its own stop rule, and the joint M-step runs on
// the device once all L E-steps of an EM iteration have ended.
// ---------------------------------------------------------------------------
namespace cofem {

struct MtBatch {
  hipStream_t stream = nullptr;
  cofem_params p{};
  int L = 0;
  int steps = 8;           // CG steps per graph launch
  int64_t kchunk = SRV_KCHUNK;
  SlotLayout lay{};
  char* arena = nullptr;   // L slot workspaces, then the shared alpha
  float* alpha = nullptr;
  SlotDev* d_slots = nullptr;
  SrvTable* d_table = nullptr;
  int* d_ctr = nullptr;
  int* d_phase = nullptr;
  int* d_count = nullptr;  // non-finite entries found by the last check
  int* h_phase[2] = {nullptr, nullptr};  // pinned, one per launch in flight
  hipEvent_t ev_ph[2] = {nullptr, nullptr};
  std::vector<SlotDev> sd;
  std::vector<char> loaded;
  std::vector<double> ms_setup;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<CGState> h_st;
  std::vector<std::vector<int>> steps_log;
  std::vector<std::vector<double>> resid_log;
  double ms_fit = 0.0;
  bool fitted = false;
};

bool mtb_eligible(const cofem_params& p) {
  return p.op_kind == COFEM_OP_DENSE && p.phi_dtype == COFEM_PHI_FP32 && p.refine_last == 0 && p.K >= 1 &&
         p.K <= SRV_QP - 1 && p.mstep_mode == COFEM_MSTEP_GAUSSIAN;
}

void mtb_destroy(MtBatch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->arena) (void)hipFree(b->arena);
  if (b->d_slots) (void)hipFree(b->d_slots);
  if (b->d_table) (void)hipFree(b->d_table);
  if (b->d_ctr) (void)hipFree(b->d_ctr);
  if (b->d_phase) (void)hipFree(b->d_phase);
  if (b->d_count) (void)hipFree(b->d_count);
  for (int i = 0; i < 2; ++i) {
    if (b->h_phase[i]) (void)hipHostFree(b->h_phase[i]);
    if (b->ev_ph[i]) (void)hipEventDestroy(b->ev_ph[i]);
  }
  delete b;
}

cofem_status mtb_create(const cofem_params& p, int L, hipStream_t stream, MtBatch** out) {
  *out = nullptr;
  if (!mtb_eligible(p))
    return sfail(COFEM_EINVAL, "the batched multi-task fit takes dense FP32 dictionaries, no refinement, K <= 31");
  if (L < 1 || L > SRV_MAXSLOTS) return sfail(COFEM_EINVAL, "bad task count");
  MtBatch* b = new (std::nothrow) MtBatch();
  if (!b) return sfail(COFEM_ENOMEM, "host allocation failed");
  b->stream = stream;
  b->p = p;
  b->L = L;
  // split the contractions finer until each launch has about two tiles per persistent
  // block (the tasks' tiles together), down to 256-long reductions
  auto tiles = [&](int64_t kc) {
    const SlotLayout t = layout_of(p, kc);
    return (int64_t)L * std::min<int64_t>((int64_t)t.nrb1 * t.splits1, (int64_t)t.nrb2 * t.splits2);
  };
  while (b->kchunk > 256 && tiles(b->kchunk) < 2 * SRV_GEMM_GRID) b->kchunk /= 2;
  b->lay = layout_of(p, b->kchunk);
  auto bail = [&](cofem_status st, const char* what) {
    (void)hipGetLastError();
    mtb_destroy(b);
    return sfail(st, what);
  };
  const size_t per = b->lay.total;
  if (hipMalloc((void**)&b->arena, per * L + (size_t)b->lay.Dp * sizeof(float)) != hipSuccess)
    return bail(COFEM_ENOMEM, "task workspace allocation failed");
  b->alpha = reinterpret_cast<float*>(b->arena + per * L);
  if (hipMalloc((void**)&b->d_slots, sizeof(SlotDev) * SRV_MAXSLOTS) != hipSuccess ||
      hipMalloc((void**)&b->d_table, sizeof(SrvTable)) != hipSuccess ||
      hipMalloc((void**)&b->d_phase, sizeof(int) * SRV_MAXSLOTS) != hipSuccess ||
      hipMalloc((void**)&b->d_ctr, sizeof(int) * 2 * b->steps) != hipSuccess ||
      hipMalloc((void**)&b->d_count, sizeof(int)) != hipSuccess)
    return bail(COFEM_ENOMEM, "task tables allocation failed");
  for (int i = 0; i < 2; ++i) {
    if (hipHostMalloc((void**)&b->h_phase[i], sizeof(int) * SRV_MAXSLOTS, hipHostMallocDefault) != hipSuccess) {
      b->h_phase[i] = nullptr;
      return bail(COFEM_ENOMEM, "pinned allocation failed");
    }
    if (hipEventCreateWithFlags(&b->ev_ph[i], hipEventDisableTiming) != hipSuccess) {
      b->ev_ph[i] = nullptr;
      return bail(COFEM_EDEVICE, "event creation failed");
    }
  }
  SrvTable tab;
  table_clear(tab);
  for (int l = 0; l < L; ++l) {
    cofem_params q = p;
    q.seed = p.seed + (uint64_t)l;  // task l's probes
    SlotDev sd = make_slot(q, b->arena + per * l, b->kchunk);
    sd.alpha = b->alpha;
    sd.grp_first = 0;
    sd.grp_n = L;
    b->sd.push_back(sd);
    table_add(tab, l, sd);
  }
  b->loaded.assign(L, 0);
  b->ms_setup.assign(L, 0.0);
  if (hipMemcpyAsync(b->d_slots, b->sd.data(), sizeof(SlotDev) * L, hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(b->d_table, &tab, sizeof(SrvTable), hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return bail(COFEM_EDEVICE, "task table upload failed");
  // capture on a stream of our own (the caller's may be the legacy default stream, which
  // cannot capture); the graph is launched on the caller's stream
  hipStream_t cap = nullptr;
  if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
    return bail(COFEM_EDEVICE, "hipStreamCreate failed");
  cofem_status rc = capture_tick_graph(cap, b->steps, b->d_slots, b->d_table, b->d_ctr, b->d_phase, &b->graph,
                                       &b->exec);
  (void)hipStreamDestroy(cap);
  if (rc != COFEM_OK) {
    mtb_destroy(b);
    return rc;
  }
  *out = b;
  return COFEM_OK;
}

// Count the non-finite entries of x[0 .. n) on the stream; an error names `what`.
static cofem_status mtb_check_finite(MtBatch* b, const float* x, int64_t n, const std::string& what) {
  SRV_TRY(hipMemsetAsync(b->d_count, 0, sizeof(int), b->stream));
  launch_count_nonfinite(x, n, b->d_count, b->stream);
  int bad = 0;
  SRV_TRY(hipMemcpyAsync(&bad, b->d_count, sizeof(int), hipMemcpyDeviceToHost, b->stream));
  SRV_TRY(hipStreamSynchronize(b->stream));
  if (bad > 0)
    return sfail(COFEM_EINVAL, what + " has " + std::to_string(bad) + " non-finite entries (NaN or infinity)");
  return COFEM_OK;
}

cofem_status mtb_set_dictionary(MtBatch* b, int task, const float* phi) {
  if (task < 0 || task >= b->L || !phi) return sfail(COFEM_EINVAL, "bad task or NULL dictionary");
  const double t0 = wall_ms();
  const SlotLayout& L = b->lay;
  const cofem_params& p = b->p;
  char* base = b->arena + L.total * task;
  float* ph = reinterpret_cast<float*>(base + L.off_phi);
  float* phT = reinterpret_cast<float*>(base + L.off_phiT);
  b->loaded[task] = 0;
  b->fitted = false;
  hipLaunchKernelGGL(ks_zero, dim3(1024), dim3(256), 0, b->stream, ph, L.Np * L.Dp);
  SRV_TRY(hipMemcpy2DAsync(ph, (size_t)L.Dp * sizeof(float), phi, (size_t)p.D * sizeof(float),
                           (size_t)p.D * sizeof(float), (size_t)p.N, hipMemcpyDeviceToDevice, b->stream));
  cofem_status rc = mtb_check_finite(b, ph, L.Np * L.Dp, "the dictionary");
  if (rc != COFEM_OK) return rc;
  hipLaunchKernelGGL(ks_transpose, dim3((unsigned)(L.Dp / 64), (unsigned)(L.Np / 64)), dim3(256), 0, b->stream, ph,
                     L.Np, L.Dp, phT);
  hipLaunchKernelGGL(ks_theta, dim3((unsigned)cdivi(L.Dp, 256)), dim3(256), 0, b->stream, ph, L.Np, p.D, L.Dp,
                     p.theta_mode == COFEM_THETA_JACOBI ? 1 : 0, b->sd[task].theta);
  SRV_TRY(hipGetLastError());
  SRV_TRY(hipStreamSynchronize(b->stream));
  b->loaded[task] = 1;
  b->ms_setup[task] = wall_ms() - t0;
  return COFEM_OK;
}

cofem_status mtb_fit(MtBatch* b, const float* const* ys) {
  const cofem_params& p = b->p;
  const SlotLayout& L = b->lay;
  for (int l = 0; l < b->L; ++l) {
    if (!ys[l]) return sfail(COFEM_EINVAL, "NULL observation");
    if (!b->loaded[l]) return sfail(COFEM_ESTATE, "cofem_mt_fit before every task has a dictionary");
  }
  const double t0 = wall_ms();
  b->fitted = false;
  for (int l = 0; l < b->L; ++l) {
    const SlotDev& sd = b->sd[l];
    float* yv = reinterpret_cast<float*>(b->arena + L.total * l + L.off_y);
    hipLaunchKernelGGL(ks_zero, dim3(64), dim3(256), 0, b->stream, yv, L.Np);
    SRV_TRY(hipMemcpyAsync(yv, ys[l], (size_t)p.N * sizeof(float), hipMemcpyDeviceToDevice, b->stream));
    cofem_status rc = mtb_check_finite(b, yv, p.N, "ys[" + std::to_string(l) + "]");
    if (rc != COFEM_OK) return rc;
    hipLaunchKernelGGL(ks_zero, dim3(256), dim3(256), 0, b->stream, sd.V, (int64_t)SRV_QP * L.Np);
    launch_rhs(sd.phiT, nullptr, L.Np, L.Np, L.Dp, yv, p.beta, sd.b, b->stream);
    hipLaunchKernelGGL(ks_slot_start, dim3(64), dim3(256), 0, b->stream, sd.st, b->alpha, L.Dp);
  }
  SRV_TRY(hipGetLastError());
  // each E-step takes at most ceil(U / steps) + 1 launches (its first starts with the
  // E-step initialisation), and the tasks advance together
  const int64_t limit = (int64_t)p.T * ((p.U + b->steps - 1) / b->steps + 2) + 2;
  // pipelined: launch k + 1 is queued before the phases of launch k are read, so the
  // device never waits for the host; the launch queued after the last one that mattered
  // finds every task DONE and does nothing (every kernel skips a finished slot)
  auto launch = [&](int64_t k) -> cofem_status {
    const int i = (int)(k & 1);
    SRV_TRY(hipGraphLaunch(b->exec, b->stream));
    SRV_TRY(hipMemcpyAsync(b->h_phase[i], b->d_phase, sizeof(int) * b->L, hipMemcpyDeviceToHost, b->stream));
    SRV_TRY(hipEventRecord(b->ev_ph[i], b->stream));
    return COFEM_OK;
  };
  cofem_status lrc = launch(0);
  if (lrc != COFEM_OK) return lrc;
  bool done = false;
  for (int64_t tick = 0; tick < limit && !done; ++tick) {
    if (tick + 1 < limit && (lrc = launch(tick + 1)) != COFEM_OK) return lrc;
    const int i = (int)(tick & 1);
    SRV_TRY(hipEventSynchronize(b->ev_ph[i]));
    done = true;
    for (int l = 0; l < b->L; ++l) done = done && b->h_phase[i][l] == PH_DONE;
  }
  if (!done) return sfail(COFEM_EDEVICE, "batched multi-task fit did not finish within its launch bound");
  b->h_st.assign(b->L, CGState{});
  b->steps_log.assign(b->L, std::vector<int>(p.T));
  b->resid_log.assign(b->L, std::vector<double>(p.T));
  for (int l = 0; l < b->L; ++l) {
    const SlotDev& sd = b->sd[l];
    SRV_TRY(hipMemcpyAsync(&b->h_st[l], sd.st, sizeof(CGState), hipMemcpyDeviceToHost, b->stream));
    SRV_TRY(hipMemcpyAsync(b->steps_log[l].data(), sd.steps_log, sizeof(int) * p.T, hipMemcpyDeviceToHost, b->stream));
    SRV_TRY(hipMemcpyAsync(b->resid_log[l].data(), sd.resid_log, sizeof(double) * p.T, hipMemcpyDeviceToHost,
                           b->stream));
  }
  SRV_TRY(hipStreamSynchronize(b->stream));
  b->ms_fit = wall_ms() - t0;
  b->fitted = true;
  for (int l = 0; l < b->L; ++l) {
    const CGState& st = b->h_st[l];
    // the mu column can only be inactive in joint mode through a breakdown
    if (st.active[0] == 0 && st.breakdown > 0 && p.stop_mode == COFEM_STOP_JOINT)
      return sfail(COFEM_EBREAKDOWN, "CG breakdown in the mu column of task " + std::to_string(l));
  }
  return COFEM_OK;
}

cofem_status mtb_posterior(MtBatch* b, int task, float* mu, float* s, float* alpha, cofem_stats* st) {
  if (task < 0 || task >= b->L) return sfail(COFEM_EINVAL, "bad task");
  if (!b->fitted) return sfail(COFEM_ESTATE, "cofem_mt_posterior before a successful cofem_mt_fit");
  const SlotDev& sd = b->sd[task];
  const size_t bytes = (size_t)b->p.D * sizeof(float);
  if (mu) SRV_TRY(hipMemcpyAsync(mu, sd.mu, bytes, hipMemcpyDeviceToDevice, b->stream));
  if (s) SRV_TRY(hipMemcpyAsync(s, sd.s, bytes, hipMemcpyDeviceToDevice, b->stream));
  if (alpha) SRV_TRY(hipMemcpyAsync(alpha, b->alpha, bytes, hipMemcpyDeviceToDevice, b->stream));
  if (st) {
    std::memset(st, 0, sizeof(*st));
    const CGState& h = b->h_st[task];
    st->T = b->p.T;
    for (int t = 0; t < b->p.T; ++t) {
      st->cg_steps[t] = b->steps_log[task][t];
      st->rel_resid[t] = b->resid_log[task][t];
    }
    st->clamped = h.clamped;
    st->breakdown = h.breakdown;
    st->total_cg_steps = h.total_steps;
    st->ms_setup = b->ms_setup[task];
    st->ms_fit = b->ms_fit;
  }
  SRV_TRY(hipStreamSynchronize(b->stream));
  return COFEM_OK;
}

}  // namespace cofem
