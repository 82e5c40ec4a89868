// gfx950 kernels of the CoFEM hot path.
//
// Layouts (all padded with zeros; Np, Dp are multiples of 256, Qp of 16):
//   dictionary  phi (Np x Dp) and phiT (Dp x Np), row-major, FP32 and/or bf16
//   CG blocks   X, R, Pd, Psi: Qp x Dp ("column q" = Dp contiguous floats)
//   V           Qp x Np
// Column 0 is the mu system (right-hand side beta Phi^T y), columns 1..K the
// probe systems, columns K+1..Qp-1 stay exactly zero.
//
// The operator Psi = beta Phi^T (Phi Pd) + alpha Pd (the line "Psi <- A P" of
// Algorithm 2) is two skinny contractions, each streaming one dictionary
// layout once with every right-hand side riding along: MFMA tiles whose
// matrix operand is read straight from HBM into VGPRs in the 16x16xK operand
// layout (the reduction index is contiguous in both layouts, so no LDS
// transpose is needed), with the right-hand-side block staged through LDS by
// LDS DMA loads.  The per-block work lives in tiles.h, shared with the serving
// kernels.
#include <algorithm>

#include "kernels.h"
#include "tiles.h"

namespace cofem {

// ---------------------------------------------------------------------------
// setup kernels
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_dict_layouts(const float* __restrict__ phi, int64_t N, int64_t D,
                                                      int64_t Np, int64_t Dp, int64_t kc16, float* __restrict__ phi32,
                                                      float* __restrict__ phi32T, uint16_t* __restrict__ phi16,
                                                      uint16_t* __restrict__ phi16T) {
  const int64_t ld32 = dict_ld(Dp, 4), ld32T = dict_ld(Np, 4), ld16T = dict_ld(Np, 2);
  __shared__ float tile[64][65];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t j0 = (int64_t)blockIdx.x * 64, i0 = (int64_t)blockIdx.y * 64;
  for (int r = ty; r < 64; r += 4) {
    const int64_t i = i0 + r, j = j0 + tx;
    const float v = (i < N && j < D) ? phi[i * D + j] : 0.0f;
    if (phi32) phi32[i * ld32 + j] = v;
    if (phi16) {
      const int64_t sp = j / kc16;  // split-blocked: split sp holds columns [sp kc16, (sp + 1) kc16)
      phi16[sp * Np * kc16 + i * kc16 + (j - sp * kc16)] = bf16_rne(v);
    }
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int64_t j = j0 + r, i = i0 + tx;
    const float v = tile[tx][r];
    if (phi32T) phi32T[j * ld32T + i] = v;
    if (phi16T) phi16T[j * ld16T + i] = bf16_rne(v);
  }
}

// theta_j = sum_i Phi_ij^2 (Jacobi) or 1, from the caller's N x D FP32 matrix; padding 1.
__global__ __launch_bounds__(256) void k_theta(const float* __restrict__ phi, int64_t N, int64_t D, int64_t Dp,
                                               int jacobi, float* __restrict__ theta) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= Dp) return;
  if (j >= D || !jacobi) {
    theta[j] = 1.0f;
    return;
  }
  double sq = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    const double v = (double)phi[i * D + j];
    sq += v * v;
  }
  theta[j] = (float)sq;
}

// b_j = beta * sum_i PhiT[j, i] y_i (FP64 sums), one wave per row of the
// transposed layout; padded rows are zero, so padding of b is zero.
template <class T>
__device__ __forceinline__ double ld_val(const T* p, int64_t i);
template <>
__device__ __forceinline__ double ld_val<float>(const float* p, int64_t i) { return (double)p[i]; }
template <>
__device__ __forceinline__ double ld_val<uint16_t>(const uint16_t* p, int64_t i) { return (double)bf16_val(p[i]); }

template <class T>
__global__ __launch_bounds__(256) void k_rhs(const T* __restrict__ MT, int64_t ld, int64_t Np, int64_t Dp,
                                             const float* __restrict__ y, double beta, float* __restrict__ b) {
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int ln = threadIdx.x & 63;
  if (j >= Dp) return;
  const T* row = MT + j * ld;
  double acc = 0.0;
  for (int64_t i = ln; i < Np; i += 64) acc += ld_val<T>(row, i) * (double)y[i];
  acc = wave_sum(acc);
  if (ln == 0) b[j] = (float)(beta * acc);
}

__global__ void k_fill(float* x, float v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ __launch_bounds__(256) void k_count_nonfinite(const float* __restrict__ x, int64_t n,
                                                         int* __restrict__ count) {
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    bad += __builtin_isfinite(x[i]) ? 0 : 1;
  if (bad) atomicAdd(count, bad);
}

__global__ void k_axpy(float* __restrict__ y, const float* __restrict__ x, float a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}

__global__ void k_state_reset(CGState* st, int Q) {
  int* w = reinterpret_cast<int*>(st);
  const int n = (int)(sizeof(CGState) / sizeof(int));
  for (int i = threadIdx.x; i < n; i += blockDim.x) w[i] = 0;
}

// ---------------------------------------------------------------------------
// single-problem kernels: one problem per launch, tile = block index
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(VBLOCK) void k_em_init(SolveCfg c, uint64_t key, int64_t D, int64_t Dp,
                                                    const float* __restrict__ b, const float* __restrict__ theta,
                                                    const float* __restrict__ alpha, float* __restrict__ minv,
                                                    float* __restrict__ X, float* __restrict__ R,
                                                    float* __restrict__ Pd, uint16_t* __restrict__ PdH,
                                                    uint16_t* __restrict__ PdL, uint16_t* __restrict__ PdX,
                                                    double* __restrict__ part) {
  em_init_block(c, key, D, Dp, blockIdx.x, b, theta, alpha, minv, X, R, Pd, PdH, PdL, PdX, part);
}

__global__ __launch_bounds__(VBLOCK) void k_em_scalars(SolveCfg c, int64_t D, int nblk,
                                                       const double* __restrict__ part, CGState* __restrict__ st) {
  em_scalars_block(c, D, nblk, part, st);
}

__global__ __launch_bounds__(VBLOCK) void k_mstep(SolveCfg c, uint64_t key, int64_t D, int64_t Dp,
                                                  const float* __restrict__ X, float* __restrict__ mu,
                                                  float* __restrict__ s_out, float* __restrict__ alpha,
                                                  double floor, int do_mstep, CGState* __restrict__ st) {
  mstep_block(c, key, D, Dp, blockIdx.x, X, mu, s_out, alpha, floor, do_mstep, st);
}

template <int RT, int CT, int KS, bool X1>
__global__ __launch_bounds__(64 * GEMM_WAVES, 2) void k_gemm_bf16(const uint16_t* __restrict__ M, int64_t ldm,
                                                      int64_t sps, const uint16_t* __restrict__ ZH,
                                                      const uint16_t* __restrict__ ZL, int64_t ldz,
                                                      float* __restrict__ Yp, int64_t ldy, int Qp, int64_t kchunk,
                                                      int64_t kdim, int nrb, int splits,
                                                      const int* __restrict__ done) {
  if (done && *done) return;
  gemm_bf16_tile<RT, CT, KS, X1>(blockIdx.x, M, ldm, ZH, ZL, ldz, Yp, ldy, Qp, kchunk, kdim, nrb, splits, sps);
}

template <int RT, int CT, int KS, bool X1>
__global__ __launch_bounds__(64 * GEMM_WAVES, 2) void k_gemm_f32(const float* __restrict__ M, int64_t ldm,
                                                     const uint16_t* __restrict__ ZH, const uint16_t* __restrict__ ZM,
                                                     const uint16_t* __restrict__ ZL, int64_t ldz,
                                                     float* __restrict__ Yp, int64_t ldy, int Qp, int64_t kchunk,
                                                     int64_t kdim, int nrb, int splits,
                                                     const int* __restrict__ done) {
  if (done && *done) return;
  gemm_f32s_tile<RT, CT, KS, X1>(blockIdx.x, M, ldm, ZH, ZM, ZL, ldz, Yp, ldy, Qp, kchunk, kdim, nrb, splits);
}

__global__ __launch_bounds__(256) void k_finish_pass1(const float* __restrict__ Yp, int splits, int64_t Np,
                                                      float* __restrict__ V, uint16_t* __restrict__ VH,
                                                      uint16_t* __restrict__ VL, uint16_t* __restrict__ VX, int Qp,
                                                      const int* __restrict__ done) {
  if (*done) return;
  finish1_tile(blockIdx.x, blockIdx.y, Yp, splits, Np, V, VH, VL, Qp, VX);
}

__global__ __launch_bounds__(VBLOCK) void k_finish_pass2(SolveCfg c, const float* __restrict__ Yp, int splits,
                                                         int64_t Dp, const float* __restrict__ alpha,
                                                         const float* __restrict__ Pd, float* __restrict__ Psi,
                                                         double* __restrict__ pipart, const CGState* __restrict__ st) {
  if (st->done) return;
  finish2_tile(c, blockIdx.x, blockIdx.y, gridDim.x, Yp, splits, Dp, alpha, Pd, Psi, pipart);
}

template <bool PRE, bool NT, bool XU>
__global__ __launch_bounds__(VBLOCK) void k_cg_update(SolveCfg c, int64_t Dp, const float* __restrict__ minv,
                                                      float* __restrict__ X, float* __restrict__ R,
                                                      const float* __restrict__ Pd, const float* __restrict__ Psi,
                                                      const double* __restrict__ pipart, double* __restrict__ part,
                                                      CGState* __restrict__ st) {
  cg_update_tile<PRE, NT, XU>(c, blockIdx.x, blockIdx.y, gridDim.x, Dp, minv, X, R, Pd, Psi, pipart, part, st,
                              &st->done);
}

// gamma_q for all columns into the state, for problems with many pi partials per column
// (the update tiles then read gamma instead of each re-reducing the partials): one
// single-wave block per column, 16 of a lane's loads in flight at once.
__global__ __launch_bounds__(64) void k_cg_gamma(SolveCfg c, int nbx, const double* __restrict__ pipart,
                                                 CGState* __restrict__ st) {
  if (st->done) return;
  column_gamma<16>(blockIdx.x, nbx, pipart, st, true);
}

// The CG scalars as a launch of their own (before the FIR dictionary's interleaved-slice
// direction kernel): one block, 16 of a lane's loads in flight at once (one block per
// launch, so its registers cost no occupancy).
__global__ __launch_bounds__(1024) void k_cg_scalars(SolveCfg c, int nbx, const double* __restrict__ part,
                                                     CGState* __restrict__ st) {
  if (st->done) return;
  cg_scalars_block<16>(c, nbx, part, st);
}

// The CG scalars and the direction update in one launch (column-major directions).  Row 0
// of the grid is the scalars: its block (0, 0) runs cg_scalars_block (the state's norms,
// stop rule, step count, done flag, new rho), dispatched first and beside the direction
// tiles rather than after one of them.  Rows 1 .. Q are the direction tiles: every block
// reduces its own column's rho' partials, in the order of cg_scalars_block, for
// eta_q = rho'_q / rho_q, with rho_q from rho_prev (recorded by the update with gamma, so
// the scalars may write the new rho while the tiles run).  A tile that starts after this
// step's stop rule has fired may skip its work: the direction is not used again in the
// E-step.  A tile's loads (its slice of R, Pd and M^-1, its column's partials, the old rho)
// go out before the done flag is tested and before the reduction, so the launch waits for
// memory once; the flag is read once per block (the scalars block may write it meanwhile),
// so a block's waves agree.  Results are those of the separate scalars and direction
// kernels, bit for bit.
template <bool NT>
__global__ __launch_bounds__(VBLOCK) void k_cg_scalars_direction(SolveCfg c, int nbx, const double* __restrict__ part,
                                                                 int64_t Dp, const float* __restrict__ minv,
                                                                 const float* __restrict__ R, float* __restrict__ Pd,
                                                                 uint16_t* __restrict__ PdH, uint16_t* __restrict__ PdL,
                                                                 uint16_t* __restrict__ PdX, CGState* __restrict__ st) {
  if (blockIdx.y == 0) {
    if (blockIdx.x == 0 && !st->done) cg_scalars_block(c, nbx, part, st);
    return;
  }
  const int q = blockIdx.y - 1;
  const DirTile dt = cg_direction_load(blockIdx.x, q, Dp, minv, R, Pd);
  double old = 0.0, b = 0.0;
  int dn = 0;
  if (threadIdx.x < 64) {
    dn = st->done;
    old = st->rho_prev[q];
    const double2* pq = reinterpret_cast<const double2*>(part + (int64_t)q * nbx * 2);
#pragma unroll 8
    for (int i = threadIdx.x; i < nbx; i += 64) b += pq[i].y;
  }
  // the scalars block may set done during this launch: one reading for the whole block
  __shared__ double s_eta;
  __shared__ int s_done;
  if (threadIdx.x < 64) {
    b = wave_sum(b);
    if (threadIdx.x == 0) {
      s_done = dn;
      s_eta = (old != 0.0) ? b / old : 0.0;
    }
  }
  __syncthreads();
  if (s_done) return;
  cg_direction_store<NT>(dt, blockIdx.x, q, Dp, s_eta, Pd, PdH, PdL, PdX);
}

// The direction update with the bf16 slices in the tile-interleaved layout (the FIR
// dictionary's bf16 phase): a block covers one 16-column tile and 256 coordinates in
// four steps of 64, 16 threads per column, so each step's slice stores are two
// contiguous 1 KB segments.
constexpr int DIR_SIG_COORDS = 256;
typedef __attribute__((ext_vector_type(4))) unsigned short u16x4v;
// XD (the bf16 form, whose direction is its hi/lo pair: the FP32 Pd is neither read nor
// written): also X += gamma P (the update left it here) when the step's update ran
// (xpend), before the done test, so the step that meets the stop rule still moves X.
// NT: X, P and its slices stored non-temporally (the operator streams them back long
// after these lines would have left the L2).
template <bool NT, bool XD>
__global__ __launch_bounds__(VBLOCK) void k_cg_direction_sig(SolveCfg c, int64_t Dp, const float* __restrict__ minv,
                                                             const float* __restrict__ R, float* __restrict__ Pd,
                                                             uint16_t* __restrict__ PdH, uint16_t* __restrict__ PdL,
                                                             float* __restrict__ X, const CGState* __restrict__ st) {
  if (XD ? !st->xpend : st->done) return;
  const int q = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (q >= c.Q) return;
  const int64_t j0 = (int64_t)blockIdx.x * DIR_SIG_COORDS + 4 * (threadIdx.x & 15);
  f32x4 mi[4], r[4], p[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t j = j0 + 64 * k, o = (int64_t)q * Dp + j;
    mi[k] = *reinterpret_cast<const f32x4*>(minv + j);
    r[k] = *reinterpret_cast<const f32x4*>(R + o);
    if constexpr (XD) {
      const int64_t os = sig_index(q, j, Dp, c.Q);
      const u16x4v h = *reinterpret_cast<const u16x4v*>(PdH + os), l = *reinterpret_cast<const u16x4v*>(PdL + os);
#pragma unroll
      for (int e = 0; e < 4; ++e) p[k][e] = bf16_val(h[e]) + bf16_val(l[e]);
    } else {
      p[k] = *reinterpret_cast<const f32x4*>(Pd + o);
    }
  }
  if constexpr (XD) {
    const double gam = st->gamma[q];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t o = (int64_t)q * Dp + j0 + 64 * k;
      f32x4 x = *reinterpret_cast<const f32x4*>(X + o);
#pragma unroll
      for (int e = 0; e < 4; ++e) x[e] = (float)((double)x[e] + gam * (double)p[k][e]);
      if constexpr (NT) __builtin_nontemporal_store(x, reinterpret_cast<f32x4*>(X + o));
      else *reinterpret_cast<f32x4*>(X + o) = x;
    }
    if (st->done) return;
  }
  const double eta = st->eta[q];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t j = j0 + 64 * k, o = (int64_t)q * Dp + j;
#pragma unroll
    for (int e = 0; e < 4; ++e) p[k][e] = (float)((double)mi[k][e] * (double)r[k][e] + eta * (double)p[k][e]);
    if constexpr (!XD) {
      if constexpr (NT) __builtin_nontemporal_store(p[k], reinterpret_cast<f32x4*>(Pd + o));
      else *reinterpret_cast<f32x4*>(Pd + o) = p[k];
    }
    store_split4<NT>(PdH, PdL, sig_index(q, j, Dp, c.Q), p[k]);
  }
}

// One block: pi_q into the state (used by the single-application test hook).
__global__ __launch_bounds__(VBLOCK) void k_reduce_pi(int Q, int nbx, const double* __restrict__ pipart,
                                                      double* __restrict__ pi) {
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  for (int q = wv; q < Q; q += 4) {
    const double a = wave_sum_strided(pipart + (int64_t)q * nbx, nbx, 1);
    if (ln == 0) pi[q] = a;
  }
}

// Multi-task M-step (Sec. III-E.1): alpha_j = 1 / max(sum_l (mu_lj^2 + s_lj) / L, floor),
// summed over the tasks in order; floor events are counted into *clamped.
__global__ __launch_bounds__(VBLOCK) void k_mt_mstep(const float* const* __restrict__ mus,
                                                     const float* const* __restrict__ ss, int L, int64_t D,
                                                     float* __restrict__ alpha, double floor, int* __restrict__ clamped) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int low = 0;
  if (j < D) {
    double acc = 0.0;
    for (int l = 0; l < L; ++l) {
      const double m = (double)mus[l][j];
      acc += m * m + (double)ss[l][j];
    }
    double den = acc / (double)L;
    if (den < floor) {
      den = floor;
      low = 1;
    }
    alpha[j] = (float)(1.0 / den);
  }
  low = wave_sum_int(low);
  if ((threadIdx.x & 63) == 0 && low) atomicAdd(clamped, low);
}

// ---------------------------------------------------------------------------
// test-hook helpers
// ---------------------------------------------------------------------------
__global__ void k_pack_block(const float* __restrict__ src, int ncols, int64_t D, int Qp, int64_t Dp,
                             float* __restrict__ dst, uint16_t* __restrict__ dH, uint16_t* __restrict__ dL,
                             uint16_t* __restrict__ dX, int sigblk) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (j >= Dp || q >= Qp) return;
  const float v = (q < ncols && j < D) ? src[(int64_t)q * D + j] : 0.0f;
  const int64_t o = (int64_t)q * Dp + j;
  dst[o] = v;
  if (dH && (!sigblk || q < ncols)) {  // the interleaved layout holds the real columns only
    uint16_t h, l;
    split_bf16(v, h, l);
    const int64_t os = sigblk ? sig_index(q, j, Dp, ncols) : o;
    dH[os] = h;
    dL[os] = l;
    if (dX) dX[os] = slice3_bf16(v, h, l);
  }
}
__global__ void k_unpack_block(const float* __restrict__ src, int ncols, int64_t D, int64_t Dp,
                               float* __restrict__ dst) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (j >= D || q >= ncols) return;
  dst[(int64_t)q * D + j] = src[(int64_t)q * Dp + j];
}
__global__ void k_copy_pad(const float* __restrict__ src, int64_t n, int64_t np, float pad,
                           float* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < np) dst[i] = (i < n) ? src[i] : pad;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

void launch_dict_layouts(const float* phi, int64_t N, int64_t D, int64_t Np, int64_t Dp, int64_t kc16, float* phi32,
                         float* phi32T, uint16_t* phi16, uint16_t* phi16T, hipStream_t s) {
  dim3 grid((unsigned)(Dp / 64), (unsigned)(Np / 64));
  hipLaunchKernelGGL(k_dict_layouts, grid, dim3(256), 0, s, phi, N, D, Np, Dp, kc16, phi32, phi32T, phi16, phi16T);
}

void launch_theta(const float* phi, int64_t N, int64_t D, int64_t Dp, int jacobi, float* theta, hipStream_t s) {
  hipLaunchKernelGGL(k_theta, dim3(cdiv(Dp, 256)), dim3(256), 0, s, phi, N, D, Dp, jacobi, theta);
}

void launch_rhs(const float* phi32T, const uint16_t* phi16T, int64_t ld, int64_t Np, int64_t Dp, const float* y,
                double beta, float* b, hipStream_t s) {
  if (phi32T)
    hipLaunchKernelGGL(k_rhs<float>, dim3(cdiv(Dp, 4)), dim3(256), 0, s, phi32T, ld, Np, Dp, y, beta, b);
  else
    hipLaunchKernelGGL(k_rhs<uint16_t>, dim3(cdiv(Dp, 4)), dim3(256), 0, s, phi16T, ld, Np, Dp, y, beta, b);
}

void launch_fill(float* x, float v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(cdiv(n, 256)), dim3(256), 0, s, x, v, n);
}

void launch_axpy(float* y, const float* x, float a, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, dim3(cdiv(n, 256)), dim3(256), 0, s, y, x, a, n);
}

void launch_state_reset(CGState* st, int Q, hipStream_t s) {
  hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(256), 0, s, st, Q);
}

void launch_em_init(const SolveCfg& c, uint64_t key, int64_t D, int64_t Dp, const float* b, const float* theta,
                    const float* alpha, float* minv, float* X, float* R, float* Pd, uint16_t* PdH, uint16_t* PdL,
                    double* part, CGState* st, hipStream_t s, uint16_t* PdX) {
  const int nblk = (int)(Dp / VBLOCK);
  hipLaunchKernelGGL(k_em_init, dim3((unsigned)nblk), dim3(VBLOCK), 0, s, c, key, D, Dp, b, theta, alpha, minv, X,
                     R, Pd, PdH, PdL, PdX, part);
  hipLaunchKernelGGL(k_em_scalars, dim3(1), dim3(VBLOCK), 0, s, c, D, nblk, (const double*)part, st);
}

void launch_mstep(const SolveCfg& c, uint64_t key, int64_t D, int64_t Dp, const float* X, float* mu,
                  float* s_out, float* alpha, double floor, int do_mstep, CGState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_mstep, dim3(cdiv(D, VBLOCK)), dim3(VBLOCK), 0, s, c, key, D, Dp, X, mu, s_out, alpha, floor,
                     do_mstep, st);
}

GemmCfg choose_gemm(int64_t rows, int64_t kdim, int bf16) {
  (void)bf16;
  GemmCfg g;
  g.rt = 4;
  while (g.rt > 1 && rows / (64 * g.rt) < 64) g.rt /= 2;
  const int64_t row_blocks = rows / (64 * g.rt);
  int64_t splits = std::max<int64_t>(1, 512 / std::max<int64_t>(row_blocks, 1));
  int64_t kchunk = (kdim + splits - 1) / splits;
  kchunk = ((kchunk + 255) / 256) * 256;
  g.kchunk = kchunk;
  g.splits = (int)((kdim + kchunk - 1) / kchunk);
  return g;
}

constexpr int KS_BF16 = 2;  // 32-k steps per stage (64 k)
constexpr int KS_F32 = 1;   // 32-k steps per stage (32 k)

// Column tiles for Q right-hand sides: MFMA tiles of 16, except that a lone column past one
// or two full tiles (Q = 17, 33) goes to the vector ALU instead of a mostly padded tile.
static inline void gemm_cols(int Q, int& ct, bool& x1) {
  x1 = Q == 17 || Q == 33;
  ct = x1 ? Q / 16 : (Q + 15) / 16;
}

#define GEMM_BF16(RT, CT, X1)                                                                                      \
  hipLaunchKernelGGL((k_gemm_bf16<RT, CT, KS_BF16, X1>), grid, dim3(64 * GEMM_WAVES), 0, s, M, ldm, sps, ZH, ZL, kdim, \
                     Yp, rows, Qp, g.kchunk, kdim, nrb, g.splits, done)
#define GEMM_F32(RT, CT, X1)                                                                                    \
  hipLaunchKernelGGL((k_gemm_f32<RT, CT, KS_F32, X1>), grid, dim3(64 * GEMM_WAVES), 0, s, M, ldm, ZH, ZM, ZL, kdim, Yp, \
                     rows, Qp, g.kchunk, kdim, nrb, g.splits, done)

template <int RT>
static void gemm_bf16_rt(const GemmCfg& g, const uint16_t* M, int64_t ldm, int64_t sps, int64_t rows, int64_t kdim,
                         const uint16_t* ZH, const uint16_t* ZL, int Q, int Qp, float* Yp, const int* done,
                         hipStream_t s) {
  const int nrb = (int)(rows / (64 * RT));
  dim3 grid((unsigned)(nrb * g.splits));
  int ct;
  bool x1;
  gemm_cols(Q, ct, x1);
  if (x1) {
    if (ct == 1) GEMM_BF16(RT, 1, true);
    else GEMM_BF16(RT, 2, true);
  } else {
    switch (ct) {
      case 1: GEMM_BF16(RT, 1, false); break;
      case 2: GEMM_BF16(RT, 2, false); break;
      case 3: GEMM_BF16(RT, 3, false); break;
      default: GEMM_BF16(RT, 4, false); break;
    }
  }
}

void launch_gemm_bf16(const GemmCfg& g, const uint16_t* M, int64_t ldm, int64_t sps, int64_t rows, int64_t kdim,
                      const uint16_t* ZH, const uint16_t* ZL, int Q, int Qp, float* Yp, const CGState* st,
                      hipStream_t s) {
  const int* done = st ? &st->done : nullptr;
  if (g.rt == 4) gemm_bf16_rt<4>(g, M, ldm, sps, rows, kdim, ZH, ZL, Q, Qp, Yp, done, s);
  else if (g.rt == 2) gemm_bf16_rt<2>(g, M, ldm, sps, rows, kdim, ZH, ZL, Q, Qp, Yp, done, s);
  else gemm_bf16_rt<1>(g, M, ldm, sps, rows, kdim, ZH, ZL, Q, Qp, Yp, done, s);
}

template <int RT>
static void gemm_f32_rt(const GemmCfg& g, const float* M, int64_t ldm, int64_t rows, int64_t kdim, const uint16_t* ZH,
                        const uint16_t* ZM, const uint16_t* ZL, int Q, int Qp, float* Yp, const int* done,
                        hipStream_t s) {
  const int nrb = (int)(rows / (64 * RT));
  dim3 grid((unsigned)(nrb * g.splits));
  int ct;
  bool x1;
  gemm_cols(Q, ct, x1);
  if (x1) {
    if (ct == 1) GEMM_F32(RT, 1, true);
    else GEMM_F32(RT, 2, true);
  } else {
    switch (ct) {
      case 1: GEMM_F32(RT, 1, false); break;
      case 2: GEMM_F32(RT, 2, false); break;
      case 3: GEMM_F32(RT, 3, false); break;
      default: GEMM_F32(RT, 4, false); break;
    }
  }
}

void launch_gemm_f32(const GemmCfg& g, const float* M, int64_t rows, int64_t kdim, const uint16_t* ZH,
                     const uint16_t* ZM, const uint16_t* ZL, int Q, int Qp, float* Yp, const CGState* st,
                     hipStream_t s) {
  const int* done = st ? &st->done : nullptr;
  const int64_t ldm = dict_ld(kdim, 4);
  if (g.rt == 4) gemm_f32_rt<4>(g, M, ldm, rows, kdim, ZH, ZM, ZL, Q, Qp, Yp, done, s);
  else if (g.rt == 2) gemm_f32_rt<2>(g, M, ldm, rows, kdim, ZH, ZM, ZL, Q, Qp, Yp, done, s);
  else gemm_f32_rt<1>(g, M, ldm, rows, kdim, ZH, ZM, ZL, Q, Qp, Yp, done, s);
}

void launch_finish_pass1(const float* Ypart, int splits, int Q, int Qp, int64_t Np, float* V, uint16_t* VH,
                         uint16_t* VL, const CGState* st, hipStream_t s, uint16_t* VX) {
  dim3 grid(cdiv(Np, VCHUNK), (unsigned)Q);
  hipLaunchKernelGGL(k_finish_pass1, grid, dim3(256), 0, s, Ypart, splits, Np, V, VH, VL, VX, Qp, &st->done);
}

void launch_finish_pass2(const SolveCfg& c, const float* Ypart, int splits, int64_t Dp, const float* alpha,
                         const float* Pd, float* Psi, double* pipart, const CGState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_finish_pass2, dim3(cdiv(Dp, VCHUNK), (unsigned)c.Q), dim3(VBLOCK), 0, s, c, Ypart, splits,
                     Dp, alpha, Pd, Psi, pipart, st);
}

// Above this many pi partials per column, one block reduces them once (k_cg_gamma)
// instead of every update tile re-reducing them.
constexpr int GAMMA_PRE_MIN_CHUNKS = 128;

void launch_cg_update(const SolveCfg& c, int64_t Dp, const float* minv, float* X, float* R, const float* Pd,
                      const float* Psi, const double* pipart, double* part, CGState* st, hipStream_t s, bool xdir,
                      bool scalars) {
  const unsigned nbx = cdiv(Dp, VCHUNK);
  const dim3 grid(nbx, (unsigned)c.Q);
  const bool pre = nbx > (unsigned)GAMMA_PRE_MIN_CHUNKS;
  if (pre) hipLaunchKernelGGL(k_cg_gamma, dim3((unsigned)c.Q), dim3(64), 0, s, c, (int)nbx, pipart, st);
  auto kern = xdir ? (pre ? k_cg_update<true, true, false> : k_cg_update<false, true, false>)
             : pre  ? (c.nt_store ? k_cg_update<true, true, true> : k_cg_update<true, false, true>)
                    : (c.nt_store ? k_cg_update<false, true, true> : k_cg_update<false, false, true>);
  hipLaunchKernelGGL(kern, grid, dim3(VBLOCK), 0, s, c, Dp, minv, X, R, Pd, Psi, pipart, part, st);
  if (scalars) hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(1024), 0, s, c, (int)nbx, (const double*)part, st);
}
bool cg_direction_fuses_scalars(const SolveCfg& c, const uint16_t* PdH) { return !(c.sigblk && PdH); }

void launch_reduce_pi(int Q, int64_t Dp, const double* pipart, double* pi, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_pi, dim3(1), dim3(VBLOCK), 0, s, Q, (int)cdiv(Dp, VCHUNK), pipart, pi);
}

void launch_cg_direction(const SolveCfg& c, int64_t Dp, const float* minv, const float* R, float* Pd,
                         uint16_t* PdH, uint16_t* PdL, CGState* st, hipStream_t s, uint16_t* PdX, float* X,
                         const double* part) {
  // FP32 P non-temporally only when the operator reads the slices instead
  const bool nt = c.nt_store && PdH;
  if (c.sigblk && PdH) {
    auto kern = X ? (nt ? k_cg_direction_sig<true, true> : k_cg_direction_sig<false, true>)
                  : (nt ? k_cg_direction_sig<true, false> : k_cg_direction_sig<false, false>);
    hipLaunchKernelGGL(kern, dim3((unsigned)(Dp / DIR_SIG_COORDS), cdiv(c.Q, 16)), dim3(VBLOCK), 0, s, c, Dp, minv,
                       R, Pd, PdH, PdL, X, st);
    return;
  }
  // column-major directions: the CG scalars run in the same launch
  hipLaunchKernelGGL(nt ? k_cg_scalars_direction<true> : k_cg_scalars_direction<false>,
                     dim3(cdiv(Dp, VCHUNK), (unsigned)c.Q + 1), dim3(VBLOCK), 0, s, c, (int)cdiv(Dp, VCHUNK), part,
                     Dp, minv, R, Pd, PdH, PdL, PdX, st);
}

void launch_mt_mstep(const float* const* mus, const float* const* ss, int L, int64_t D, float* alpha, double floor,
                     int* clamped, hipStream_t s) {
  hipLaunchKernelGGL(k_mt_mstep, dim3(cdiv(D, VBLOCK)), dim3(VBLOCK), 0, s, mus, ss, L, D, alpha, floor, clamped);
}

void launch_pack_block(const float* src, int ncols, int64_t D, int Qp, int64_t Dp, float* dst, uint16_t* dH,
                       uint16_t* dL, hipStream_t s, uint16_t* dX, int sigblk) {
  hipLaunchKernelGGL(k_pack_block, dim3(cdiv(Dp, 256), (unsigned)Qp), dim3(256), 0, s, src, ncols, D, Qp, Dp, dst,
                     dH, dL, dX, sigblk);
}
void launch_unpack_block(const float* src, int ncols, int64_t D, int64_t Dp, float* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_unpack_block, dim3(cdiv(D, 256), (unsigned)ncols), dim3(256), 0, s, src, ncols, D, Dp,
                     dst);
}
void launch_count_nonfinite(const float* x, int64_t n, int* count, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>(std::max<int64_t>(cdiv(n, 256), 1), 4096);
  hipLaunchKernelGGL(k_count_nonfinite, dim3((unsigned)blocks), dim3(256), 0, s, x, n, count);
}
void launch_copy_pad(const float* src, int64_t n, int64_t np, float pad, float* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_pad, dim3(cdiv(np, 256)), dim3(256), 0, s, src, n, np, pad, dst);
}

}  // namespace cofem
