// Block-level building blocks of one CoFEM E-step (Algorithm 1 around Algorithm 2).
// Each function is the work of one thread block on one tile, with the tile's
// coordinates passed explicitly, so that the single-problem kernels (one problem
// per launch, tile = block index) and the serving kernels (many problems per
// launch, tiles taken from a table) run the same code and produce bitwise the
// same results for a problem.
#pragma once
#include "device_common.h"

namespace cofem {

// ---------------------------------------------------------------------------
// E-step initialisation: B = [b | p_1..p_K | 0], X = 0, R = B, W = M^-1 R, P = W,
// M^-1 = 1 / (beta theta + alpha).  Block blk covers coordinates [256 blk, +256).
// Partial sums for rho and ||B_q||^2 go to part[blk * 3 + {0,1,2}].
// ---------------------------------------------------------------------------
__device__ __forceinline__ void em_init_block(const SolveCfg& c, uint64_t key, int64_t D, int64_t Dp, int blk,
                                              const float* __restrict__ b, const float* __restrict__ theta,
                                              const float* __restrict__ alpha, float* __restrict__ minv,
                                              float* __restrict__ X, float* __restrict__ R, float* __restrict__ Pd,
                                              uint16_t* __restrict__ PdH, uint16_t* __restrict__ PdL,
                                              uint16_t* __restrict__ PdX, double* __restrict__ part) {
  const int64_t j = (int64_t)blk * VBLOCK + threadIdx.x;  // Dp is a multiple of VBLOCK
  const bool real = j < D;
  const float mi = (float)(1.0 / (c.beta * (double)theta[j] + (double)alpha[j]));
  minv[j] = mi;
  const double mid = (double)mi;
  const uint64_t w = real ? probe_word(key, j) : 0ull;
  const float bj = real ? b[j] : 0.0f;
  for (int q = 0; q < c.Qp; ++q) {
    float bq = 0.0f;
    if (real) bq = (q == 0) ? bj : (q <= c.K ? (c.hadamard ? hadamard_sign(j, q - 1) : probe_sign(w, q - 1)) : 0.0f);
    const int64_t o = (int64_t)q * Dp + j;
    X[o] = 0.0f;
    R[o] = bq;
    const float p = (float)(mid * (double)bq);
    Pd[o] = p;
    if (PdH && (!c.sigblk || q < c.Q)) {  // the interleaved layout holds the real columns only
      uint16_t h, l;
      split_bf16(p, h, l);
      const int64_t os = c.sigblk ? sig_index(q, j, Dp, c.Q) : o;
      PdH[os] = h;
      PdL[os] = l;
      if (PdX) PdX[os] = slice3_bf16(p, h, l);
    }
  }
  // rho_0 = sum_j b_j (minv_j b_j); rho_q = sum_j minv_j for probes (entries square to 1); ||b||^2
  const double s_minv = block_sum(real ? mid : 0.0);
  const double s_bw = block_sum(real ? (double)bj * (mid * (double)bj) : 0.0);
  const double s_bb = block_sum(real ? (double)bj * (double)bj : 0.0);
  if (threadIdx.x == 0) {
    part[(int64_t)blk * 3 + 0] = s_minv;
    part[(int64_t)blk * 3 + 1] = s_bw;
    part[(int64_t)blk * 3 + 2] = s_bb;
  }
}

// One block: rho_q, ||B_q||^2, ||B||_F^2, active flags, done = 0 (or 1 when the
// per-column rule has nothing to solve), steps = 0.
__device__ __forceinline__ void em_scalars_block(const SolveCfg& c, int64_t D, int nblk, const double* __restrict__ part,
                                                 CGState* __restrict__ st) {
  if (threadIdx.x >= 64) return;
  const double t_minv = wave_sum_strided(part + 0, nblk, 3);
  const double t_bw = wave_sum_strided(part + 1, nblk, 3);
  const double t_bb = wave_sum_strided(part + 2, nblk, 3);
  if (threadIdx.x != 0) return;
  int nact = 0;
  for (int q = 0; q < QMAX; ++q) {
    double rho = 0.0, bn2 = 0.0;
    if (q == 0) {
      rho = t_bw;
      bn2 = t_bb;
    } else if (q <= c.K) {
      rho = t_minv;
      bn2 = (double)D;
    }
    st->rho[q] = rho;
    st->bn2[q] = bn2;
    st->pi[q] = 0.0;
    st->gamma[q] = 0.0;
    st->eta[q] = 0.0;
    st->rn2[q] = bn2;
    int act = (q < c.Q) ? 1 : 0;
    if (c.stop_mode == 1 && bn2 <= 0.0) act = 0;
    st->active[q] = act;
    nact += act;
  }
  st->bnorm2 = t_bb + (double)c.K * (double)D;
  st->delta = 1.0;
  st->steps = 0;
  st->done = (c.stop_mode == 1 && nact == 0) ? 1 : 0;
  st->xpend = 0;
}

// mu = X_0, s_j = (1/K) sum_k p_kj X_kj (Eq. diag-estimate; probes regenerated from
// the key), and for do_mstep: alpha_j = 1 / max(E_j, floor), counting floor events, with
// E_j = mu_j^2 + s_j (Eq. mstep) or, for the non-negative model, the second moment of
// the rectified Gaussian posterior (Eq. nonneg-sbl) with s_j in place of Sigma_jj:
// E_j = mu^2 + v + mu sqrt(2 v / pi) / erfcx(-xi), v = max(s_j, floor), xi = mu / sqrt(2 v)
// (the sqrt(2 v / pi) factor is the truncated-Gaussian moment; exp(-xi^2) / erfc(-xi) is
// evaluated as 1 / erfcx(-xi), ROCm's scaled complementary error function).
// Block blk covers coordinates [256 blk, +256).
__device__ __forceinline__ void mstep_block(const SolveCfg& c, uint64_t key, int64_t D, int64_t Dp, int blk,
                                            const float* __restrict__ X, float* __restrict__ mu,
                                            float* __restrict__ s_out, float* __restrict__ alpha, double floor,
                                            int do_mstep, CGState* __restrict__ st) {
  const int64_t j = (int64_t)blk * VBLOCK + threadIdx.x;
  int clamped = 0;
  if (j < D) {
    const float m = X[j];
    const uint64_t w = probe_word(key, j);
    double acc = 0.0;
    for (int k = 0; k < c.K; ++k) {
      const float pk = c.hadamard ? hadamard_sign(j, k) : probe_sign(w, k);
      acc += (double)pk * (double)X[(int64_t)(k + 1) * Dp + j];
    }
    const double s = acc / (double)c.K;
    mu[j] = m;
    s_out[j] = (float)s;
    if (do_mstep) {
      const double md = (double)m;
      double den;
      if (c.nonneg) {
        const double v = s > floor ? s : floor;
        const double xi = md / sqrt(2.0 * v);
        den = md * md + v + md * sqrt(2.0 * v / M_PI) / erfcx(-xi);
      } else {
        den = md * md + s;
      }
      if (den < floor) {
        den = floor;
        clamped = 1;
      }
      alpha[j] = (float)(1.0 / den);
    }
  }
  clamped = wave_sum_int(clamped);
  if ((threadIdx.x & 63) == 0 && clamped) atomicAdd(&st->clamped, clamped);
}

// ---------------------------------------------------------------------------
// The operator's contractions: Ypart[split][q][row] = sum_{k in split} M[row, k] Z[q, k].
//
// Block = 4 waves.  Wave w owns rows row0 .. row0 + 16 RT - 1 and all CT*16
// columns, and streams its rows of M from HBM straight into VGPRs in the MFMA
// operand layout, one stage (KS MFMA k-steps) ahead.  The right-hand-side
// fragments of a stage (already in MFMA lane order: lane l's 16 bytes) are copied
// from L2 into LDS by the compute waves themselves with 16-byte LDS DMA loads
// (global_load_lds_dwordx4: lane l's bytes land at base + 16 l), a quarter of the
// fragments per wave, into a double buffer; they take no VGPRs while in flight.
// Per stage: wait for this wave's loads of the stage, one barrier (every wave's
// fragments have landed, and the other buffer is free), issue the next stage's
// loads (branch-free: the last stage reloads itself), then the MFMAs.  The
// sched_barrier keeps the prefetch ahead of the MFMAs.  L is the tile index
// (split and row block via tile_of).  Every call ends with no DMA in flight.
// ---------------------------------------------------------------------------
constexpr int GEMM_WAVES = 4;  // waves per contraction tile (launch with 64 * GEMM_WAVES threads)

typedef __attribute__((ext_vector_type(8))) unsigned short u16x8v;

__device__ __forceinline__ void lds_dma16(const void* src, void* lds_base) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)lds_base, 16, 0, 0);
}
__device__ __forceinline__ void wait_vm_all() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// The extra column's partials: lane (r16, g) holds row r16 of each row tile summed over its
// k-subset; the four g-lanes of a row are added in a fixed order and lane g = 0 stores.
template <int RT>
__device__ __forceinline__ void store_x1(float (&xacc)[RT], float* __restrict__ ycol, int64_t row0, int r16, int g) {
#pragma unroll
  for (int a = 0; a < RT; ++a) {
    float v = xacc[a];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    if (g == 0) ycol[row0 + a * 16 + r16] = v;
  }
}

// bf16: v_mfma_f32_16x16x32_bf16, lane l holds A[l%16][8(l/16) .. +8), B[8(l/16) .. +8)[l%16]
// and returns D[4(l/16) .. +4)[l%16].  ZH + ZL carries each right-hand side to ~2^-17.
// X1: one more right-hand side (column 16 CT, e.g. the 33rd of K = 32 probes) in a third
// MFMA column tile that carries its hi piece as column 0 and its lo piece as column 1 (the
// other 14 columns of that tile are don't-care: an MFMA output column depends on its own B
// column only), so it costs one MFMA per row tile and 32-k step instead of two, and the
// two result columns are added lane to lane at the end.
// sps: 0 when M is one block of rows (row r, reduction index k at M[r ldm + k]); else M is
// split-blocked, split s being its own row block at M + s sps (k at M[s sps + r ldm + k - s
// kchunk]).
template <int RT, int CT, int KS, bool X1>
__device__ __forceinline__ void gemm_bf16_tile(int L, const uint16_t* __restrict__ M, int64_t ldm,
                                               const uint16_t* __restrict__ ZH, const uint16_t* __restrict__ ZL,
                                               int64_t ldz, float* __restrict__ Yp, int64_t ldy, int Qp,
                                               int64_t kchunk, int64_t kdim, int nrb, int splits, int64_t sps) {
  constexpr int FS = CT * 2 + (X1 ? 1 : 0);  // fragments per 32-k step
  constexpr int NF = KS * FS;                 // fragments per stage
  constexpr int SK = 32 * KS;                 // k per stage
  __shared__ bf16x8_t sB[2][NF][64];
  int rb, sp;
  tile_of(L, nrb, splits, rb, sp);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const int64_t kb = (int64_t)sp * kchunk;
  const int64_t ke = (kb + kchunk < kdim) ? kb + kchunk : kdim;
  const int nst = (ke > kb) ? (int)((ke - kb) / SK) : 0;
  if (nst == 0 || wave >= GEMM_WAVES) return;  // the tile is 64 RT rows: waves past the fourth have none
  auto issue_B = [&](int st, int buf) {
#pragma unroll
    for (int i = 0; i < (NF + 3) / 4; ++i) {
      const int f = wave + 4 * i;
      if (f < NF) {
        const int s = f / FS, rem = f % FS;
        const int64_t k = kb + (int64_t)st * SK + s * 32 + 8 * g;
        if (X1 && rem == CT * 2) {
          // the extra column: lanes of column 1 take its lo piece, all others its hi piece
          lds_dma16((r16 == 1 ? ZL : ZH) + (int64_t)(CT * 16) * ldz + k, &sB[buf][f][0]);
        } else {
          const int ct = rem >> 1, hl = rem & 1;
          lds_dma16((hl ? ZL : ZH) + (int64_t)(ct * 16 + r16) * ldz + k, &sB[buf][f][0]);
        }
      }
    }
  };
  const int64_t row0 = (int64_t)rb * (64 * RT) + (int64_t)wave * (16 * RT);
  f32x4 acc[RT][CT], accx[RT];
#pragma unroll
  for (int a = 0; a < RT; ++a) {
#pragma unroll
    for (int b = 0; b < CT; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    accx[a] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  const uint16_t* ap[RT];
#pragma unroll
  for (int a = 0; a < RT; ++a) ap[a] = M + (sps ? (int64_t)sp * sps : kb) + (row0 + a * 16 + r16) * ldm + 8 * g;
  bf16x8_t acur[RT][KS];
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int s = 0; s < KS; ++s) acur[a][s] = *reinterpret_cast<const bf16x8_t*>(ap[a] + s * 32);
  issue_B(0, 0);
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    wait_vm_all();    // this wave's A and B pieces of stage st
    __syncthreads();  // every wave's B pieces; buf ^ 1 is no longer read
    const int nx = (st + 1 < nst) ? st + 1 : st;
    bf16x8_t anxt[RT][KS];
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
      for (int s = 0; s < KS; ++s) anxt[a][s] = *reinterpret_cast<const bf16x8_t*>(ap[a] + (int64_t)nx * SK + s * 32);
    issue_B(nx, buf ^ 1);
    __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of this stage's MFMAs
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      bf16x8_t bh[CT], bl[CT];
#pragma unroll
      for (int b = 0; b < CT; ++b) {
        bh[b] = sB[buf][s * FS + b * 2 + 0][lane];
        bl[b] = sB[buf][s * FS + b * 2 + 1][lane];
      }
#pragma unroll
      for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int b = 0; b < CT; ++b) {
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(acur[a][s], bh[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(acur[a][s], bl[b], acc[a][b], 0, 0, 0);
        }
      if constexpr (X1) {
        const bf16x8_t bx = sB[buf][s * FS + CT * 2][lane];
#pragma unroll
        for (int a = 0; a < RT; ++a) accx[a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(acur[a][s], bx, accx[a], 0, 0, 0);
      }
    }
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
      for (int s = 0; s < KS; ++s) acur[a][s] = anxt[a][s];
  }
  wait_vm_all();  // the last (self-reloading) DMA has landed before the LDS is released
  float* yb = Yp + (int64_t)sp * Qp * ldy;
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int b = 0; b < CT; ++b) {
      const int64_t q = b * 16 + r16;
      const int64_t row = row0 + a * 16 + 4 * g;
      *reinterpret_cast<f32x4*>(yb + q * ldy + row) = acc[a][b];
    }
  if constexpr (X1) {
    // column 16 CT = hi column (lanes r16 = 0) + lo column (lanes r16 = 1)
    float* ycol = yb + (int64_t)(CT * 16) * ldy;
#pragma unroll
    for (int a = 0; a < RT; ++a) {
      f32x4 v = accx[a];
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] += __shfl_down(v[e], 1, 64);
      if (r16 == 0) *reinterpret_cast<f32x4*>(ycol + row0 + a * 16 + 4 * g) = v;
    }
  }
}

// FP32: v_mfma_f32_16x16x4_f32.  Each lane holds 4 consecutive k of its row (and of its
// column of Z) and feeds element e to the e-th MFMA, so the four MFMAs of a 16-k step
// see the same k order in both operands.  1 KB fragment per 16-k step and column tile.
// X1: one more right-hand side (column 16 CT) on the vector ALU, as in the bf16 tile.
template <int RT, int CT, int KS, bool X1>
__device__ __forceinline__ void gemm_f32_tile(int L, const float* __restrict__ M, int64_t ldm,
                                              const float* __restrict__ Z, int64_t ldz, float* __restrict__ Yp,
                                              int64_t ldy, int Qp, int64_t kchunk, int64_t kdim, int nrb,
                                              int splits) {
  constexpr int NF = KS * CT;
  constexpr int SK = 16 * KS;
  __shared__ f32x4 sB[2][NF][64];
  int rb, sp;
  tile_of(L, nrb, splits, rb, sp);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const int64_t kb = (int64_t)sp * kchunk;
  const int64_t ke = (kb + kchunk < kdim) ? kb + kchunk : kdim;
  const int nst = (ke > kb) ? (int)((ke - kb) / SK) : 0;
  if (nst == 0 || wave >= GEMM_WAVES) return;  // the tile is 64 RT rows: waves past the fourth have none
  auto issue_B = [&](int st, int buf) {
#pragma unroll
    for (int i = 0; i < (NF + 3) / 4; ++i) {
      const int f = wave + 4 * i;
      if (f < NF) {
        const int s = f / CT, ct = f % CT;
        lds_dma16(Z + (int64_t)(ct * 16 + r16) * ldz + kb + (int64_t)st * SK + s * 16 + 4 * g, &sB[buf][f][0]);
      }
    }
  };
  const int64_t row0 = (int64_t)rb * (64 * RT) + (int64_t)wave * (16 * RT);
  f32x4 acc[RT][CT];
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int b = 0; b < CT; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  const float* ap[RT];
#pragma unroll
  for (int a = 0; a < RT; ++a) ap[a] = M + (row0 + a * 16 + r16) * ldm + kb + 4 * g;
  f32x4 acur[RT][KS];
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int s = 0; s < KS; ++s) acur[a][s] = *reinterpret_cast<const f32x4*>(ap[a] + s * 16);
  const float* xp = Z + (int64_t)(CT * 16) * ldz + kb + 4 * g;
  f32x4 xcur[KS];
  float xacc[RT];
  if constexpr (X1) {
#pragma unroll
    for (int s = 0; s < KS; ++s) xcur[s] = *reinterpret_cast<const f32x4*>(xp + s * 16);
#pragma unroll
    for (int a = 0; a < RT; ++a) xacc[a] = 0.0f;
  }
  issue_B(0, 0);
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    wait_vm_all();
    __syncthreads();
    const int nx = (st + 1 < nst) ? st + 1 : st;
    f32x4 anxt[RT][KS];
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
      for (int s = 0; s < KS; ++s) anxt[a][s] = *reinterpret_cast<const f32x4*>(ap[a] + (int64_t)nx * SK + s * 16);
    f32x4 xnxt[KS];
    if constexpr (X1) {
#pragma unroll
      for (int s = 0; s < KS; ++s) xnxt[s] = *reinterpret_cast<const f32x4*>(xp + (int64_t)nx * SK + s * 16);
    }
    issue_B(nx, buf ^ 1);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      f32x4 bz[CT];
#pragma unroll
      for (int b = 0; b < CT; ++b) bz[b] = sB[buf][s * CT + b][lane];
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int a = 0; a < RT; ++a)
#pragma unroll
          for (int b = 0; b < CT; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(acur[a][s][e], bz[b][e], acc[a][b], 0, 0, 0);
      if constexpr (X1) {
#pragma unroll
        for (int a = 0; a < RT; ++a)
#pragma unroll
          for (int e = 0; e < 4; ++e) xacc[a] = __builtin_fmaf(acur[a][s][e], xcur[s][e], xacc[a]);
      }
    }
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
      for (int s = 0; s < KS; ++s) acur[a][s] = anxt[a][s];
    if constexpr (X1) {
#pragma unroll
      for (int s = 0; s < KS; ++s) xcur[s] = xnxt[s];
    }
  }
  wait_vm_all();
  float* yb = Yp + (int64_t)sp * Qp * ldy;
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int b = 0; b < CT; ++b) {
      const int64_t q = b * 16 + r16;
      const int64_t row = row0 + a * 16 + 4 * g;
      *reinterpret_cast<f32x4*>(yb + q * ldy + row) = acc[a][b];
    }
  if constexpr (X1) store_x1<RT>(xacc, yb + (int64_t)(CT * 16) * ldy, row0, r16, g);
}


// FP32 operands on the bf16 matrix cores.  Every FP32 value x is cut into three bf16
// slices x = h + m + l exactly: h = bf16(x), m = bf16(x - h), l = x - h - m (x - h has
// at most 16 significant bits and x - h - m at most 8, so both differences are exact in
// FP32 and l is a bf16 value).  A product x y is the sum of the six slice products of
// order 2^-16 |x y| or more (hh, hm, mh, hl, mm, lh); the three dropped ones are below
// 2^-26 |x y| (round-to-nearest slices), under the FP32 rounding of the product itself.
// v_mfma_f32_16x16x32_bf16 forms each slice product exactly and accumulates in FP32, so
// six of them per 32-k step take 3/8 of the matrix-core time of the eight
// v_mfma_f32_16x16x4_f32 the same step needs: the FP32 operator stays off the FP32
// matrix peak, which it would otherwise need 81 % of to stream at 8 TB/s.  The
// right-hand sides arrive already sliced (split3_bf16 where they are produced); the
// dictionary is sliced in registers on the vector ALU beside the MFMAs (about 5.5
// operations per value).
__device__ __forceinline__ void slice3(const f32x4& x0, const f32x4& x1, bf16x8_t& h, bf16x8_t& m, bf16x8_t& l) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float x = e < 4 ? x0[e] : x1[e - 4];
    const __bf16 hb = (__bf16)x;
    const float r = x - (float)hb;
    const __bf16 mb = (__bf16)r;
    h[e] = hb;
    m[e] = mb;
    l[e] = (__bf16)(r - (float)mb);
  }
}

// The FP32 contraction on sliced operands: the layout of gemm_bf16_tile (lane l holds
// A[l%16][8(l/16) .. +8) and B[8(l/16) .. +8)[l%16]), with A read as FP32 straight from
// HBM (two 16-byte loads per row tile and 32-k step) and sliced in registers, and the
// right-hand sides' three slices ZH, ZM, ZL staged through LDS by DMA as in the bf16
// tile.  X1: the extra column's slices h, m, l ride as columns 0, 1, 2 of one more MFMA
// tile (the other columns are don't-care), multiplied by all three slices of A, so that
// tile's columns 0 + 1 + 2 are the full product; they are added lane to lane at the end.
template <int RT, int CT, int KS, bool X1>
__device__ __forceinline__ void gemm_f32s_tile(int L, const float* __restrict__ M, int64_t ldm,
                                               const uint16_t* __restrict__ ZH, const uint16_t* __restrict__ ZM,
                                               const uint16_t* __restrict__ ZL, int64_t ldz, float* __restrict__ Yp,
                                               int64_t ldy, int Qp, int64_t kchunk, int64_t kdim, int nrb,
                                               int splits) {
  constexpr int FS = CT * 3 + (X1 ? 1 : 0);  // fragments per 32-k step
  constexpr int NF = KS * FS;                 // fragments per stage
  constexpr int SK = 32 * KS;                 // k per stage
  __shared__ bf16x8_t sB[2][NF][64];
  int rb, sp;
  tile_of(L, nrb, splits, rb, sp);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const int64_t kb = (int64_t)sp * kchunk;
  const int64_t ke = (kb + kchunk < kdim) ? kb + kchunk : kdim;
  const int nst = (ke > kb) ? (int)((ke - kb) / SK) : 0;
  if (nst == 0 || wave >= GEMM_WAVES) return;  // the tile is 64 RT rows: waves past the fourth have none
  auto issue_B = [&](int st, int buf) {
#pragma unroll
    for (int i = 0; i < (NF + 3) / 4; ++i) {
      const int f = wave + 4 * i;
      if (f < NF) {
        const int s = f / FS, rem = f % FS;
        const int64_t k = kb + (int64_t)st * SK + s * 32 + 8 * g;
        if (X1 && rem == CT * 3) {
          // the extra column: lanes of columns 1 and 2 take its m and l slices, all others h
          lds_dma16((r16 == 1 ? ZM : (r16 == 2 ? ZL : ZH)) + (int64_t)(CT * 16) * ldz + k, &sB[buf][f][0]);
        } else {
          const int ct = rem / 3, piece = rem % 3;
          lds_dma16((piece == 0 ? ZH : (piece == 1 ? ZM : ZL)) + (int64_t)(ct * 16 + r16) * ldz + k,
                    &sB[buf][f][0]);
        }
      }
    }
  };
  const int64_t row0 = (int64_t)rb * (64 * RT) + (int64_t)wave * (16 * RT);
  f32x4 acc[RT][CT], accx[RT];
#pragma unroll
  for (int a = 0; a < RT; ++a) {
#pragma unroll
    for (int b = 0; b < CT; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    accx[a] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  const float* ap[RT];
#pragma unroll
  for (int a = 0; a < RT; ++a) ap[a] = M + (row0 + a * 16 + r16) * ldm + kb + 8 * g;
  f32x4 acur[RT][KS][2];
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int h = 0; h < 2; ++h) acur[a][s][h] = *reinterpret_cast<const f32x4*>(ap[a] + s * 32 + 4 * h);
  issue_B(0, 0);
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    wait_vm_all();    // this wave's A and B pieces of stage st
    __syncthreads();  // every wave's B pieces; buf ^ 1 is no longer read
    const int nx = (st + 1 < nst) ? st + 1 : st;
    f32x4 anxt[RT][KS][2];
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int h = 0; h < 2; ++h)
          anxt[a][s][h] = *reinterpret_cast<const f32x4*>(ap[a] + (int64_t)nx * SK + s * 32 + 4 * h);
    issue_B(nx, buf ^ 1);
    __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of this stage's MFMAs
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      bf16x8_t bh[CT], bm[CT], bl[CT];
#pragma unroll
      for (int b = 0; b < CT; ++b) {
        bh[b] = sB[buf][s * FS + 3 * b + 0][lane];
        bm[b] = sB[buf][s * FS + 3 * b + 1][lane];
        bl[b] = sB[buf][s * FS + 3 * b + 2][lane];
      }
#pragma unroll
      for (int a = 0; a < RT; ++a) {
        bf16x8_t ah, am, al;
        slice3(acur[a][s][0], acur[a][s][1], ah, am, al);
#pragma unroll
        for (int b = 0; b < CT; ++b) {
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[b], acc[a][b], 0, 0, 0);
        }
        if constexpr (X1) {
          const bf16x8_t bx = sB[buf][s * FS + CT * 3][lane];
          accx[a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bx, accx[a], 0, 0, 0);
          accx[a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bx, accx[a], 0, 0, 0);
          accx[a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bx, accx[a], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int h = 0; h < 2; ++h) acur[a][s][h] = anxt[a][s][h];
  }
  wait_vm_all();  // the last (self-reloading) DMA has landed before the LDS is released
  float* yb = Yp + (int64_t)sp * Qp * ldy;
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int b = 0; b < CT; ++b) {
      const int64_t q = b * 16 + r16;
      const int64_t row = row0 + a * 16 + 4 * g;
      *reinterpret_cast<f32x4*>(yb + q * ldy + row) = acc[a][b];
    }
  if constexpr (X1) {
    // column 16 CT = columns 0 + 1 + 2 of the extra tile (lanes r16 = 0, 1, 2)
    float* ycol = yb + (int64_t)(CT * 16) * ldy;
#pragma unroll
    for (int a = 0; a < RT; ++a) {
      f32x4 v = accx[a];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float c1 = __shfl_down(v[e], 1, 64), c2 = __shfl_down(v[e], 2, 64);
        v[e] = (v[e] + c1) + c2;
      }
      if (r16 == 0) *reinterpret_cast<f32x4*>(ycol + row0 + a * 16 + 4 * g) = v;
    }
  }
}

// ---------------------------------------------------------------------------
// Split-K finishes and the CG vector updates.  Vector tiles: (chunk bx of VCHUNK
// coordinates, column q); each thread owns 4 consecutive coordinates.
// ---------------------------------------------------------------------------
// V[q][i] = sum_split Ypart[split][q][i] (fixed split order); V (FP32) and/or VH/VL (and
// the third slice VX).
__device__ __forceinline__ void finish1_tile(int bx, int q, const float* __restrict__ Yp, int splits, int64_t Np,
                                             float* __restrict__ V, uint16_t* __restrict__ VH,
                                             uint16_t* __restrict__ VL, int Qp, uint16_t* __restrict__ VX = nullptr) {
  const int64_t i = (int64_t)bx * VCHUNK + 4 * threadIdx.x;
  if (i >= Np) return;
  const int64_t o = (int64_t)q * Np + i;
  f32x4 v = *reinterpret_cast<const f32x4*>(Yp + o);
  for (int sp = 1; sp < splits; ++sp) v += *reinterpret_cast<const f32x4*>(Yp + (int64_t)sp * Qp * Np + o);
  if (V) *reinterpret_cast<f32x4*>(V + o) = v;
  if (VH) store_split4<true>(VH, VL, o, v, VX);
}

// Psi = beta * sum_split Ypart + alpha Pd and the tile's partial of pi_q = sum_j Pd_jq Psi_jq
// at pipart[q * nbx + bx].
__device__ __forceinline__ void finish2_tile(const SolveCfg& c, int bx, int q, int nbx, const float* __restrict__ Yp,
                                             int splits, int64_t Dp, const float* __restrict__ alpha,
                                             const float* __restrict__ Pd, float* __restrict__ Psi,
                                             double* __restrict__ pipart) {
  const int64_t j = (int64_t)bx * VCHUNK + 4 * threadIdx.x;
  double acc = 0.0;
  if (j < Dp) {
    const int64_t o = (int64_t)q * Dp + j;
    f32x4 y = *reinterpret_cast<const f32x4*>(Yp + o);
    for (int sp = 1; sp < splits; ++sp) y += *reinterpret_cast<const f32x4*>(Yp + (int64_t)sp * c.Qp * Dp + o);
    const f32x4 al = *reinterpret_cast<const f32x4*>(alpha + j);
    const f32x4 p = *reinterpret_cast<const f32x4*>(Pd + o);
    f32x4 ps;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      ps[e] = (float)(c.beta * (double)y[e] + (double)al[e] * (double)p[e]);
      acc += (double)p[e] * (double)ps[e];
    }
    *reinterpret_cast<f32x4*>(Psi + o) = ps;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) pipart[(int64_t)q * nbx + bx] = acc;
}

// gamma_q = rho_q / pi_q from the column's nbx pi partials, summed in a fixed order; a
// column with pi_q <= 0 and rho_q != 0 breaks down and is frozen.  Lane 0 of the calling
// wave gets the result; with `record` it also writes pi, gamma and the breakdown flag.
// Two halves, so that a kernel can have the inputs in flight while it does other work:
// rho_q, the active flag and, with at most one partial per lane (nbx <= 64), the lane's
// partial (the sum keeps the order of wave_sum_strided).
struct GammaIn {
  double rho, pp;
  int act;
};
__device__ __forceinline__ GammaIn column_gamma_load(int q, int nbx, const double* __restrict__ pipart,
                                                     const CGState* __restrict__ st) {
  GammaIn g;
  g.rho = st->rho[q];
  g.act = st->active[q];
  const int ln = threadIdx.x & 63;
  g.pp = (nbx <= 64 && ln < nbx) ? pipart[(int64_t)q * nbx + ln] : 0.0;
  return g;
}
template <int UNR = 8>
__device__ __forceinline__ double column_gamma_finish(int q, int nbx, const double* __restrict__ pipart,
                                                      CGState* __restrict__ st, bool record, const GammaIn& g) {
  double pi;
  if (nbx <= 64) {
    double a = 0.0;
    if ((int)(threadIdx.x & 63) < nbx) a += g.pp;
    pi = wave_sum(a);
  } else {
    pi = wave_sum_strided<UNR>(pipart + (int64_t)q * nbx, nbx, 1);
  }
  const double gam = (g.act && pi > 0.0) ? g.rho / pi : 0.0;
  if (record && (threadIdx.x & 63) == 0) {
    st->pi[q] = pi;
    st->gamma[q] = gam;
    st->rho_prev[q] = g.rho;
    if (g.act && !(pi > 0.0) && g.rho != 0.0) {  // breakdown: freeze the column
      st->active[q] = 0;
      atomicAdd(&st->breakdown, 1);
    }
  }
  return gam;
}
template <int UNR = 8>
__device__ __forceinline__ double column_gamma(int q, int nbx, const double* __restrict__ pipart,
                                               CGState* __restrict__ st, bool record) {
  return column_gamma_finish<UNR>(q, nbx, pipart, st, record, column_gamma_load(q, nbx, pipart, st));
}

// X += gamma Pd, R -= gamma Psi; partials of ||R_q||^2 and rho'_q = sum R (M^-1 R) at
// part[(q * nbx + bx) * 2 + {0, 1}].  gamma_q comes from the state (PRE, after
// k_cg_gamma) or is reduced here by every tile of the column, in the same order, so
// all tiles get the same value (the tile of chunk 0 records it).
// XU = false (the FIR dictionary's bf16 form): X is left to the direction kernel, which
// reads P anyway; block (0, 0) flags it in the state (xpend).
template <bool PRE, bool NT = false, bool XU = true>  // NT: X (and for PRE, R) stored non-temporally
__device__ __forceinline__ void cg_update_tile(const SolveCfg& c, int bx, int q, int nbx, int64_t Dp,
                                               const float* __restrict__ minv, float* __restrict__ X,
                                               float* __restrict__ R, const float* __restrict__ Pd,
                                               const float* __restrict__ Psi, const double* __restrict__ pipart,
                                               double* __restrict__ part, CGState* __restrict__ st,
                                               const int* __restrict__ done = nullptr) {
  // the block's loads go out before gamma's reduction, which they do not depend on, and
  // before the done flag (when given) is tested
  const int64_t j = (int64_t)bx * VCHUNK + 4 * threadIdx.x;
  const bool in = j < Dp;
  const int64_t o = (int64_t)q * Dp + j;
  f32x4 mi, x, r, p, ps;
  if (in) {
    mi = *reinterpret_cast<const f32x4*>(minv + j);
    if constexpr (XU) {
      x = *reinterpret_cast<const f32x4*>(X + o);
      p = *reinterpret_cast<const f32x4*>(Pd + o);
    }
    r = *reinterpret_cast<const f32x4*>(R + o);
    ps = *reinterpret_cast<const f32x4*>(Psi + o);
  }
  GammaIn gin;
  if (!PRE && threadIdx.x < 64) gin = column_gamma_load(q, nbx, pipart, st);
  if (done && *done) return;
  if (!XU && bx == 0 && q == 0 && threadIdx.x == 0) st->xpend = 1;
  double gam;
  if (PRE) {
    gam = st->gamma[q];
  } else {
    __shared__ double s_gam;
    if (threadIdx.x < 64) {
      const double g = column_gamma_finish(q, nbx, pipart, st, bx == 0, gin);
      if (threadIdx.x == 0) s_gam = g;
    }
    __syncthreads();
    gam = s_gam;
  }
  double rr = 0.0, rw = 0.0;
  if (in) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if constexpr (XU) x[e] = (float)((double)x[e] + gam * (double)p[e]);
      r[e] = (float)((double)r[e] - gam * (double)ps[e]);
      const double rd = (double)r[e];
      rr += rd * rd;
      rw += rd * ((double)mi[e] * rd);
    }
    if constexpr (XU) {
      if constexpr (NT) __builtin_nontemporal_store(x, reinterpret_cast<f32x4*>(X + o));
      else *reinterpret_cast<f32x4*>(X + o) = x;
    }
    // R too once the columns are long enough for gamma to come precomputed (over 128
    // chunks): the vectors then far exceed the L2s, and a plain store leaves dirty lines
    // that the end of the launch writes back
    if constexpr (NT && PRE) __builtin_nontemporal_store(r, reinterpret_cast<f32x4*>(R + o));
    else *reinterpret_cast<f32x4*>(R + o) = r;
  }
  rr = block_sum(rr);
  rw = block_sum(rw);
  if (threadIdx.x == 0) {
    part[((int64_t)q * nbx + bx) * 2 + 0] = rr;
    part[((int64_t)q * nbx + bx) * 2 + 1] = rw;
  }
}

// One block: ||R_q||^2 and rho'_q from the partials (one wave per column, any block
// size), the stop rule of Algorithm 2 (joint Frobenius ratio, or per-column freezing),
// steps, eta_q = rho'_q / rho_q.  The block is on the critical path of its launch, so its
// global loads go out early: the state's entries first, then, with at most one partial
// per lane and column, the partials of SCB_BATCH of the wave's columns at once (the
// additions keep the order of the one-column loop; a larger batch costs the launch's
// other blocks occupancy).
constexpr int SCB_BATCH = 6;
template <int UNR = 8>
__device__ __forceinline__ void cg_scalars_block(const SolveCfg& c, int nbx, const double* __restrict__ part,
                                                 CGState* __restrict__ st) {
  __shared__ double s_rr[QMAX], s_rw[QMAX];
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63, nw = blockDim.x >> 6;
  const int q = threadIdx.x;
  int act = 0;
  double bn2 = 0.0, old = 0.0, bnorm2 = 0.0;
  int steps = 0;
  if (q < c.Q) {
    act = st->active[q];
    bn2 = st->bn2[q];
    old = st->rho[q];
  }
  if (threadIdx.x == 0) {
    bnorm2 = st->bnorm2;
    steps = st->steps;
  }
  if (nbx <= 64) {
    for (int q0 = wv; q0 < c.Q; q0 += SCB_BATCH * nw) {
      double2 v[SCB_BATCH];
#pragma unroll
      for (int k = 0; k < SCB_BATCH; ++k) {
        const int qk = q0 + k * nw;
        if (qk < c.Q && ln < nbx) v[k] = reinterpret_cast<const double2*>(part + (int64_t)qk * nbx * 2)[ln];
      }
#pragma unroll
      for (int k = 0; k < SCB_BATCH; ++k) {
        const int qk = q0 + k * nw;
        if (qk >= c.Q) break;  // wave-uniform
        double a = 0.0, b = 0.0;
        if (ln < nbx) {
          a += v[k].x;
          b += v[k].y;
        }
        a = wave_sum(a);
        b = wave_sum(b);
        if (ln == 0) {
          s_rr[qk] = a;
          s_rw[qk] = b;
        }
      }
    }
  } else {
    for (int qk = wv; qk < c.Q; qk += nw) {
      const double2* pq = reinterpret_cast<const double2*>(part + (int64_t)qk * nbx * 2);
      double a = 0.0, b = 0.0;
#pragma unroll UNR
      for (int i = ln; i < nbx; i += 64) {  // loads issued together, additions in order
        const double2 v = pq[i];
        a += v.x;
        b += v.y;
      }
      a = wave_sum(a);
      b = wave_sum(b);
      if (ln == 0) {
        s_rr[qk] = a;
        s_rw[qk] = b;
      }
    }
  }
  __syncthreads();
  // per column, one thread each: the column stop test (column mode), ||R_q||^2, eta and rho
  __shared__ int s_act[QMAX];
  if (q < c.Q) {
    if (c.stop_mode != 0 && act && sqrt(s_rr[q] / bn2) <= c.tol) {
      act = 0;
      st->active[q] = 0;
    }
    s_act[q] = act;
    st->rn2[q] = s_rr[q];
    st->eta[q] = (old != 0.0) ? s_rw[q] / old : 0.0;
    st->rho[q] = s_rw[q];
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double rsum = 0.0;
  int nact = 0;
  for (int k = 0; k < c.Q; ++k) {
    rsum += s_rr[k];
    nact += s_act[k];
  }
  const double delta = sqrt(rsum / bnorm2);
  st->delta = delta;
  steps += 1;
  st->steps = steps;
  int done = (c.stop_mode == 0) ? (delta <= c.tol) : (nact == 0);
  if (steps >= c.U) done = 1;
  st->done = done;
}

// P = M^-1 R + eta P (FP32, and bf16 hi/lo when PdH is not null, and the third slice
// when PdX is not null; column-major slices: the interleaved layout of the FIR dictionary
// has a kernel of its own).  Two halves, so that a kernel can issue the tile's loads
// before it reduces eta, on which they do not depend.  NT: P stored non-temporally (the
// slices are what the operator reads).
struct DirTile {
  f32x4 mi, r, p;
  bool in;
};
__device__ __forceinline__ DirTile cg_direction_load(int bx, int q, int64_t Dp, const float* __restrict__ minv,
                                                     const float* __restrict__ R, const float* __restrict__ Pd) {
  DirTile d;
  const int64_t j = (int64_t)bx * VCHUNK + 4 * threadIdx.x;
  d.in = j < Dp;
  if (d.in) {
    const int64_t o = (int64_t)q * Dp + j;
    d.mi = *reinterpret_cast<const f32x4*>(minv + j);
    d.r = *reinterpret_cast<const f32x4*>(R + o);
    d.p = *reinterpret_cast<const f32x4*>(Pd + o);
  }
  return d;
}
template <bool NT = false>
__device__ __forceinline__ void cg_direction_store(const DirTile& d, int bx, int q, int64_t Dp, double eta,
                                                   float* __restrict__ Pd, uint16_t* __restrict__ PdH,
                                                   uint16_t* __restrict__ PdL, uint16_t* __restrict__ PdX) {
  if (!d.in) return;
  const int64_t o = (int64_t)q * Dp + (int64_t)bx * VCHUNK + 4 * threadIdx.x;
  f32x4 p;
#pragma unroll
  for (int e = 0; e < 4; ++e) p[e] = (float)((double)d.mi[e] * (double)d.r[e] + eta * (double)d.p[e]);
  if constexpr (NT) __builtin_nontemporal_store(p, reinterpret_cast<f32x4*>(Pd + o));
  else *reinterpret_cast<f32x4*>(Pd + o) = p;
  if (PdH) store_split4<true>(PdH, PdL, o, p, PdX);
}

}  // namespace cofem
