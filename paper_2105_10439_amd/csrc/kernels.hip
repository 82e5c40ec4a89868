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
// transpose is needed), with the right-hand-side block read through L2.
#include "kernels.h"

#include <algorithm>

namespace cofem {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8_t;
typedef __attribute__((ext_vector_type(4))) float f32x4;

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------
// SplitMix64 finaliser (Steele, Lea & Flood 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// Word j of the stream started at the iteration key (output j + 1).
__device__ __forceinline__ uint64_t probe_word(uint64_t key, int64_t j) {
  return mix64(key + (uint64_t)(j + 1) * GOLDEN_GAMMA);
}
__device__ __forceinline__ float probe_sign(uint64_t w, int k) { return ((w >> k) & 1ull) ? -1.0f : 1.0f; }

// float -> bfloat16, round to nearest even (NaN -> quiet NaN).
__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_val(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// x = hi + lo + O(2^-17 |x|): hi = RNE(x), lo = RNE(x - hi) (x - hi is exact in FP32).
__device__ __forceinline__ void split_bf16(float x, uint16_t& hi, uint16_t& lo) {
  hi = bf16_rne(x);
  lo = bf16_rne(x - bf16_val(hi));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double ld_agent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Returns true in exactly one block: the last of `total` blocks to arrive.
// Only thread 0 of a block may have written the block's partial result before
// the call; it publishes it (release) before counting in, and the last block
// acquires before it reads the partials of the others.
__device__ bool arrive_last(unsigned* cnt, unsigned total) {
  __shared__ int s_last;
  if (threadIdx.x == 0) {
    __threadfence();
    unsigned prev = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    s_last = (prev + 1u == total) ? 1 : 0;
    if (s_last) __threadfence();
  }
  __syncthreads();
  return s_last != 0;
}

// Sum of v over the 256 threads of a block, in a fixed order; result in thread 0.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double sh[4];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = ((sh[0] + sh[1]) + sh[2]) + sh[3];
  __syncthreads();
  return r;
}
__device__ __forceinline__ void reset_counter(unsigned* cnt) {
  __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum part[b * stride + off] over b < nblk within one wave, in a fixed order.
__device__ __forceinline__ double wave_sum_parts(const double* part, int nblk, int stride, int off) {
  const int lane = threadIdx.x & 63;
  double a = 0.0;
  for (int b = lane; b < nblk; b += 64) a += ld_agent(part + (int64_t)b * stride + off);
  return wave_sum(a);
}

// ---------------------------------------------------------------------------
// setup kernels
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_dict_layouts(const float* __restrict__ phi, int64_t N, int64_t D,
                                                      int64_t Np, int64_t Dp, float* __restrict__ phi32,
                                                      float* __restrict__ phi32T, uint16_t* __restrict__ phi16,
                                                      uint16_t* __restrict__ phi16T) {
  __shared__ float tile[64][65];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t j0 = (int64_t)blockIdx.x * 64, i0 = (int64_t)blockIdx.y * 64;
  for (int r = ty; r < 64; r += 4) {
    const int64_t i = i0 + r, j = j0 + tx;
    const float v = (i < N && j < D) ? phi[i * D + j] : 0.0f;
    if (phi32) phi32[i * Dp + j] = v;
    if (phi16) phi16[i * Dp + j] = bf16_rne(v);
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int64_t j = j0 + r, i = i0 + tx;
    const float v = tile[tx][r];
    if (phi32T) phi32T[j * Np + i] = v;
    if (phi16T) phi16T[j * Np + i] = bf16_rne(v);
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
__global__ __launch_bounds__(256) void k_rhs(const T* __restrict__ MT, int64_t Np, int64_t Dp,
                                             const float* __restrict__ y, double beta, float* __restrict__ b) {
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int ln = threadIdx.x & 63;
  if (j >= Dp) return;
  const T* row = MT + j * Np;
  double acc = 0.0;
  for (int64_t i = ln; i < Np; i += 64) acc += ld_val<T>(row, i) * (double)y[i];
  acc = wave_sum(acc);
  if (ln == 0) b[j] = (float)(beta * acc);
}

__global__ void k_fill(float* x, float v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ void k_state_reset(CGState* st, int Q) {
  int* w = reinterpret_cast<int*>(st);
  const int n = (int)(sizeof(CGState) / sizeof(int));
  for (int i = threadIdx.x; i < n; i += blockDim.x) w[i] = 0;
}

// ---------------------------------------------------------------------------
// per-EM-iteration kernels (Algorithm 1 around Algorithm 2)
// ---------------------------------------------------------------------------
// B = [b | p_1..p_K | 0], X = 0, R = B, W = M^-1 R, Pd = W, rho, ||B_q||^2.
__global__ __launch_bounds__(VBLOCK) void k_em_init(SolveCfg c, uint64_t key, int64_t D, int64_t Dp,
                                                    const float* __restrict__ b, const float* __restrict__ theta,
                                                    const float* __restrict__ alpha, float* __restrict__ minv,
                                                    float* __restrict__ X, float* __restrict__ R,
                                                    float* __restrict__ Pd, uint16_t* __restrict__ PdH,
                                                    uint16_t* __restrict__ PdL, double* __restrict__ part,
                                                    CGState* __restrict__ st) {
  const int64_t j = (int64_t)blockIdx.x * VBLOCK + threadIdx.x;  // grid covers Dp exactly
  const bool real = j < D;
  const float mi = (float)(1.0 / (c.beta * (double)theta[j] + (double)alpha[j]));
  minv[j] = mi;
  const double mid = (double)mi;
  const uint64_t w = real ? probe_word(key, j) : 0ull;
  const float bj = real ? b[j] : 0.0f;
  for (int q = 0; q < c.Qp; ++q) {
    float bq = 0.0f;
    if (real) bq = (q == 0) ? bj : (q <= c.K ? probe_sign(w, q - 1) : 0.0f);
    const int64_t o = (int64_t)q * Dp + j;
    X[o] = 0.0f;
    R[o] = bq;
    const float p = (float)(mid * (double)bq);
    Pd[o] = p;
    if (PdH) {
      uint16_t h, l;
      split_bf16(p, h, l);
      PdH[o] = h;
      PdL[o] = l;
    }
  }
  // rho_0 = sum b_j (minv_j b_j); rho_q = sum minv_j (probe entries square to 1); ||b||^2.
  double s_minv = real ? mid : 0.0;
  double s_bw = real ? (double)bj * (mid * (double)bj) : 0.0;
  double s_bb = real ? (double)bj * (double)bj : 0.0;
  __shared__ double sh[3][VBLOCK / 64];
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  s_minv = wave_sum(s_minv);
  s_bw = wave_sum(s_bw);
  s_bb = wave_sum(s_bb);
  if (ln == 0) {
    sh[0][wv] = s_minv;
    sh[1][wv] = s_bw;
    sh[2][wv] = s_bb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int a = 0; a < 3; ++a) {
      double t = 0.0;
      for (int v = 0; v < VBLOCK / 64; ++v) t += sh[a][v];
      part[(int64_t)blockIdx.x * 3 + a] = t;
    }
  }
  if (!arrive_last(&st->cnt[0], gridDim.x)) return;
  if (wv == 0) {
    const double t_minv = wave_sum_parts(part, gridDim.x, 3, 0);
    const double t_bw = wave_sum_parts(part, gridDim.x, 3, 1);
    const double t_bb = wave_sum_parts(part, gridDim.x, 3, 2);
    if (ln == 0) {
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
      reset_counter(&st->cnt[0]);
    }
  }
}

// mu, s = (1/K) sum_k p_k x_k, and the M-step alpha = 1 / max(mu^2 + s, floor).
__global__ __launch_bounds__(VBLOCK) void k_mstep(SolveCfg c, uint64_t key, int64_t D, int64_t Dp,
                                                  const float* __restrict__ X, float* __restrict__ mu,
                                                  float* __restrict__ s_out, float* __restrict__ alpha,
                                                  double floor, int do_mstep, CGState* __restrict__ st) {
  const int64_t j = (int64_t)blockIdx.x * VBLOCK + threadIdx.x;
  int clamped = 0;
  if (j < D) {
    const float m = X[j];
    const uint64_t w = probe_word(key, j);
    double acc = 0.0;
    for (int k = 0; k < c.K; ++k) acc += (double)probe_sign(w, k) * (double)X[(int64_t)(k + 1) * Dp + j];
    const double s = acc / (double)c.K;
    mu[j] = m;
    s_out[j] = (float)s;
    if (do_mstep) {
      double den = (double)m * (double)m + s;
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
// operator: skinny MFMA contractions
// ---------------------------------------------------------------------------
// Tile order of the contractions.  Workgroups of a 1-D grid are dispatched
// round-robin over the 8 XCDs (workgroup L runs on XCD L % 8), and each XCD has
// its own L2.  Blocks that share a split of the reduction dimension read the
// same slice of the right-hand-side block, so they are placed on the same XCD.
__device__ __forceinline__ void tile_of(int L, int nrb, int splits, int& rb, int& sp) {
  const int xcd = L & 7, slot = L >> 3;
  if ((splits & 7) == 0) {
    const int spx = splits >> 3;
    sp = xcd * spx + slot % spx;
    rb = slot / spx;
  } else if ((8 % splits) == 0 && (nrb % (8 / splits)) == 0) {
    const int g = 8 / splits;
    sp = xcd / g;
    rb = slot * g + xcd % g;
  } else {
    rb = L % nrb;
    sp = L / nrb;
  }
}

// Ypart[split][q][row] = sum_{k in split} M[row, k] * (ZH[q, k] + ZL[q, k]).
//
// Block = 5 waves.  Waves 0-3 compute: wave w owns rows row0 .. row0 + 16 RT - 1
// and all CT*16 columns, and streams its rows of M from HBM straight into VGPRs
// in the MFMA operand layout, one stage ahead.  Wave 4 is a producer: it copies
// the right-hand-side fragments of the next stage (KS * CT * {hi, lo}, 1 KB each,
// already in MFMA lane order) from L2 into a double-buffered LDS tile, so the
// compute waves never wait on those loads (vmcnt counts in issue order per wave).
// v_mfma_f32_16x16x32_bf16: lane l holds A[l%16][8(l/16) .. +8), B[8(l/16) .. +8)[l%16]
// and returns D[4(l/16) .. +4)[l%16].
template <int RT, int CT, int KS>
__global__ __launch_bounds__(320, 2) void k_gemm_bf16(const uint16_t* __restrict__ M, int64_t ldm,
                                                      const uint16_t* __restrict__ ZH,
                                                      const uint16_t* __restrict__ ZL, int64_t ldz,
                                                      float* __restrict__ Yp, int64_t ldy, int Qp, int64_t kchunk,
                                                      int64_t kdim, int nrb, int splits,
                                                      const int* __restrict__ done) {
  if (done && *done) return;
  constexpr int NF = KS * CT * 2;  // fragments per stage
  constexpr int SK = 32 * KS;      // k per stage
  __shared__ bf16x8_t sB[2][NF][64];
  int rb, sp;
  tile_of(blockIdx.x, nrb, splits, rb, sp);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const int64_t kb = (int64_t)sp * kchunk;
  const int64_t ke = (kb + kchunk < kdim) ? kb + kchunk : kdim;
  const int nst = (ke > kb) ? (int)((ke - kb) / SK) : 0;
  if (wave == 4) {
    const uint16_t* src[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int s = f / (CT * 2), rem = f % (CT * 2), ct = rem >> 1, hl = rem & 1;
      src[f] = (hl ? ZL : ZH) + (int64_t)(ct * 16 + r16) * ldz + kb + s * 32 + 8 * g;
    }
    if (nst > 0) {
#pragma unroll
      for (int f = 0; f < NF; ++f) sB[0][f][lane] = *reinterpret_cast<const bf16x8_t*>(src[f]);
    }
    __syncthreads();
    for (int st = 0; st < nst; ++st) {
      // the next stage's fragments (the last stage reloads its own into the idle buffer)
      const int64_t off = (int64_t)((st + 1 < nst) ? st + 1 : st) * SK;
      bf16x8_t t[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) t[f] = *reinterpret_cast<const bf16x8_t*>(src[f] + off);
#pragma unroll
      for (int f = 0; f < NF; ++f) sB[(st + 1) & 1][f][lane] = t[f];
      __syncthreads();
    }
    return;
  }
  const int64_t row0 = (int64_t)rb * (64 * RT) + (int64_t)wave * (16 * RT);
  f32x4 acc[RT][CT];
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int b = 0; b < CT; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  const uint16_t* ap[RT];
#pragma unroll
  for (int a = 0; a < RT; ++a) ap[a] = M + (row0 + a * 16 + r16) * ldm + kb + 8 * g;
  bf16x8_t acur[RT][KS];
  if (nst > 0) {
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
      for (int s = 0; s < KS; ++s) acur[a][s] = *reinterpret_cast<const bf16x8_t*>(ap[a] + s * 32);
  }
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    // prefetch the next stage (the last stage re-reads its own rows: always in bounds);
    // no branch here, so the prefetch stays in flight across the stage
    const int64_t off = (int64_t)((st + 1 < nst) ? st + 1 : st) * SK;
    bf16x8_t anxt[RT][KS];
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
      for (int s = 0; s < KS; ++s) anxt[a][s] = *reinterpret_cast<const bf16x8_t*>(ap[a] + off + s * 32);
    __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of this stage's MFMAs
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      bf16x8_t bh[CT], bl[CT];
#pragma unroll
      for (int b = 0; b < CT; ++b) {
        bh[b] = sB[buf][(s * CT + b) * 2 + 0][lane];
        bl[b] = sB[buf][(s * CT + b) * 2 + 1][lane];
      }
#pragma unroll
      for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int b = 0; b < CT; ++b) {
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(acur[a][s], bh[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(acur[a][s], bl[b], acc[a][b], 0, 0, 0);
        }
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
      for (int s = 0; s < KS; ++s) acur[a][s] = anxt[a][s];
  }
  float* yb = Yp + (int64_t)sp * Qp * ldy;
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int b = 0; b < CT; ++b) {
      const int64_t q = b * 16 + r16;
      const int64_t row = row0 + a * 16 + 4 * g;
      *reinterpret_cast<f32x4*>(yb + q * ldy + row) = acc[a][b];
    }
}

// FP32 version with v_mfma_f32_16x16x4_f32.  Each lane holds 4 consecutive k of
// its row (and of its column of Z) and feeds element e to the e-th MFMA, so the
// four MFMAs of a 16-k step see the same k order in both operands.  Same wave
// roles and staging as above (1 KB fragment per 16-k step and column tile).
template <int RT, int CT, int KS>
__global__ __launch_bounds__(320, 2) void k_gemm_f32(const float* __restrict__ M, int64_t ldm,
                                                     const float* __restrict__ Z, int64_t ldz,
                                                     float* __restrict__ Yp, int64_t ldy, int Qp, int64_t kchunk,
                                                     int64_t kdim, int nrb, int splits,
                                                     const int* __restrict__ done) {
  if (done && *done) return;
  constexpr int NF = KS * CT;
  constexpr int SK = 16 * KS;
  __shared__ f32x4 sB[2][NF][64];
  int rb, sp;
  tile_of(blockIdx.x, nrb, splits, rb, sp);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const int64_t kb = (int64_t)sp * kchunk;
  const int64_t ke = (kb + kchunk < kdim) ? kb + kchunk : kdim;
  const int nst = (ke > kb) ? (int)((ke - kb) / SK) : 0;
  if (wave == 4) {
    const float* src[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int s = f / CT, ct = f % CT;
      src[f] = Z + (int64_t)(ct * 16 + r16) * ldz + kb + s * 16 + 4 * g;
    }
    if (nst > 0) {
#pragma unroll
      for (int f = 0; f < NF; ++f) sB[0][f][lane] = *reinterpret_cast<const f32x4*>(src[f]);
    }
    __syncthreads();
    for (int st = 0; st < nst; ++st) {
      const int64_t off = (int64_t)((st + 1 < nst) ? st + 1 : st) * SK;
      f32x4 t[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) t[f] = *reinterpret_cast<const f32x4*>(src[f] + off);
#pragma unroll
      for (int f = 0; f < NF; ++f) sB[(st + 1) & 1][f][lane] = t[f];
      __syncthreads();
    }
    return;
  }
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
  if (nst > 0) {
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
      for (int s = 0; s < KS; ++s) acur[a][s] = *reinterpret_cast<const f32x4*>(ap[a] + s * 16);
  }
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    const int64_t off = (int64_t)((st + 1 < nst) ? st + 1 : st) * SK;
    f32x4 anxt[RT][KS];
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
      for (int s = 0; s < KS; ++s) anxt[a][s] = *reinterpret_cast<const f32x4*>(ap[a] + off + s * 16);
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
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
      for (int s = 0; s < KS; ++s) acur[a][s] = anxt[a][s];
  }
  float* yb = Yp + (int64_t)sp * Qp * ldy;
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int b = 0; b < CT; ++b) {
      const int64_t q = b * 16 + r16;
      const int64_t row = row0 + a * 16 + 4 * g;
      *reinterpret_cast<f32x4*>(yb + q * ldy + row) = acc[a][b];
    }
}

// V[q][i] = sum_split Ypart[split][q][i] (fixed split order).
__global__ __launch_bounds__(256) void k_finish_pass1(const float* __restrict__ Yp, int splits, int64_t Np,
                                                      float* __restrict__ V, uint16_t* __restrict__ VH,
                                                      uint16_t* __restrict__ VL, int Qp,
                                                      const int* __restrict__ done) {
  if (*done) return;
  const int q = blockIdx.y;
  const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  if (i >= Np) return;
  const int64_t o = (int64_t)q * Np + i;
  f32x4 v = *reinterpret_cast<const f32x4*>(Yp + o);
  for (int sp = 1; sp < splits; ++sp) v += *reinterpret_cast<const f32x4*>(Yp + (int64_t)sp * Qp * Np + o);
  if (V) *reinterpret_cast<f32x4*>(V + o) = v;
  if (VH) {
    uint16_t h[4], l[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) split_bf16(v[e], h[e], l[e]);
    *reinterpret_cast<uint2*>(VH + o) = make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16),
                                                   (uint32_t)h[2] | ((uint32_t)h[3] << 16));
    *reinterpret_cast<uint2*>(VL + o) = make_uint2((uint32_t)l[0] | ((uint32_t)l[1] << 16),
                                                   (uint32_t)l[2] | ((uint32_t)l[3] << 16));
  }
}

// The per-column vector kernels run one block per (chunk of VCHUNK coordinates,
// column q): each thread owns 4 consecutive coordinates of one column, and a
// block contributes one partial per reduced quantity, stored at [q][chunk].
constexpr int VCHUNK = 1024;

// Psi = beta * sum_split Ypart + alpha Pd, and the block's partial of
// pi_q = sum_j Pd_jq Psi_jq, stored at pipart[q * nbx + chunk].
__global__ __launch_bounds__(VBLOCK) void k_finish_pass2(SolveCfg c, const float* __restrict__ Yp, int splits,
                                                         int64_t Dp, const float* __restrict__ alpha,
                                                         const float* __restrict__ Pd, float* __restrict__ Psi,
                                                         double* __restrict__ pipart, const CGState* __restrict__ st) {
  if (st->done) return;
  const int q = blockIdx.y, nbx = gridDim.x;
  const int64_t j = (int64_t)blockIdx.x * VCHUNK + 4 * threadIdx.x;
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
  if (threadIdx.x == 0) pipart[(int64_t)q * nbx + blockIdx.x] = acc;
}

// pi_q from its nbx partials (fixed order), the same value in every block that asks.
__device__ __forceinline__ double column_pi(const double* pipart, int q, int nbx) {
  __shared__ double s_pi;
  if (threadIdx.x < 64) {
    double a = 0.0;
    for (int b = threadIdx.x; b < nbx; b += 64) a += pipart[(int64_t)q * nbx + b];
    a = wave_sum(a);
    if (threadIdx.x == 0) s_pi = a;
  }
  __syncthreads();
  return s_pi;
}

// gamma_q = rho_q / pi_q; X += gamma Pd, R -= gamma Psi; partials of ||R_q||^2 and
// rho'_q = sum R (M^-1 R) at part[(q * nbx + chunk) * 2 + {0, 1}].
__global__ __launch_bounds__(VBLOCK) void k_cg_update(SolveCfg c, int64_t Dp, const float* __restrict__ minv,
                                                      float* __restrict__ X, float* __restrict__ R,
                                                      const float* __restrict__ Pd, const float* __restrict__ Psi,
                                                      const double* __restrict__ pipart, double* __restrict__ part,
                                                      CGState* __restrict__ st) {
  if (st->done) return;
  const int q = blockIdx.y, nbx = gridDim.x;
  const double pi = column_pi(pipart, q, nbx);
  const double rho = st->rho[q];
  const int act = st->active[q];
  const double gam = (act && pi > 0.0) ? rho / pi : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->pi[q] = pi;
    st->gamma[q] = gam;
    if (act && !(pi > 0.0) && rho != 0.0) {  // breakdown: freeze the column
      st->active[q] = 0;
      atomicAdd(&st->breakdown, 1);
    }
  }
  const int64_t j = (int64_t)blockIdx.x * VCHUNK + 4 * threadIdx.x;
  double rr = 0.0, rw = 0.0;
  if (j < Dp) {
    const int64_t o = (int64_t)q * Dp + j;
    const f32x4 mi = *reinterpret_cast<const f32x4*>(minv + j);
    f32x4 x = *reinterpret_cast<const f32x4*>(X + o);
    f32x4 r = *reinterpret_cast<const f32x4*>(R + o);
    const f32x4 p = *reinterpret_cast<const f32x4*>(Pd + o);
    const f32x4 ps = *reinterpret_cast<const f32x4*>(Psi + o);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      x[e] = (float)((double)x[e] + gam * (double)p[e]);
      r[e] = (float)((double)r[e] - gam * (double)ps[e]);
      const double rd = (double)r[e];
      rr += rd * rd;
      rw += rd * ((double)mi[e] * rd);
    }
    *reinterpret_cast<f32x4*>(X + o) = x;
    *reinterpret_cast<f32x4*>(R + o) = r;
  }
  rr = block_sum(rr);
  rw = block_sum(rw);
  if (threadIdx.x == 0) {
    part[((int64_t)q * nbx + blockIdx.x) * 2 + 0] = rr;
    part[((int64_t)q * nbx + blockIdx.x) * 2 + 1] = rw;
  }
}

// One block: ||R_q||^2 and rho'_q from the partials (fixed order), the stop rule of
// Algorithm 2 (joint Frobenius ratio, or per-column freezing), eta_q = rho'_q / rho_q.
__global__ __launch_bounds__(VBLOCK) void k_cg_scalars(SolveCfg c, int nbx, const double* __restrict__ part,
                                                       CGState* __restrict__ st) {
  if (st->done) return;
  __shared__ double s_rr[QMAX], s_rw[QMAX];
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  for (int q = wv; q < c.Q; q += 4) {
    double a = 0.0, b = 0.0;
    for (int i = ln; i < nbx; i += 64) {
      a += part[((int64_t)q * nbx + i) * 2 + 0];
      b += part[((int64_t)q * nbx + i) * 2 + 1];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (ln == 0) {
      s_rr[q] = a;
      s_rw[q] = b;
    }
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double rsum = 0.0;
  for (int q = 0; q < c.Q; ++q) rsum += s_rr[q];
  const double delta = sqrt(rsum / st->bnorm2);
  st->delta = delta;
  const int steps = st->steps + 1;
  st->steps = steps;
  int done = 0;
  if (c.stop_mode == 0) {
    if (delta <= c.tol) done = 1;
  } else {
    int nact = 0;
    for (int q = 0; q < c.Q; ++q) {
      if (st->active[q] && sqrt(s_rr[q] / st->bn2[q]) <= c.tol) st->active[q] = 0;
      nact += st->active[q];
    }
    if (nact == 0) done = 1;
  }
  if (steps >= c.U) done = 1;
  for (int q = 0; q < c.Q; ++q) {
    st->rn2[q] = s_rr[q];
    const double old = st->rho[q];
    st->eta[q] = (old != 0.0) ? s_rw[q] / old : 0.0;
    st->rho[q] = s_rw[q];
  }
  st->done = done;
}

// One block: pi_q into the state (used by the single-application test hook).
__global__ __launch_bounds__(VBLOCK) void k_reduce_pi(int Q, int nbx, const double* __restrict__ pipart,
                                                      CGState* __restrict__ st) {
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  for (int q = wv; q < Q; q += 4) {
    double a = 0.0;
    for (int i = ln; i < nbx; i += 64) a += pipart[(int64_t)q * nbx + i];
    a = wave_sum(a);
    if (ln == 0) st->pi[q] = a;
  }
}

// Pd = M^-1 R + eta Pd.
__global__ __launch_bounds__(VBLOCK) void k_cg_direction(SolveCfg c, int64_t Dp, const float* __restrict__ minv,
                                                         const float* __restrict__ R, float* __restrict__ Pd,
                                                         uint16_t* __restrict__ PdH, uint16_t* __restrict__ PdL,
                                                         const CGState* __restrict__ st) {
  if (st->done) return;
  const int q = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * VCHUNK + 4 * threadIdx.x;
  if (j >= Dp) return;
  const double eta = st->eta[q];
  const int64_t o = (int64_t)q * Dp + j;
  const f32x4 mi = *reinterpret_cast<const f32x4*>(minv + j);
  const f32x4 r = *reinterpret_cast<const f32x4*>(R + o);
  f32x4 p = *reinterpret_cast<const f32x4*>(Pd + o);
#pragma unroll
  for (int e = 0; e < 4; ++e) p[e] = (float)((double)mi[e] * (double)r[e] + eta * (double)p[e]);
  *reinterpret_cast<f32x4*>(Pd + o) = p;
  if (PdH) {
    uint16_t h[4], l[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) split_bf16(p[e], h[e], l[e]);
    *reinterpret_cast<uint2*>(PdH + o) = make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16),
                                                    (uint32_t)h[2] | ((uint32_t)h[3] << 16));
    *reinterpret_cast<uint2*>(PdL + o) = make_uint2((uint32_t)l[0] | ((uint32_t)l[1] << 16),
                                                    (uint32_t)l[2] | ((uint32_t)l[3] << 16));
  }
}

// ---------------------------------------------------------------------------
// test-hook helpers
// ---------------------------------------------------------------------------
__global__ void k_pack_block(const float* __restrict__ src, int ncols, int64_t D, int Qp, int64_t Dp,
                             float* __restrict__ dst, uint16_t* __restrict__ dH, uint16_t* __restrict__ dL) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (j >= Dp || q >= Qp) return;
  const float v = (q < ncols && j < D) ? src[(int64_t)q * D + j] : 0.0f;
  const int64_t o = (int64_t)q * Dp + j;
  dst[o] = v;
  if (dH) {
    uint16_t h, l;
    split_bf16(v, h, l);
    dH[o] = h;
    dL[o] = l;
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

void launch_dict_layouts(const float* phi, int64_t N, int64_t D, int64_t Np, int64_t Dp, float* phi32,
                         float* phi32T, uint16_t* phi16, uint16_t* phi16T, hipStream_t s) {
  dim3 grid((unsigned)(Dp / 64), (unsigned)(Np / 64));
  hipLaunchKernelGGL(k_dict_layouts, grid, dim3(256), 0, s, phi, N, D, Np, Dp, phi32, phi32T, phi16, phi16T);
}

void launch_theta(const float* phi, int64_t N, int64_t D, int64_t Dp, int jacobi, float* theta, hipStream_t s) {
  hipLaunchKernelGGL(k_theta, dim3(cdiv(Dp, 256)), dim3(256), 0, s, phi, N, D, Dp, jacobi, theta);
}

void launch_rhs(const float* phi32T, const uint16_t* phi16T, int64_t Np, int64_t Dp, const float* y, double beta,
                float* b, hipStream_t s) {
  if (phi32T)
    hipLaunchKernelGGL(k_rhs<float>, dim3(cdiv(Dp, 4)), dim3(256), 0, s, phi32T, Np, Dp, y, beta, b);
  else
    hipLaunchKernelGGL(k_rhs<uint16_t>, dim3(cdiv(Dp, 4)), dim3(256), 0, s, phi16T, Np, Dp, y, beta, b);
}

void launch_fill(float* x, float v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(cdiv(n, 256)), dim3(256), 0, s, x, v, n);
}

void launch_state_reset(CGState* st, int Q, hipStream_t s) {
  hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(256), 0, s, st, Q);
}

void launch_em_init(const SolveCfg& c, uint64_t key, int64_t D, int64_t Dp, const float* b, const float* theta,
                    const float* alpha, float* minv, float* X, float* R, float* Pd, uint16_t* PdH,
                    uint16_t* PdL, double* part, CGState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_em_init, dim3((unsigned)(Dp / VBLOCK)), dim3(VBLOCK), 0, s, c, key, D, Dp, b, theta,
                     alpha, minv, X, R, Pd, PdH, PdL, part, st);
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
constexpr int KS_F32 = 4;   // 16-k steps per stage (64 k)

template <int RT>
static void gemm_bf16_rt(const GemmCfg& g, const uint16_t* M, int64_t rows, int64_t kdim, const uint16_t* ZH,
                         const uint16_t* ZL, int Qp, float* Yp, const int* done, hipStream_t s) {
  const int nrb = (int)(rows / (64 * RT));
  dim3 grid((unsigned)(nrb * g.splits));
  switch (Qp / 16) {
    case 1: hipLaunchKernelGGL((k_gemm_bf16<RT, 1, KS_BF16>), grid, dim3(320), 0, s, M, kdim, ZH, ZL, kdim, Yp, rows, Qp, g.kchunk, kdim, nrb, g.splits, done); break;
    case 2: hipLaunchKernelGGL((k_gemm_bf16<RT, 2, KS_BF16>), grid, dim3(320), 0, s, M, kdim, ZH, ZL, kdim, Yp, rows, Qp, g.kchunk, kdim, nrb, g.splits, done); break;
    case 3: hipLaunchKernelGGL((k_gemm_bf16<RT, 3, KS_BF16>), grid, dim3(320), 0, s, M, kdim, ZH, ZL, kdim, Yp, rows, Qp, g.kchunk, kdim, nrb, g.splits, done); break;
    default: hipLaunchKernelGGL((k_gemm_bf16<RT, 4, KS_BF16>), grid, dim3(320), 0, s, M, kdim, ZH, ZL, kdim, Yp, rows, Qp, g.kchunk, kdim, nrb, g.splits, done); break;
  }
}

void launch_gemm_bf16(const GemmCfg& g, const uint16_t* M, int64_t rows, int64_t kdim, const uint16_t* ZH,
                      const uint16_t* ZL, int Qp, float* Yp, const CGState* st, hipStream_t s) {
  const int* done = st ? &st->done : nullptr;
  if (g.rt == 4) gemm_bf16_rt<4>(g, M, rows, kdim, ZH, ZL, Qp, Yp, done, s);
  else if (g.rt == 2) gemm_bf16_rt<2>(g, M, rows, kdim, ZH, ZL, Qp, Yp, done, s);
  else gemm_bf16_rt<1>(g, M, rows, kdim, ZH, ZL, Qp, Yp, done, s);
}

template <int RT>
static void gemm_f32_rt(const GemmCfg& g, const float* M, int64_t rows, int64_t kdim, const float* Z, int Qp,
                        float* Yp, const int* done, hipStream_t s) {
  const int nrb = (int)(rows / (64 * RT));
  dim3 grid((unsigned)(nrb * g.splits));
  switch (Qp / 16) {
    case 1: hipLaunchKernelGGL((k_gemm_f32<RT, 1, KS_F32>), grid, dim3(320), 0, s, M, kdim, Z, kdim, Yp, rows, Qp, g.kchunk, kdim, nrb, g.splits, done); break;
    case 2: hipLaunchKernelGGL((k_gemm_f32<RT, 2, KS_F32>), grid, dim3(320), 0, s, M, kdim, Z, kdim, Yp, rows, Qp, g.kchunk, kdim, nrb, g.splits, done); break;
    case 3: hipLaunchKernelGGL((k_gemm_f32<RT, 3, KS_F32>), grid, dim3(320), 0, s, M, kdim, Z, kdim, Yp, rows, Qp, g.kchunk, kdim, nrb, g.splits, done); break;
    default: hipLaunchKernelGGL((k_gemm_f32<RT, 4, KS_F32>), grid, dim3(320), 0, s, M, kdim, Z, kdim, Yp, rows, Qp, g.kchunk, kdim, nrb, g.splits, done); break;
  }
}

void launch_gemm_f32(const GemmCfg& g, const float* M, int64_t rows, int64_t kdim, const float* Z, int Qp,
                     float* Yp, const CGState* st, hipStream_t s) {
  const int* done = st ? &st->done : nullptr;
  if (g.rt == 4) gemm_f32_rt<4>(g, M, rows, kdim, Z, Qp, Yp, done, s);
  else if (g.rt == 2) gemm_f32_rt<2>(g, M, rows, kdim, Z, Qp, Yp, done, s);
  else gemm_f32_rt<1>(g, M, rows, kdim, Z, Qp, Yp, done, s);
}

void launch_finish_pass1(const float* Ypart, int splits, int Qp, int64_t Np, float* V, uint16_t* VH,
                         uint16_t* VL, const CGState* st, hipStream_t s) {
  dim3 grid(cdiv(Np, 1024), (unsigned)Qp);
  hipLaunchKernelGGL(k_finish_pass1, grid, dim3(256), 0, s, Ypart, splits, Np, V, VH, VL, Qp, &st->done);
}

void launch_finish_pass2(const SolveCfg& c, const float* Ypart, int splits, int64_t Dp, const float* alpha,
                         const float* Pd, float* Psi, double* pipart, const CGState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_finish_pass2, dim3(cdiv(Dp, VCHUNK), (unsigned)c.Q), dim3(VBLOCK), 0, s, c, Ypart, splits,
                     Dp, alpha, Pd, Psi, pipart, st);
}

void launch_cg_update(const SolveCfg& c, int64_t Dp, const float* minv, float* X, float* R, const float* Pd,
                      const float* Psi, const double* pipart, double* part, CGState* st, hipStream_t s) {
  const unsigned nbx = cdiv(Dp, VCHUNK);
  hipLaunchKernelGGL(k_cg_update, dim3(nbx, (unsigned)c.Q), dim3(VBLOCK), 0, s, c, Dp, minv, X, R, Pd, Psi, pipart,
                     part, st);
  hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(VBLOCK), 0, s, c, (int)nbx, (const double*)part, st);
}

void launch_reduce_pi(int Q, int64_t Dp, const double* pipart, CGState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_pi, dim3(1), dim3(VBLOCK), 0, s, Q, (int)cdiv(Dp, VCHUNK), pipart, st);
}

void launch_cg_direction(const SolveCfg& c, int64_t Dp, const float* minv, const float* R, float* Pd,
                         uint16_t* PdH, uint16_t* PdL, const CGState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_direction, dim3(cdiv(Dp, VCHUNK), (unsigned)c.Q), dim3(VBLOCK), 0, s, c, Dp, minv, R, Pd,
                     PdH, PdL, st);
}

void launch_pack_block(const float* src, int ncols, int64_t D, int Qp, int64_t Dp, float* dst, uint16_t* dH,
                       uint16_t* dL, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_block, dim3(cdiv(Dp, 256), (unsigned)Qp), dim3(256), 0, s, src, ncols, D, Qp, Dp, dst,
                     dH, dL);
}
void launch_unpack_block(const float* src, int ncols, int64_t D, int64_t Dp, float* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_unpack_block, dim3(cdiv(D, 256), (unsigned)ncols), dim3(256), 0, s, src, ncols, D, Dp,
                     dst);
}
void launch_copy_pad(const float* src, int64_t n, int64_t np, float pad, float* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_pad, dim3(cdiv(np, 256)), dim3(256), 0, s, src, n, np, pad, dst);
}

}  // namespace cofem
