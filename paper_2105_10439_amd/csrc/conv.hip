// The convolutional dictionary of Sec. V-A.2 on gfx950: N = D and
// Phi_ij = h[i - j] for 0 <= i - j < L, a lower-triangular band Toeplitz matrix.
// Applying it is a causal FIR filter and applying Phi^T the time-reversed one, so
// the operator Psi = beta Phi^T (Phi Pd) + alpha Pd of Algorithm 2 costs 2 L
// multiply-adds per coordinate and right-hand side and never forms Phi.
//
// Both filters run on the matrix cores.  Cut the time axis into 16-sample
// blocks: output block a of the causal filter is sum_d T_d Pd_{a-d}, where T_d is
// the 16 x 16 Toeplitz block T_d[r][c] = h[16 d + r - c] (zero outside [0, L)),
// d = 0 .. NB-1 with NB = floor((L + 14) / 16) + 1 (17 for L = 256, so the
// blocks carry 6 % more multiply-adds than the taps).  A wave owns one 16-column
// tile of right-hand sides and a run of VCHUNK output samples, and the input
// blocks pass through a sliding window of VGPR slots, so each input sample is
// loaded once per run and used NB times.  The anti-causal filter is the same with
// T_d^T and the window running forward, and it carries the rest of the operator
// application: Psi = beta (.) + alpha Pd and the FP64 partials of
// pi_q = sum_j Pd_jq Psi_jq, one per (column, VCHUNK run), in the layout the CG
// update kernel reduces.  FP32 form: two passes (k_conv_f32), V through memory, the
// Toeplitz blocks in VGPRs for the whole run.  bf16 form: one launch per application
// (k_conv_bf16_op), V = Phi Pd kept in registers, the Toeplitz blocks of both filters
// in LDS.
//
// FP32 form: v_mfma_f32_16x16x4_f32, taps and signals in FP32.
// bf16 form: v_mfma_f32_16x16x32_bf16 with the taps rounded to bfloat16 once (the
// dictionary of the precision form) and each signal carried as a hi + lo pair of
// bfloat16 (about 2^-17 relative) in the tile-interleaved layout of sig_index, so a
// wave's load of one block of its 16 columns is one contiguous 1 KB segment (column-major
// signals made it sixteen 64-byte pieces 2 MB apart; the last tile stores only its real
// columns, so padding columns cost no traffic), over 32-sample input blocks: output block
// a = 2 m + par is sum_d T^(par)_d Pd_{m-d} with T^(par)_d[r][c] = h[32 d + 16 par
// + r - c], d = 0 .. NB-1, NB = floor((L + 30) / 32) + 1 (9 for L = 256).
#include <algorithm>

#include "kernels.h"
#include "device_common.h"

namespace cofem {

typedef __attribute__((ext_vector_type(8))) unsigned short u16x8;

// Padded taps: hp[CONV_HOFF + m] = h[m] for 0 <= m < L, zero for the rest of the
// CONV_HPAD entries (every index the Toeplitz blocks touch stays inside).
constexpr int CONV_HOFF = 32;

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------
__global__ void k_conv_taps(const float* __restrict__ h, int L, float* __restrict__ hp32,
                            uint16_t* __restrict__ hp16) {
  for (int i = threadIdx.x; i < CONV_HPAD; i += blockDim.x) {
    const int m = i - CONV_HOFF;
    const float v = (m >= 0 && m < L) ? h[m] : 0.0f;
    hp32[i] = v;
    hp16[i] = bf16_rne(v);
  }
}

// theta_j = sum_i Phi_ij^2 = sum_{t < min(L, D - j)} h[t]^2 (Jacobi, FP64) or 1; padding 1.
__global__ __launch_bounds__(256) void k_conv_theta(const float* __restrict__ hp32, int L, int64_t D, int64_t Dp,
                                                    int jacobi, float* __restrict__ theta) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= Dp) return;
  if (j >= D || !jacobi) {
    theta[j] = 1.0f;
    return;
  }
  const int64_t n = std::min<int64_t>(L, D - j);
  double sq = 0.0;
  for (int64_t t = 0; t < n; ++t) {
    const double v = (double)hp32[CONV_HOFF + t];
    sq += v * v;
  }
  theta[j] = (float)sq;
}

// b_j = beta sum_{t < L, j + t < D} h[t] y_{j+t} (the anti-causal filter of y, FP64
// sums) with the FP32 taps, or with the bfloat16 taps for the bf16 phase.
__global__ __launch_bounds__(256) void k_conv_rhs(const float* __restrict__ hp32, const uint16_t* __restrict__ hp16,
                                                  int L, int64_t D, int64_t Dp, const float* __restrict__ y,
                                                  double beta, float* __restrict__ b) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= Dp) return;
  double acc = 0.0;
  if (j < D) {
    const int64_t n = std::min<int64_t>(L, D - j);
    for (int64_t t = 0; t < n; ++t) {
      const double h = hp16 ? (double)bf16_val(hp16[CONV_HOFF + t]) : (double)hp32[CONV_HOFF + t];
      acc += h * (double)y[j + t];
    }
  }
  b[j] = (float)(beta * acc);
}

// ---------------------------------------------------------------------------
// The two filter passes.  DIR 0: out = Phi in (causal).  DIR 1: out = beta Phi^T in +
// alpha Pd with the pi partials (anti-causal).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void conv_epilogue(const ConvArgs& a, int dir, int64_t q, bool qv, int64_t row, f32x4 v,
                                              const f32x4& al, const f32x4& pd, double& pacc) {
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (row + e >= a.D) v[e] = 0.0f;
  const int64_t o = q * a.Dp + row;
  if (dir == 0) {
    if (qv) {
      if (a.out32) *reinterpret_cast<f32x4*>(a.out32 + o) = v;
      if (a.outH) store_split4(a.outH, a.outL, sig_index(q, row, a.Dp, a.Q), v);
    }
  } else {
    f32x4 ps;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      ps[e] = (float)(a.beta * (double)v[e] + (double)al[e] * (double)pd[e]);
      pacc += (double)pd[e] * (double)ps[e];
    }
    // non-temporal: Psi (Q x D FP32, 88 MB at D = 2^20) is read once, by the update launch,
    // long after these lines would have left the L2
    if (qv) __builtin_nontemporal_store(ps, reinterpret_cast<f32x4*>(a.out32 + o));
  }
}

__device__ __forceinline__ void conv_pi_store(const ConvArgs& a, int64_t q, bool qv, int g, int bx, double pacc) {
  pacc += __shfl_xor(pacc, 16, 64);
  pacc += __shfl_xor(pacc, 32, 64);
  if (g == 0 && qv) a.pipart[q * a.nbx + bx] = pacc;
}

// The window is a ring of S = NB + PF slots: the block for window position p sits in
// slot p % S and is loaded PF iterations before its first use, so PF loads per wave are
// in flight behind the MFMAs.  The loop body is unrolled over S iterations, which
// makes every slot index a constant; loads are unconditional (clamped address, zero
// outside the signal) and only the MFMAs and the epilogue are skipped past the run.
template <int NB, int DIR>
__global__ __launch_bounds__(256) void k_conv_f32(ConvArgs a) {
  constexpr int PF = 3, S = NB + PF;
  if (a.done && *a.done) return;
  const int wid = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wid >= a.nbx * a.nct) return;
  const int bx = wid / a.nct, ct = wid - bx * a.nct;
  const int lane = threadIdx.x & 63, r16 = lane & 15, g = lane >> 4;
  const int64_t q = ct * 16 + r16;
  const bool qv = q < a.Q;
  const int64_t qld = qv ? q : 0;  // idle columns read column 0 (no extra lines) and use zeros
  const int64_t nblk = a.Dp >> 4;
  const int64_t a0 = (int64_t)bx * (VCHUNK / 16);
  const int cnt = (int)std::min<int64_t>(VCHUNK / 16, nblk - a0);

  // Toeplitz blocks in the operand layout of MFMA e: lane (r16, g) holds T[r16][4 g + e].
  f32x4 A[NB];
#pragma unroll
  for (int d = 0; d < NB; ++d)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int m = DIR == 0 ? 16 * d + r16 - 4 * g - e : 16 * d + 4 * g + e - r16;
      A[d][e] = a.hp32[CONV_HOFF + m];
    }

  const float* src = a.in32 + qld * a.Dp + 4 * g;
  const float* pdp = a.Pd ? a.Pd + qld * a.Dp : nullptr;
  const int64_t base = DIR == 0 ? a0 - (NB - 1) : a0;  // input block of window position 0
  auto load = [&](int64_t b) -> f32x4 {
    const bool ok = qv && b >= 0 && b < nblk;
    f32x4 v = *reinterpret_cast<const f32x4*>(src + 16 * (ok ? b : 0));
    return ok ? v : f32x4{0.f, 0.f, 0.f, 0.f};
  };
  // epilogue operands of output block a0 + i (clamped row; only used while i < cnt)
  auto row_of = [&](int i) -> int64_t { return (a0 + std::min(i, cnt - 1)) * 16 + 4 * g; };

  f32x4 win[S];
#pragma unroll
  for (int p = 0; p < S - 1; ++p) win[p] = load(base + p);
  f32x4 aln{0.f, 0.f, 0.f, 0.f}, pdn{0.f, 0.f, 0.f, 0.f};
  if (DIR == 1) {
    aln = *reinterpret_cast<const f32x4*>(a.alpha + row_of(0));
    pdn = *reinterpret_cast<const f32x4*>(pdp + row_of(0));
  }
  double pacc = 0.0;
  for (int i0 = 0; i0 < cnt; i0 += S) {
#pragma unroll
    for (int u = 0; u < S; ++u) {
      const int i = i0 + u;
      win[(u + S - 1) % S] = load(base + i + S - 1);
      const f32x4 al = aln, pd = pdn;
      if (DIR == 1) {
        aln = *reinterpret_cast<const f32x4*>(a.alpha + row_of(i + 1));
        pdn = *reinterpret_cast<const f32x4*>(pdp + row_of(i + 1));
      }
      __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the MFMAs
      if (i < cnt) {
        f32x4 acc[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int d = 0; d < NB; ++d) {
          const f32x4 bv = win[DIR == 0 ? (u + NB - 1 - d) % S : (u + d) % S];
#pragma unroll
          for (int e = 0; e < 4; ++e)
            acc[d & 3] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[d][e], bv[e], acc[d & 3], 0, 0, 0);
        }
        const f32x4 v = (acc[0] + acc[1]) + (acc[2] + acc[3]);
        conv_epilogue(a, DIR, q, qv, (a0 + i) * 16 + 4 * g, v, al, pd, pacc);
      }
    }
  }
  if (DIR == 1) conv_pi_store(a, q, qv, g, bx, pacc);
}

// ---------------------------------------------------------------------------
// The whole bf16 operator application in one pass: Psi = beta Phi^T (Phi Pd) + alpha Pd
// and the pi partials, with V = Phi Pd kept in registers instead of going through HBM.
// A wave owns one column tile and one run of output blocks [m0, m0 + cnt) as in the
// two-pass form.  Step k computes V block m0 + k by the causal filter (from Pd blocks
// m0 + k - NB + 1 .. m0 + k, a window of S slots loaded PF steps ahead) and pushes it,
// as its hi/lo bf16 pair in the MFMA operand layout, into a ring of S slots; from step
// NB - 1 on it also computes the anti-causal output block m0 + k - NB + 1 from the NB
// newest V blocks and runs the epilogue.  The run thus computes NB - 1 V blocks past
// its end (the halo the anti-causal filter reads), which the two-pass form read back
// from HBM.  The arithmetic is that of the two passes step for step (the same MFMAs in
// the same order, V rounded to the same pair, rows >= D zeroed), so Psi and pi are
// bitwise the same.  The causal filter's output leaves the MFMA with lane (c, g)
// holding rows 16 par + 4 g .. + 3 of column c; the anti-causal filter takes lane
// (c, g) = rows 8 g .. 8 g + 7, so each V block is regrouped across lanes (16 lane
// shuffles) before it is split.  The epilogue's Pd block is the oldest block of the
// causal filter's window at that step, so it is regrouped from there the other way
// instead of read again.  The Toeplitz blocks of both filters (36 KB) sit in LDS.
template <int NB>
__global__ __launch_bounds__(256, 2) void k_conv_bf16_op(ConvArgs a) {
  constexpr int PF = 2, S = NB + PF;
  if (a.xclear && blockIdx.x == 0 && threadIdx.x == 0) *a.xclear = 0;  // a new CG step
  if (a.done && *a.done) return;
  __shared__ bf16x8_t sT[2][2][NB][64];  // [filter][par][d][lane]: causal, anti-causal
  for (int f = threadIdx.x; f < 4 * NB * 64; f += blockDim.x) {
    const int l = f & 63, blk = f >> 6;
    const int d = blk % NB, par = (blk / NB) & 1, dir = blk / (2 * NB);
    const int r16 = l & 15, g = l >> 4;
    u16x8 t;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int m = dir == 0 ? 32 * d + 16 * par + r16 - 8 * g - j : 32 * d + 8 * g + j - 16 * par - r16;
      t[j] = a.hp16[CONV_HOFF + m];
    }
    sT[dir][par][d][l] = __builtin_bit_cast(bf16x8_t, t);
  }
  __syncthreads();
  const int wid = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wid >= a.nbx * a.nct) return;
  const int bx = wid / a.nct, ct = wid - bx * a.nct;
  const int lane = threadIdx.x & 63, r16 = lane & 15, g = lane >> 4;
  const int64_t q = ct * 16 + r16;
  const bool qv = q < a.Q;
  const int64_t nb32 = a.Dp >> 5;
  const int64_t m0 = (int64_t)bx * (VCHUNK / 32);
  const int cnt = (int)std::min<int64_t>(VCHUNK / 32, nb32 - m0);
  const int steps = cnt + NB - 1;

  // Pd pair in the tile-interleaved layout of sig_index: block b of this tile is 32 w
  // contiguous elements for the tile's w real columns, lane (r16, g) at 32 r16 + 8 g;
  // padding-column lanes load column 16 ct's segment and use zeros
  const int64_t qs = qv ? q : (int64_t)ct * 16;
  const int64_t bstride = 32 * sig_tile_width(qs, a.Q);
  const uint16_t* sh = a.inH + sig_index(qs, 8 * g, a.Dp, a.Q);
  const uint16_t* sl = a.inL + sig_index(qs, 8 * g, a.Dp, a.Q);
  const int64_t base = m0 - (NB - 1);  // Pd block of window position 0
  const bf16x8_t zero = __builtin_bit_cast(bf16x8_t, u16x8{0, 0, 0, 0, 0, 0, 0, 0});
  auto load = [&](const uint16_t* s, int64_t p) -> bf16x8_t {
    const int64_t b = base + p;
    const bool inb = b >= 0 && b < nb32;
    const bf16x8_t v = *reinterpret_cast<const bf16x8_t*>(s + bstride * (inb ? b : 0));
    return (qv && inb) ? v : zero;
  };
  // alpha at the rows of anti-causal output block i of the run (clamped to the run)
  auto clampi = [&](int i) -> int { return i < 0 ? 0 : (i < cnt ? i : cnt - 1); };
  auto rowp_of = [&](int i) -> int64_t { return (m0 + clampi(i)) * 32 + 4 * g; };
  // regrouping of a V block: lane (c, g) takes rows 8 g .. 8 g + 7, i.e. rows 16 par' + 8 h'
  // + j with par' = g >> 1, h' = g & 1, from lanes (c, 2 h') (j < 4) and (c, 2 h' + 1)
  const int src0 = r16 + 16 * (2 * (g & 1)), src1 = src0 + 16;
  const bool hi_par = (g >> 1) != 0;
  // the epilogue's Pd: the anti-causal output block of step k is window position k, so it
  // comes from the window (the value hi + lo the filters used) regrouped the other way:
  // lane (c, g) takes rows 16 par + 4 g + e from lane (c, 2 par + (g >> 1)), element
  // 4 (g & 1) + e
  const int pdsrc = r16 + 16 * (g >> 1);
  const bool pd_hi = (g & 1) != 0;

  bf16x8_t wh[S], wl[S], vh[S], vl[S];
#pragma unroll
  for (int p = 0; p < S - 1; ++p) {
    wh[p] = load(sh, p);
    wl[p] = load(sl, p);
  }
#pragma unroll
  for (int p = 0; p < S; ++p) vh[p] = vl[p] = zero;
  f32x4 aln[2];
#pragma unroll
  for (int par = 0; par < 2; ++par) aln[par] = *reinterpret_cast<const f32x4*>(a.alpha + rowp_of(1 - NB) + 16 * par);
  double pacc = 0.0;
  for (int k0 = 0; k0 < steps; k0 += S) {
#pragma unroll
    for (int u = 0; u < S; ++u) {
      const int k = k0 + u;
      wh[(u + S - 1) % S] = load(sh, k + S - 1);
      wl[(u + S - 1) % S] = load(sl, k + S - 1);
      const int i = k - (NB - 1);  // anti-causal output block of this step
      f32x4 al[2];
#pragma unroll
      for (int par = 0; par < 2; ++par) {
        al[par] = aln[par];
        aln[par] = *reinterpret_cast<const f32x4*>(a.alpha + rowp_of(i + 1) + 16 * par);
      }
      __builtin_amdgcn_sched_barrier(0);
      if (k < steps) {
        // causal: V block m0 + k
        f32x4 acc[2];
#pragma unroll
        for (int par = 0; par < 2; ++par) acc[par] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int d = 0; d < NB; ++d) {
          const int w = (u + NB - 1 - d) % S;
#pragma unroll
          for (int par = 0; par < 2; ++par) {
            const bf16x8_t t = sT[0][par][d][lane];
            acc[par] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(t, wh[w], acc[par], 0, 0, 0);
            acc[par] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(t, wl[w], acc[par], 0, 0, 0);
          }
        }
        const int64_t vrow = (m0 + k) * 32 + 4 * g;
#pragma unroll
        for (int par = 0; par < 2; ++par)
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (vrow + 16 * par + e >= a.D) acc[par][e] = 0.0f;
        u16x8 hh, ll;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float x0 = __shfl(acc[0][e], src0, 64), x1 = __shfl(acc[1][e], src0, 64);
          const float y0 = __shfl(acc[0][e], src1, 64), y1 = __shfl(acc[1][e], src1, 64);
          uint16_t h, l;
          split_bf16(hi_par ? x1 : x0, h, l);
          hh[e] = h;
          ll[e] = l;
          split_bf16(hi_par ? y1 : y0, h, l);
          hh[4 + e] = h;
          ll[4 + e] = l;
        }
        vh[u] = __builtin_bit_cast(bf16x8_t, hh);
        vl[u] = __builtin_bit_cast(bf16x8_t, ll);
        if (i >= 0 && i < cnt) {
          // anti-causal: output block m0 + i from V blocks m0 + i .. m0 + i + NB - 1
          f32x4 acc2[2];
#pragma unroll
          for (int par = 0; par < 2; ++par) acc2[par] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int d = 0; d < NB; ++d) {
            const int w = (u + S - (NB - 1) + d) % S;
#pragma unroll
            for (int par = 0; par < 2; ++par) {
              const bf16x8_t t = sT[1][par][d][lane];
              acc2[par] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(t, vh[w], acc2[par], 0, 0, 0);
              acc2[par] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(t, vl[w], acc2[par], 0, 0, 0);
            }
          }
          float x[8];
          {
            const u16x8 ph = __builtin_bit_cast(u16x8, wh[u]), pl = __builtin_bit_cast(u16x8, wl[u]);
#pragma unroll
            for (int j = 0; j < 8; ++j) x[j] = bf16_val(ph[j]) + bf16_val(pl[j]);
          }
          const int64_t rowp = (m0 + i) * 32 + 4 * g;
#pragma unroll
          for (int par = 0; par < 2; ++par) {
            f32x4 pd;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const float lo = __shfl(x[e], pdsrc + 32 * par, 64), hi = __shfl(x[4 + e], pdsrc + 32 * par, 64);
              pd[e] = pd_hi ? hi : lo;
            }
            conv_epilogue(a, 1, q, qv, rowp + 16 * par, acc2[par], al[par], pd, pacc);
          }
        }
      }
    }
  }
  conv_pi_store(a, q, qv, g, bx, pacc);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned cdiv_(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

int conv_blocks_f32(int L) { return (L + 14) / 16 + 1; }
int conv_blocks_bf16(int L) { return (L + 30) / 32 + 1; }

void launch_conv_taps(const float* h, int L, float* hp32, uint16_t* hp16, hipStream_t s) {
  hipLaunchKernelGGL(k_conv_taps, dim3(1), dim3(256), 0, s, h, L, hp32, hp16);
}

void launch_conv_setup(const float* h, int L, int64_t D, int64_t Dp, int jacobi, float* hp32, uint16_t* hp16,
                       float* theta, hipStream_t s) {
  launch_conv_taps(h, L, hp32, hp16, s);
  hipLaunchKernelGGL(k_conv_theta, dim3(cdiv_(Dp, 256)), dim3(256), 0, s, (const float*)hp32, L, D, Dp, jacobi,
                     theta);
}

void launch_conv_rhs(const float* hp32, const uint16_t* hp16, int L, int64_t D, int64_t Dp, const float* y,
                     double beta, float* b, hipStream_t s) {
  hipLaunchKernelGGL(k_conv_rhs, dim3(cdiv_(Dp, 256)), dim3(256), 0, s, hp32, hp16, L, D, Dp, y, beta, b);
}

template <int DIR>
static void conv_f32_dir(const ConvArgs& a, int nb, dim3 grid, hipStream_t s) {
  if (nb <= 5) hipLaunchKernelGGL((k_conv_f32<5, DIR>), grid, dim3(256), 0, s, a);
  else if (nb <= 9) hipLaunchKernelGGL((k_conv_f32<9, DIR>), grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL((k_conv_f32<17, DIR>), grid, dim3(256), 0, s, a);
}

void launch_conv_op_bf16(const ConvArgs& a, hipStream_t s) {
  const dim3 grid(cdiv_((int64_t)a.nbx * a.nct, 4));
  const int nb = conv_blocks_bf16(a.L);
  if (nb <= 3) hipLaunchKernelGGL((k_conv_bf16_op<3>), grid, dim3(256), 0, s, a);
  else if (nb <= 5) hipLaunchKernelGGL((k_conv_bf16_op<5>), grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL((k_conv_bf16_op<9>), grid, dim3(256), 0, s, a);
}

void launch_conv_pass(const ConvArgs& a, int dir, hipStream_t s) {
  const dim3 grid(cdiv_((int64_t)a.nbx * a.nct, 4));
  const int nb = conv_blocks_f32(a.L);
  if (dir == 0) conv_f32_dir<0>(a, nb, grid, s);
  else conv_f32_dir<1>(a, nb, grid, s);
}

}  // namespace cofem
