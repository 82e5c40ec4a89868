// The subsampled DCT dictionary of Sec. V-A.2 on gfx950: Phi = M Omega^{-1}, where
// Omega is the orthonormal DCT-II of size D (Omega^{-1} = Omega^T, the DCT-III) and
// M keeps N of the D samples.  The operator of Algorithm 2 is then
//
//   Psi = beta Omega diag(m) Omega^T Pd + alpha Pd,   m_n = 1 for kept samples n,
//
// two fast transforms and a mask per right-hand side, O(D log D) work
// (Sec. III-B: applying a structured Phi costs tau_D = O(D log D)).
//
// Two forms of the operator: for D = 2^11, 2^13 and 2^15 a column is
// split over several workgroups with a four-step FFT and three launches (see the
// split operator below); for every other size one workgroup owns one right-hand side
// and keeps the whole transform chain in LDS, so a column makes one trip through HBM
// per operator application (read Pd and alpha, write Psi).  Both transforms go
// through one complex FFT of length L = D / 2 (D a power of two, 16 <= D <= 2^15,
// so the L complex FP32 points take at most 128 KB of the 160 KB of LDS):
//
// * DCT-II via a real DFT of length D (Makhoul, "A fast cosine transform in one
//   and two dimensions", IEEE TASSP 1980): reorder v_n = x_2n, v_{D-1-n} = x_{2n+1};
//   then C_k = Re(e^{-i pi k / 2D} V_k) and C_{D-k} = -Im(e^{-i pi k / 2D} V_k),
//   where V = DFT_D(v).  The real DFT of length D is a complex DFT of length L of
//   z_m = v_2m + i v_{2m+1} followed by the usual even/odd split.
// * DCT-III (the inverse) runs the same steps backwards: from the coefficients
//   build the half-length Hermitian-split spectrum, take an inverse complex DFT of
//   length L (a forward one on conjugates), and read v off the real and imaginary
//   parts.  The mask is applied in the reordered domain, where both transforms
//   meet, so x itself is never formed.
//
// The complex DFT is a Stockham autosort FFT in place in LDS (radix-16 passes, one
// radix-2, 4 or 8 pass for the rest): each pass loads its butterflies into
// registers, applies the twiddles and the butterfly there, waits at a barrier and
// stores; a slot of padding per 16 points keeps the strided stores free of bank
// conflicts.  Twiddles, the DCT phase factors and the mask come from small tables
// built once in FP64 and rounded to FP32.
#include <algorithm>

#include "kernels.h"
#include "device_common.h"

namespace cofem {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 ctimes_i(float2 a) { return make_float2(-a.y, a.x); }       // i a
__device__ __forceinline__ float2 ctimes_minus_i(float2 a) { return make_float2(a.y, -a.x); }  // -i a

// Workgroup barrier that orders LDS only: the waves' global loads (twiddles, the
// next values of Pd and alpha) stay in flight across it.  Every barrier in this
// file protects LDS data.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Threads per workgroup for L complex points: one radix-16 butterfly per thread
// up to 1024 threads, at least one wave.
constexpr int dct_threads(int log2L) {
  return ((1 << log2L) / 16 < 64) ? 64 : (((1 << log2L) / 16 > 1024) ? 1024 : (1 << log2L) / 16);
}

// LDS layout: complex point i lives at float2 slot i + i / 16.  The Stockham passes
// write with strides of 16, 256, ... points; one slot of padding per 16 points
// turns each of them into a stride that hits every bank once per half-wave.
__device__ __forceinline__ int lds_slot(int i) { return i + (i >> 4); }
// The same buffer read as D real values: value f at float f + 2 (f / 32).
__device__ __forceinline__ int lds_real(int f) { return f + 2 * (f >> 5); }
constexpr int lds_slots(int L) { return L + L / 16; }

// Phase factors W_4D^m = e^{-2 pi i m / 4D} (m < 4D) from a two-level table kept in LDS:
// W^m = lo[m mod 2^LO] * hi[m >> LO], 2^LO + 2^HI entries for 4D = 2^(LO + HI).  The
// DCT factors are e^{-i pi k / 2D} = W_4D^k and e^{-2 pi i k / D} = W_4D^{4k}.
constexpr int wt_lo(int log2L) { return (log2L + 3 + 1) / 2; }
constexpr int wt_hi(int log2L) { return log2L + 3 - wt_lo(log2L); }
constexpr int wt_size(int log2L) { return (1 << wt_lo(log2L)) + (1 << wt_hi(log2L)); }
template <int LOG2L>
__device__ __forceinline__ float2 w4d(const float2* wt, int m) {
  constexpr int LO = wt_lo(LOG2L);
  return cmul(wt[m & ((1 << LO) - 1)], wt[(1 << LO) + (m >> LO)]);
}
// Copy the table into LDS (callers place a barrier before its first use).
template <int LOG2L, int NT>
__device__ __forceinline__ void load_wt(float2* wt, const float2* __restrict__ w2) {
  for (int i = threadIdx.x; i < wt_size(LOG2L); i += NT) wt[i] = w2[i];
}

// In-register forward DFTs of 2, 4, 8 and 16 points, natural order in and out.
__device__ __forceinline__ void dft2(float2* v) {
  const float2 a = v[0];
  v[0] = cadd(a, v[1]);
  v[1] = csub(a, v[1]);
}
__device__ __forceinline__ void dft4(float2* v) {
  const float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
  const float2 t2 = cadd(v[1], v[3]), t3 = ctimes_minus_i(csub(v[1], v[3]));
  v[0] = cadd(t0, t2);
  v[1] = cadd(t1, t3);
  v[2] = csub(t0, t2);
  v[3] = csub(t1, t3);
}
// W_16^m = e^{-2 pi i m / 16} = (cos(2 pi m / 16), -sin(2 pi m / 16)); m is a
// compile-time constant wherever this is called.
__device__ __forceinline__ float2 w16(int m) {
  constexpr float C1 = 0.92387953251128674f, C2 = 0.70710678118654752f, C3 = 0.38268343236508977f;
  constexpr float cs[16] = {1.0f, C1, C2, C3, 0.0f, -C3, -C2, -C1, -1.0f, -C1, -C2, -C3, 0.0f, C3, C2, C1};
  constexpr float sn[16] = {0.0f, C3, C2, C1, 1.0f, C1, C2, C3, 0.0f, -C3, -C2, -C1, -1.0f, -C1, -C2, -C3};
  return make_float2(cs[m & 15], -sn[m & 15]);
}
// 8 points as 2 x 4: n = 2 n1 + n2, k = k1 + 4 k2.
__device__ __forceinline__ void dft8(float2* v) {
  float2 e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
  dft4(e);
  dft4(o);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    const float2 t = cmul(o[k1], w16(2 * k1));
    v[k1] = cadd(e[k1], t);
    v[k1 + 4] = csub(e[k1], t);
  }
}
// 16 points as 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2.
__device__ __forceinline__ void dft16(float2* v) {
  float2 y[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) y[n2][n1] = v[4 * n1 + n2];
    dft4(y[n2]);
  }
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 z[4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) z[n2] = (n2 * k1 == 0) ? y[n2][k1] : cmul(y[n2][k1], w16(n2 * k1));
    dft4(z);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = z[k2];
  }
}
template <int R>
__device__ __forceinline__ void dft(float2* v) {
  if constexpr (R == 2) dft2(v);
  if constexpr (R == 4) dft4(v);
  if constexpr (R == 8) dft8(v);
  if constexpr (R == 16) dft16(v);
}

// One radix-R Stockham pass over L points with NT threads; ns = size of the
// sub-transforms already done.  Butterfly j reads points j + r L/R, multiplies
// point r by W_{R ns}^{k r} (k = j mod ns), takes their R-point DFT and, after a
// barrier (every butterfly has read its inputs), writes output r to point
// (j - k) R + k + r ns.  MASK: the pass reads the conjugated output of an inverse
// transform and applies the sample mask to it (see the operator kernel).
template <int L, int NT, int R, bool MASK>
__device__ __forceinline__ void fft_pass(float2* buf, const float2* __restrict__ tw, int ns,
                                         const float2* __restrict__ mz) {
  constexpr int NB = L / R;
  constexpr int BPT = (NB + NT - 1) / NT;
  float2 v[BPT][R];
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int j = threadIdx.x + b * NT;
    if (j < NB) {
      // W_{R ns}^{k r} = W_L^{r st}: powers 1, 2, 4, 8 from the table (loads issued
      // first), the others as products of at most four of them
      const int st = (j & (ns - 1)) * (NB / ns);
      float2 w[4];
      if (ns > 1) {
#pragma unroll
        for (int e = 0; (1 << e) < R; ++e) w[e] = tw[(1 << e) * st];
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        float2 x = buf[lds_slot(j + r * NB)];
        if (MASK) {
          const float2 m = mz[j + r * NB];
          x = make_float2(m.x * x.x, -m.y * x.y);
        }
        v[b][r] = x;
      }
      if (ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 f = make_float2(1.0f, 0.0f);
          bool first = true;
#pragma unroll
          for (int e = 0; (1 << e) < R; ++e)
            if (r & (1 << e)) {
              f = first ? w[e] : cmul(f, w[e]);
              first = false;
            }
          v[b][r] = cmul(v[b][r], f);
        }
      }
      dft<R>(v[b]);
    }
  }
  lds_barrier();
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int j = threadIdx.x + b * NT;
    if (j < NB) {
      const int k = j & (ns - 1);
      const int o = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[lds_slot(o + r * ns)] = v[b][r];
    }
  }
  lds_barrier();
}

// Forward DFT of the L points in buf (natural order in and out): radix-16 passes,
// then one radix-2, 4 or 8 pass for the rest of log2 L.  Callers place a barrier
// between their last write to buf and this call.
template <int LOG2L, bool MASK_FIRST>
__device__ __forceinline__ void fft_forward(float2* buf, const float2* __restrict__ tw,
                                            const float2* __restrict__ mz) {
  constexpr int L = 1 << LOG2L, NT = dct_threads(LOG2L);
  constexpr int P16 = LOG2L / 4, REM = LOG2L % 4;
  if constexpr (P16 > 0) {
    fft_pass<L, NT, 16, MASK_FIRST>(buf, tw, 1, mz);
    int ns = 16;
#pragma unroll
    for (int p = 1; p < P16; ++p, ns *= 16) fft_pass<L, NT, 16, false>(buf, tw, ns, mz);
    if constexpr (REM != 0) fft_pass<L, NT, (1 << REM), false>(buf, tw, ns, mz);
  } else {
    fft_pass<L, NT, (1 << REM), MASK_FIRST>(buf, tw, 1, mz);
  }
}

// V(k) = (Za + conj Zb) / 2 - i wh_k (Za - conj Zb) / 2: bin k of the real DFT of
// length D from bins k and L - k of the half-length complex DFT.
__device__ __forceinline__ float2 real_split(float2 za, float2 zb, float2 whk) {
  const float2 e = cscale(cadd(za, cconj(zb)), 0.5f);
  const float2 d = cmul(whk, cscale(csub(za, cconj(zb)), 0.5f));
  return cadd(e, ctimes_minus_i(d));
}

// After fft_forward: the DCT-II of the reordered signal, C_k = sum_n x_n
// cos(pi (2n + 1) k / 2D) (unnormalised), written over buf as D real values.
template <int LOG2L>
__device__ __forceinline__ void dct_post(float2* buf, const float2* wt) {
  constexpr int L = 1 << LOG2L, NT = dct_threads(LOG2L);
  constexpr int IT = (L / 2 + 1 + NT - 1) / NT;
  const int D = 2 * L;
  float2 A[IT], B[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int t = threadIdx.x + i * NT;
    if (t <= L / 2) {
      A[i] = buf[lds_slot(t)];
      B[i] = buf[lds_slot((L - t) & (L - 1))];
    }
  }
  lds_barrier();
  float* cb = reinterpret_cast<float*>(buf);
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int t = threadIdx.x + i * NT;
    if (t <= L / 2) {
      float2 w = cmul(w4d<LOG2L>(wt, t), real_split(A[i], B[i], w4d<LOG2L>(wt, 4 * t)));
      cb[lds_real(t)] = w.x;
      if (t > 0) cb[lds_real(D - t)] = -w.y;
      if (t == 0) {
        w = cmul(w4d<LOG2L>(wt, L), real_split(A[i], A[i], w4d<LOG2L>(wt, 4 * L)));
        cb[lds_real(L)] = w.x;
      } else if (t < L / 2) {
        w = cmul(w4d<LOG2L>(wt, L - t), real_split(B[i], A[i], w4d<LOG2L>(wt, 4 * (L - t))));
        cb[lds_real(L - t)] = w.x;
        cb[lds_real(L + t)] = -w.y;
      }
    }
  }
  lds_barrier();
}

// Operator over one column per workgroup: Psi = beta Omega diag(m) Omega^T Pd +
// alpha Pd, and the FP64 partials of pi_q = sum_j Pd_jq Psi_jq per 1024
// coordinates at pipart[q * nbx + chunk].
template <int LOG2L>
__global__ __launch_bounds__(dct_threads(LOG2L)) void k_dct_operator(DctArgs a) {
  constexpr int L = 1 << LOG2L, NT = dct_threads(LOG2L), NW = NT / 64;
  constexpr int D = 2 * L;
  constexpr int IT = (L / 2 + 1 + NT - 1) / NT;
  __shared__ __align__(16) float2 buf[lds_slots(L)];
  __shared__ double red[(D + 255) / 256 + 4];
  __shared__ float2 wt[wt_size(LOG2L)];
  if (a.done && *a.done) return;  // a step enqueued after the stop rule fired
  const int q = blockIdx.x;
  const float* __restrict__ p = a.in + (int64_t)q * a.Dp;
  load_wt<LOG2L, NT>(wt, a.w2);
  // Inverse transform, spectrum side.  With c_k = s_k Pd_k, the Hermitian
  // spectrum of the reordered output is H_0 = c_0, H_k = e^{i pi k / 2D} (c_k -
  // i c_{D-k}) / 2; its half-length form is Z_k = E_k + i O_k with E_k = H_k +
  // conj H_{L-k}, O_k = (H_k - conj H_{L-k}) e^{2 pi i k / D}.  buf gets conj Z,
  // so that a forward DFT yields the conjugate of the inverse one.  Item t makes
  // Z_t and Z_{L-t} from Pd at t, D - t, L - t and L + t (all loads issued first).
  auto hval = [&](int k, float pk, float pdk, float2 wqk) -> float2 {
    if (k == 0) return make_float2(a.s0 * pk, 0.0f);
    return cscale(cmul(cconj(wqk), make_float2(a.s1 * pk, -a.s1 * pdk)), 0.5f);
  };
  auto zval = [&](float2 h1, float2 h2, float2 whk) -> float2 {
    const float2 e = cadd(h1, cconj(h2));
    const float2 o = cmul(csub(h1, cconj(h2)), cconj(whk));
    return cadd(e, ctimes_i(o));
  };
  lds_barrier();  // the phase-factor table is in LDS
  constexpr int G1 = IT < 3 ? IT : 3;  // items whose loads are issued together
#pragma unroll 1
  for (int i0 = 0; i0 < IT; i0 += G1) {
    float c_t[G1], c_dt[G1], c_lt[G1], c_lpt[G1];
#pragma unroll
    for (int g = 0; g < G1; ++g) {
      const int t = threadIdx.x + (i0 + g) * NT;
      if (i0 + g < IT && t <= L / 2) {
        c_t[g] = p[t];
        c_dt[g] = t > 0 ? p[D - t] : 0.0f;
        c_lt[g] = p[L - t];
        c_lpt[g] = p[L + t];
      }
    }
#pragma unroll
    for (int g = 0; g < G1; ++g) {
      const int t = threadIdx.x + (i0 + g) * NT;
      if (i0 + g < IT && t <= L / 2) {
        const float2 h1 = hval(t, c_t[g], c_dt[g], w4d<LOG2L>(wt, t));
        const float2 h2 = hval(L - t, c_lt[g], c_lpt[g], w4d<LOG2L>(wt, L - t));
        buf[lds_slot(t)] = cconj(zval(h1, h2, w4d<LOG2L>(wt, 4 * t)));
        if (t > 0 && t < L / 2) buf[lds_slot(L - t)] = cconj(zval(h2, h1, w4d<LOG2L>(wt, 4 * (L - t))));
      }
    }
  }
  lds_barrier();
  fft_forward<LOG2L, false>(buf, a.tw, a.mz);
  // buf = conj(z), z_m = v_2m + i v_{2m+1} the reordered Omega^T Pd.  The next
  // transform's first pass reads z' = (m_2m v_2m, m_{2m+1} v_{2m+1}).
  fft_forward<LOG2L, true>(buf, a.tw, a.mz);
  dct_post<LOG2L>(buf, wt);
  // Psi = beta s_k C_k + alpha_k Pd_k, 4 coordinates per thread and iteration; the
  // pi partial of each run of 256 coordinates is one wave's sum, and chunk c of
  // 1024 coordinates adds runs 4c .. 4c + 3 in order.
  const float* __restrict__ cb = reinterpret_cast<const float*>(buf);
  float* __restrict__ out = a.out + (int64_t)q * a.Dp;
  constexpr int IT2 = (D + 4 * NT - 1) / (4 * NT);
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  constexpr int G = IT2 < 4 ? IT2 : 4;  // iterations whose loads are issued together
#pragma unroll 1
  for (int i0 = 0; i0 < IT2; i0 += G) {
    f32x4 pv[G], al[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int j = 4 * (threadIdx.x + (i0 + g) * NT);
      if (i0 + g < IT2 && j < D) {
        pv[g] = *reinterpret_cast<const f32x4*>(p + j);
        al[g] = *reinterpret_cast<const f32x4*>(a.alpha + j);
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int i = i0 + g;
      if (i >= IT2) break;
      const int j = 4 * (threadIdx.x + i * NT);
      double acc = 0.0;
      if (j < D) {
        const float2 c01 = *reinterpret_cast<const float2*>(cb + lds_real(j));
        const float2 c23 = *reinterpret_cast<const float2*>(cb + lds_real(j + 2));
        const float cv[4] = {c01.x, c01.y, c23.x, c23.y};
        f32x4 ps;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float sk = (j + e == 0) ? a.s0 : a.s1;
          ps[e] = (float)(a.beta * (double)(sk * cv[e]) + (double)al[g][e] * (double)pv[g][e]);
          acc += (double)pv[g][e] * (double)ps[e];
        }
        *reinterpret_cast<f32x4*>(out + j) = ps;
      }
      if ((i * NT + 64 * wv) * 4 < D) {
        acc = wave_sum(acc);
        if (ln == 0) red[i * NW + wv] = acc;
      }
    }
  }
  // zero Psi on [D, Dp) (D < 256 only)
  for (int64_t j = D + threadIdx.x; j < a.Dp; j += NT) out[j] = 0.0f;
  lds_barrier();
  constexpr int RUNS = (D + 255) / 256;
  for (int c = threadIdx.x; c < a.nbx; c += NT) {
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (4 * c + r < RUNS) s += red[4 * c + r];
    a.pipart[(int64_t)q * a.nbx + c] = s;
  }
}

// out = beta Omega u for one signal u of D samples (the right-hand side b = beta
// Phi^T y once y is scattered to its samples); out is zero on [D, Dp).
template <int LOG2L>
__global__ __launch_bounds__(dct_threads(LOG2L)) void k_dct_forward(DctArgs a) {
  constexpr int L = 1 << LOG2L, NT = dct_threads(LOG2L);
  constexpr int D = 2 * L;
  constexpr int IT = (L + NT - 1) / NT;
  __shared__ __align__(16) float2 buf[lds_slots(L)];
  __shared__ float2 wt[wt_size(LOG2L)];
  const float* __restrict__ u = a.in;
  load_wt<LOG2L, NT>(wt, a.w2);
  // z_m = v_2m + i v_{2m+1} with v_n = u_2n (n < L), v_n = u_{2(D-1-n)+1} (n >= L)
  float2 z[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int m = threadIdx.x + i * NT;
    if (m < L)
      z[i] = (m < L / 2) ? make_float2(u[4 * m], u[4 * m + 2]) : make_float2(u[2 * D - 4 * m - 1], u[2 * D - 4 * m - 3]);
  }
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int m = threadIdx.x + i * NT;
    if (m < L) buf[lds_slot(m)] = z[i];
  }
  lds_barrier();
  fft_forward<LOG2L, false>(buf, a.tw, a.mz);
  dct_post<LOG2L>(buf, wt);
  const float* __restrict__ cb = reinterpret_cast<const float*>(buf);
  for (int64_t j = threadIdx.x; j < a.Dp; j += NT) {
    const float sk = (j == 0) ? a.s0 : a.s1;
    a.out[j] = (j < D) ? (float)(a.beta * (double)(sk * cb[lds_real((int)j)])) : 0.0f;
  }
}

// ---------------------------------------------------------------------------
// Split operator: one column over several workgroups, three launches
// ---------------------------------------------------------------------------
// For L = S^2 (log2 L even) the length-L DFT is a four-step one: with n = n1 + S n2
// and k = k2 + S k1,
//   Y[n1][k2] = W_L^{n1 k2} sum_{n2} x[n1 + S n2] W_S^{n2 k2},
//   X[k2 + S k1] = sum_{n1} Y[n1][k2] W_S^{n1 k1},
// two sets of S transforms of length S with an exchange through global memory (L2)
// in between.  The operator's two transforms chain as
//   launch 1: spectrum of Pd + first half of transform 1 (over n2, per residue n1),
//   launch 2: second half of transform 1 (over n1, per k2), the mask, and first half
//             of transform 2: the outputs of transform 1 with a fixed k2 mod S are
//             exactly the inputs of transform 2 with n1 = k2, so no exchange is needed,
//   launch 3: second half of transform 2, the DCT post-processing and the epilogue.
// Each workgroup owns SP_RC residues mod S, chosen closed under r -> -r mod S (the
// post-processing pairs bins k and L - k, and L - k = -k mod S): rows i < 8 are
// residues 8g + i, rows 8 + i their negatives (S / 2 in place of S - 0).  Each
// length-S transform is S = 16 R2 points: a 16-point DFT in registers per (row, a)
// over n = a + R2 b, the twiddles W_S^{ac}, an LDS exchange, and an R2-point DFT per
// (row, c), giving bin k = c + 16 d in register d.  A column becomes G = S / SP_RC
// workgroups, so the 21 or 33 columns of a step fill the chip instead of 21 or 33 CUs.
constexpr int SP_RC = 16;           // residues (rows) per workgroup
constexpr int SP_NT = SP_RC * 16;   // threads per workgroup
constexpr bool dct_split_log2(int log2L) { return log2L == 10 || log2L == 12 || log2L == 14; }

template <int LOG2L>
struct SplitShape {
  static constexpr int L = 1 << LOG2L, D = 2 * L, S = 1 << (LOG2L / 2), R2 = S / 16, G = S / SP_RC;
  static constexpr int CS = SP_RC * R2 + (SP_RC & 31);  // LDS stride per c in the (a, c) exchange
};

// Residue mod S of row `row` of workgroup g.
template <int S>
__device__ __forceinline__ int sp_residue(int g, int row) {
  const int i = row & 7;
  if (row < 8) return g * 8 + i;
  const int r = S - (g * 8 + i);
  return r == S ? S / 2 : r;
}
// The row holding residue -r mod S.
__device__ __forceinline__ int sp_partner_row(int g, int row) {
  if (g == 0 && (row & 7) == 0) return row;  // residues 0 and S / 2
  return row < 8 ? row + 8 : row - 8;
}
// Block -> (column, group): with the grid a multiple of 8, the G groups of a column
// run on one XCD (blocks are dealt to the 8 XCDs round-robin), so the column's
// exchange buffers and Pd stay in that XCD's L2 across the three launches.
__device__ __forceinline__ void sp_tile(int G, int& q, int& g) {
  const int b = blockIdx.x, n = gridDim.x;
  const int pos = (n & 7) == 0 ? (b & 7) * (n >> 3) + (b >> 3) : b;
  q = pos / G;
  g = pos % G;
}

// First half of a length-S transform: thread (row, a) holds x[a + R2 b] in v[b]; the
// 16-point DFT over b, the twiddles W_S^{ac}, and the exchange store.
template <int LOG2L>
__device__ __forceinline__ void sp_half1(float2 (&v)[16], int row, int a, float2* ex, const float2* twS) {
  using SS = SplitShape<LOG2L>;
  dft16(v);
#pragma unroll
  for (int c = 0; c < 16; ++c) ex[c * SS::CS + a * SP_RC + row] = (c == 0 || a == 0) ? v[c] : cmul(v[c], twS[a * c]);
}
// Second half: thread (row, c) takes the R2 values of its c and their R2-point DFT;
// y[d] is bin c + 16 d of the row's transform.
template <int LOG2L>
__device__ __forceinline__ void sp_half2(float2 (&y)[SplitShape<LOG2L>::R2], int row, int c, const float2* ex) {
  using SS = SplitShape<LOG2L>;
#pragma unroll
  for (int a = 0; a < SS::R2; ++a) y[a] = ex[c * SS::CS + a * SP_RC + row];
  dft<SS::R2>(y);
}
// Tables every split launch uses: the W_4D table and W_S^i = tw[S i].
template <int LOG2L>
__device__ __forceinline__ void sp_tables(float2* wt, float2* twS, const DctArgs& a) {
  using SS = SplitShape<LOG2L>;
  load_wt<LOG2L, SP_NT>(wt, a.w2);
  for (int i = threadIdx.x; i < SS::S; i += SP_NT) twS[i] = a.tw[i * SS::S];
}

// Launch 1: x[m] = conj Z_m (the spectrum side of the inverse transform, as in
// k_dct_operator) for m = r + S n2, the first half over n2, and
// y1[q][k2][r] = W_L^{r k2} (its result).  The spectrum is built by all threads into
// LDS: item m of rows 0..7 makes Z_m and, when its residue r is not 0, also
// Z_{L-m} (row 8 + i, n2' = S - 1 - n2) from the same four loads of Pd; in group 0,
// rows 0 and 8 (residues 0 and S / 2) pair within themselves, so row 8's points are
// items of their own there.
template <int LOG2L>
__global__ __launch_bounds__(SP_NT) void k_dct_split1(DctArgs a) {
  using SS = SplitShape<LOG2L>;
  constexpr int L = SS::L, D = SS::D, S = SS::S, R2 = SS::R2;
  constexpr int XS = S + 2;                 // LDS row stride of the spectrum
  constexpr int NI = 8 * S, IPT = NI / SP_NT;  // items of rows 0..7, per thread
  static_assert(NI % SP_NT == 0, "items per thread");
  __shared__ float2 wt[wt_size(LOG2L)];
  __shared__ float2 twS[S];
  __shared__ float2 ex[16 * SS::CS];
  __shared__ float2 xs[SP_RC * XS];
  int q, g;
  sp_tile(SS::G, q, g);
  const float* __restrict__ p = a.in + (int64_t)q * a.Dp;
  // item i < IPT: e = tid + i NT (row e % 8, n2 = e / 8); item IPT: group 0's row 8
  const bool extra = g == 0 && (int)threadIdx.x < S;
  float pm[IPT + 1], pdm[IPT + 1], plm[IPT + 1], plpm[IPT + 1];
  int mi[IPT + 1];
#pragma unroll
  for (int i = 0; i <= IPT; ++i) {
    const int e = threadIdx.x + i * SP_NT;
    const int m = i < IPT ? sp_residue<S>(g, e & 7) + S * (e >> 3) : S / 2 + S * (int)threadIdx.x;
    mi[i] = m;
    if (i < IPT || extra) {
      pm[i] = p[m];
      pdm[i] = m > 0 ? p[D - m] : 0.0f;
      plm[i] = p[L - m];
      plpm[i] = p[L + m];
    }
  }
  sp_tables<LOG2L>(wt, twS, a);
  if (a.done && *a.done) return;  // a step enqueued after the stop rule fired (tested once the loads are out)
  lds_barrier();
#pragma unroll
  for (int i = 0; i <= IPT; ++i) {
    if (i == IPT && !extra) break;
    const int e = threadIdx.x + i * SP_NT;
    const int m = mi[i], lm = L - m;
    const int row = i < IPT ? (e & 7) : 8, n2 = i < IPT ? (e >> 3) : (int)threadIdx.x;
    const float2 h1 = m == 0 ? make_float2(a.s0 * pm[i], 0.0f)
                             : cscale(cmul(cconj(w4d<LOG2L>(wt, m)), make_float2(a.s1 * pm[i], -a.s1 * pdm[i])), 0.5f);
    const float2 h2 = cscale(cmul(cconj(w4d<LOG2L>(wt, lm)), make_float2(a.s1 * plm[i], -a.s1 * plpm[i])), 0.5f);
    const float2 zm = cadd(cadd(h1, cconj(h2)), ctimes_i(cmul(csub(h1, cconj(h2)), cconj(w4d<LOG2L>(wt, 4 * m)))));
    xs[row * XS + n2] = cconj(zm);
    if (i < IPT && (m % S) != 0) {
      const float2 zl = cadd(cadd(h2, cconj(h1)), ctimes_i(cmul(csub(h2, cconj(h1)), cconj(w4d<LOG2L>(wt, 4 * lm)))));
      xs[(row + 8) * XS + (S - 1 - n2)] = cconj(zl);
    }
  }
  lds_barrier();
  const int row = threadIdx.x % SP_RC, grp = threadIdx.x / SP_RC;
  const int r = sp_residue<S>(g, row);
  if (grp < R2) {
    float2 v[16];
#pragma unroll
    for (int b = 0; b < 16; ++b) v[b] = xs[row * XS + grp + R2 * b];
    sp_half1<LOG2L>(v, row, grp, ex, twS);
  }
  lds_barrier();
  float2 y[R2];
  sp_half2<LOG2L>(y, row, grp, ex);
  float2* __restrict__ y1 = a.y1 + (int64_t)q * L;
#pragma unroll
  for (int d = 0; d < R2; ++d) {
    const int k2 = grp + 16 * d;
    y1[k2 * S + r] = cmul(y[d], w4d<LOG2L>(wt, 8 * r * k2));
  }
}

// Launch 2: row k2 = r of y1, the second half of transform 1 (bins r + S k1), the
// mask, then the first half of transform 2 over k1 (its n2) with n1 = r, and
// y2[q][k2'][r] = W_L^{r k2'} (its result).
template <int LOG2L>
__global__ __launch_bounds__(SP_NT) void k_dct_split2(DctArgs a) {
  using SS = SplitShape<LOG2L>;
  constexpr int L = SS::L, S = SS::S, R2 = SS::R2;
  __shared__ float2 wt[wt_size(LOG2L)];
  __shared__ float2 twS[S];
  __shared__ float2 ex[16 * SS::CS];
  __shared__ float2 ex2[S * SP_RC];
  int q, g;
  sp_tile(SS::G, q, g);
  const int row = threadIdx.x % SP_RC, grp = threadIdx.x / SP_RC;
  const int r = sp_residue<S>(g, row);
  const float2* __restrict__ y1 = a.y1 + (int64_t)q * L + (int64_t)r * S;
  float2 v[16];
  if (grp < R2) {
#pragma unroll
    for (int b = 0; b < 16; ++b) v[b] = y1[grp + R2 * b];
  }
  float2 m[R2];
#pragma unroll
  for (int d = 0; d < R2; ++d) m[d] = a.mzt[r * S + grp + 16 * d];
  sp_tables<LOG2L>(wt, twS, a);
  if (a.done && *a.done) return;
  lds_barrier();
  if (grp < R2) sp_half1<LOG2L>(v, row, grp, ex, twS);
  lds_barrier();
  float2 y[R2];
  sp_half2<LOG2L>(y, row, grp, ex);
  // bin k1 = grp + 16 d of transform 1 -> masked input n2 = k1 of transform 2
#pragma unroll
  for (int d = 0; d < R2; ++d)
    ex2[(grp + 16 * d) * SP_RC + row] = make_float2(m[d].x * y[d].x, -m[d].y * y[d].y);
  lds_barrier();
  if (grp < R2) {
#pragma unroll
    for (int b = 0; b < 16; ++b) v[b] = ex2[(grp + R2 * b) * SP_RC + row];
    sp_half1<LOG2L>(v, row, grp, ex, twS);
  }
  lds_barrier();
  sp_half2<LOG2L>(y, row, grp, ex);
  float2* __restrict__ y2 = a.y2 + (int64_t)q * L;
#pragma unroll
  for (int d = 0; d < R2; ++d) {
    const int k2 = grp + 16 * d;
    y2[k2 * S + r] = cmul(y[d], w4d<LOG2L>(wt, 8 * r * k2));
  }
}

// Launch 3: row k2' = r of y2, the second half of transform 2 (bins X_k, k = r + S k1),
// then per bin the DCT post-processing with its partner bin L - k (row of -r, held
// by this workgroup): C_k and C_{D-k} (and C_L from bin 0), and the epilogue
// Psi_j = beta s_j C_j + alpha_j Pd_j.  The workgroup's pi partial (FP64, fixed order)
// goes to pipart[q * nbx + g]; the column's slots G .. nbx - 1 are zeroed.
template <int LOG2L>
__global__ __launch_bounds__(SP_NT) void k_dct_split3(DctArgs a) {
  using SS = SplitShape<LOG2L>;
  constexpr int L = SS::L, D = SS::D, S = SS::S, R2 = SS::R2, G = SS::G;
  __shared__ float2 wt[wt_size(LOG2L)];
  __shared__ float2 twS[S];
  __shared__ float2 ex[16 * SS::CS];
  __shared__ float2 ex2[S * SP_RC];
  __shared__ double red[SP_NT / 64];
  int q, g;
  sp_tile(G, q, g);
  const int row = threadIdx.x % SP_RC, grp = threadIdx.x / SP_RC;
  const int r = sp_residue<S>(g, row);
  const float2* __restrict__ y2 = a.y2 + (int64_t)q * L + (int64_t)r * S;
  const float* __restrict__ p = a.in + (int64_t)q * a.Dp;
  float2 v[16];
  if (grp < R2) {
#pragma unroll
    for (int b = 0; b < 16; ++b) v[b] = y2[grp + R2 * b];
  }
  // Pd and alpha at the outputs k and D - k of this thread's bins
  float pk[R2], ak[R2], pdk[R2], adk[R2];
#pragma unroll
  for (int d = 0; d < R2; ++d) {
    const int k = r + S * (grp + 16 * d);
    const int j = k > 0 ? D - k : L;
    pk[d] = p[k];
    ak[d] = a.alpha[k];
    pdk[d] = p[j];
    adk[d] = a.alpha[j];
  }
  sp_tables<LOG2L>(wt, twS, a);
  if (a.done && *a.done) return;
  lds_barrier();
  if (grp < R2) sp_half1<LOG2L>(v, row, grp, ex, twS);
  lds_barrier();
  float2 y[R2];
  sp_half2<LOG2L>(y, row, grp, ex);
#pragma unroll
  for (int d = 0; d < R2; ++d) ex2[(grp + 16 * d) * SP_RC + row] = y[d];
  lds_barrier();
  const int prow = sp_partner_row(g, row);
  float* __restrict__ out = a.out + (int64_t)q * a.Dp;
  double acc = 0.0;
#pragma unroll
  for (int d = 0; d < R2; ++d) {
    const int k1 = grp + 16 * d, k = r + S * k1;
    const int pk1 = r > 0 ? S - 1 - k1 : (S - k1) & (S - 1);
    const float2 B = ex2[pk1 * SP_RC + prow];
    const float2 w = cmul(w4d<LOG2L>(wt, k), real_split(y[d], B, w4d<LOG2L>(wt, 4 * k)));
    const float sk = k == 0 ? a.s0 : a.s1;
    const float psi_k = (float)(a.beta * (double)(sk * w.x) + (double)ak[d] * (double)pk[d]);
    out[k] = psi_k;
    acc += (double)pk[d] * (double)psi_k;
    // k > 0: C_{D-k} = -Im w;  k = 0: C_L from bin 0 paired with itself
    float cj;
    if (k > 0) {
      cj = -w.y;
    } else {
      cj = cmul(w4d<LOG2L>(wt, L), real_split(y[d], y[d], w4d<LOG2L>(wt, 4 * L))).x;
    }
    const int j = k > 0 ? D - k : L;
    const float psi_j = (float)(a.beta * (double)(a.s1 * cj) + (double)adk[d] * (double)pdk[d]);
    out[j] = psi_j;
    acc += (double)pdk[d] * (double)psi_j;
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  lds_barrier();
  if (threadIdx.x == 0) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < SP_NT / 64; ++w) s += red[w];
    a.pipart[(int64_t)q * a.nbx + g] = s;
  }
  if (g == 0)
    for (int c = G + (int)threadIdx.x; c < a.nbx; c += SP_NT) a.pipart[(int64_t)q * a.nbx + c] = 0.0;
}

// ---------------------------------------------------------------------------
// Set-up: tables, mask, theta, right-hand side
// ---------------------------------------------------------------------------
// tw_i = e^{-2 pi i i / L} (i < L) and the two-level table of W_4D = e^{-2 pi i / 4D}:
// w2[i] = W^i (i < 2^lo), w2[2^lo + i] = W^(i 2^lo) (i < 2^hi), from FP64 sincospi (the
// arguments are exact binary fractions).
__global__ void k_dct_tables(int L, int lo, int hi, float2* __restrict__ tw, float2* __restrict__ w2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const double D = 2.0 * L;
  double s, c;
  if (i < (1 << lo)) {
    sincospi(2.0 * i / (4.0 * D), &s, &c);
    w2[i] = make_float2((float)c, (float)-s);
  }
  if (i < (1 << hi)) {
    sincospi(2.0 * (double)i * (double)(1 << lo) / (4.0 * D), &s, &c);
    w2[(1 << lo) + i] = make_float2((float)c, (float)-s);
  }
  if (i < L) {
    sincospi(2.0 * i / L, &s, &c);
    tw[i] = make_float2((float)c, (float)-s);
  }
}

// mx[rows_i] = v_i (v = null: 1).  mx must be zero beforehand; rows are distinct.
__global__ void k_dct_scatter(const int32_t* __restrict__ rows, const float* __restrict__ v, int64_t N,
                              float* __restrict__ mx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) mx[rows[i]] = v ? v[i] : 1.0f;
}

// The mask in the order of the half-length transform: mz_m = (mv_2m, mv_{2m+1})
// with mv_n = mx_2n (n < L) and mv_n = mx_{2(D-1-n)+1} (n >= L).
// With mzt (S = sqrt L), also the transposed copy mzt[(m mod S) S + m / S] = mz_m.
__global__ void k_dct_mask(int L, int S, const float* __restrict__ mx, float2* __restrict__ mz,
                           float2* __restrict__ mzt) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= L) return;
  const int D = 2 * L;
  auto mv = [&](int n) { return n < L ? mx[2 * n] : mx[2 * (D - 1 - n) + 1]; };
  const float2 z = make_float2(mv(2 * m), mv(2 * m + 1));
  mz[m] = z;
  if (mzt) mzt[(m % S) * S + m / S] = z;
}

// Jacobi theta_j = sum_i Omega_{j, rows_i}^2 = s_j^2 sum_i cos^2(pi (2 rows_i + 1) j / 2D),
// in FP64 with the angle reduced exactly modulo 4D; theta = 1 on [D, Dp).
__global__ void k_dct_theta(const int32_t* __restrict__ rows, int64_t N, int64_t D, int64_t Dp,
                            float* __restrict__ theta) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= Dp) return;
  if (j >= D) {
    theta[j] = 1.0f;
    return;
  }
  double acc = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    const int64_t r = ((2 * (int64_t)rows[i] + 1) * j) % (4 * D);
    const double c = cospi((double)r / (2.0 * (double)D));
    acc += c * c;
  }
  theta[j] = (float)(acc * (j == 0 ? 1.0 / (double)D : 2.0 / (double)D));
}

namespace {

int log2_half(int64_t D) {
  int l = 0;
  while ((int64_t(2) << l) < D) ++l;
  return l;  // D = 2^(l + 1)
}

#define DCT_DISPATCH(KERNEL, GRID, ARGS, STREAM)                                                             \
  switch (log2_half(ARGS.D)) {                                                                               \
    case 3: hipLaunchKernelGGL(KERNEL<3>, dim3(GRID), dim3(dct_threads(3)), 0, STREAM, ARGS); break;         \
    case 4: hipLaunchKernelGGL(KERNEL<4>, dim3(GRID), dim3(dct_threads(4)), 0, STREAM, ARGS); break;         \
    case 5: hipLaunchKernelGGL(KERNEL<5>, dim3(GRID), dim3(dct_threads(5)), 0, STREAM, ARGS); break;         \
    case 6: hipLaunchKernelGGL(KERNEL<6>, dim3(GRID), dim3(dct_threads(6)), 0, STREAM, ARGS); break;         \
    case 7: hipLaunchKernelGGL(KERNEL<7>, dim3(GRID), dim3(dct_threads(7)), 0, STREAM, ARGS); break;         \
    case 8: hipLaunchKernelGGL(KERNEL<8>, dim3(GRID), dim3(dct_threads(8)), 0, STREAM, ARGS); break;         \
    case 9: hipLaunchKernelGGL(KERNEL<9>, dim3(GRID), dim3(dct_threads(9)), 0, STREAM, ARGS); break;         \
    case 10: hipLaunchKernelGGL(KERNEL<10>, dim3(GRID), dim3(dct_threads(10)), 0, STREAM, ARGS); break;      \
    case 11: hipLaunchKernelGGL(KERNEL<11>, dim3(GRID), dim3(dct_threads(11)), 0, STREAM, ARGS); break;      \
    case 12: hipLaunchKernelGGL(KERNEL<12>, dim3(GRID), dim3(dct_threads(12)), 0, STREAM, ARGS); break;      \
    case 13: hipLaunchKernelGGL(KERNEL<13>, dim3(GRID), dim3(dct_threads(13)), 0, STREAM, ARGS); break;      \
    case 14: hipLaunchKernelGGL(KERNEL<14>, dim3(GRID), dim3(dct_threads(14)), 0, STREAM, ARGS); break;      \
    default: break;                                                                                          \
  }

}  // namespace

bool dct_size_ok(int64_t D) { return D >= DCT_MIN_D && D <= DCT_MAX_D && (D & (D - 1)) == 0; }

bool dct_split_ok(int64_t D) { return dct_size_ok(D) && dct_split_log2(log2_half(D)); }

void launch_dct_setup(const int32_t* rows, int64_t N, int64_t D, int64_t Dp, int jacobi, float2* tw, float2* w2,
                      float2* mz, float2* mzt, float* mx, float* theta, hipStream_t s) {
  const int L = (int)(D / 2);
  const int lg = log2_half(D) + 3, lo = (lg + 1) / 2, hi = lg - lo;
  const int n = std::max(L, 1 << lo);
  hipLaunchKernelGGL(k_dct_tables, dim3((n + 255) / 256), dim3(256), 0, s, L, lo, hi, tw, w2);
  launch_fill(mx, 0.0f, Dp, s);
  hipLaunchKernelGGL(k_dct_scatter, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, rows,
                     static_cast<const float*>(nullptr), N, mx);
  const int S = dct_split_ok(D) ? 1 << (log2_half(D) / 2) : 1;
  hipLaunchKernelGGL(k_dct_mask, dim3((L + 255) / 256), dim3(256), 0, s, L, S, mx, mz, dct_split_ok(D) ? mzt : nullptr);
  if (jacobi)
    hipLaunchKernelGGL(k_dct_theta, dim3((unsigned)((Dp + 255) / 256)), dim3(256), 0, s, rows, N, D, Dp, theta);
  else
    launch_fill(theta, 1.0f, Dp, s);
}

void launch_dct_rhs(const DctArgs& a, const float* y, const int32_t* rows, int64_t N, float* u, hipStream_t s) {
  launch_fill(u, 0.0f, a.Dp, s);
  hipLaunchKernelGGL(k_dct_scatter, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, rows, y, N, u);
  DctArgs f = a;
  f.in = u;
  DCT_DISPATCH(k_dct_forward, 1, f, s);
}

template <int LOG2L>
void launch_split(const DctArgs& a, int Q, hipStream_t s) {
  const dim3 grid((unsigned)(Q * SplitShape<LOG2L>::G)), block(SP_NT);
  hipLaunchKernelGGL(k_dct_split1<LOG2L>, grid, block, 0, s, a);
  hipLaunchKernelGGL(k_dct_split2<LOG2L>, grid, block, 0, s, a);
  hipLaunchKernelGGL(k_dct_split3<LOG2L>, grid, block, 0, s, a);
}

void launch_dct_operator(const DctArgs& a, int Q, hipStream_t s) {
  if (a.y1 && a.y2 && a.mzt && dct_split_ok(a.D)) {
    switch (log2_half(a.D)) {
      case 10: launch_split<10>(a, Q, s); return;
      case 12: launch_split<12>(a, Q, s); return;
      case 14: launch_split<14>(a, Q, s); return;
      default: break;
    }
  }
  DCT_DISPATCH(k_dct_operator, Q, a, s);
}

}  // namespace cofem
