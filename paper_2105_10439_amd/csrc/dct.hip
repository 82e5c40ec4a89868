// The subsampled DCT dictionary of Sec. V-A.2 on gfx950: Phi = M Omega^{-1}, where
// Omega is the orthonormal DCT-II of size D (Omega^{-1} = Omega^T, the DCT-III) and
// M keeps N of the D samples.  The operator of Algorithm 2 is then
//
//   Psi = beta Omega diag(m) Omega^T Pd + alpha Pd,   m_n = 1 for kept samples n,
//
// two fast transforms and a mask per right-hand side, O(D log D) work
// (Sec. III-B: applying a structured Phi costs tau_D = O(D log D)).
//
// One workgroup owns one right-hand side and keeps the whole transform chain in
// LDS, so a column makes one trip through HBM per operator application (read Pd
// and alpha, write Psi).  Both transforms go through one complex FFT of length
// L = D / 2 (D a power of two, 16 <= D <= 2^15, so the L complex FP32 points take
// at most 128 KB of the 160 KB of LDS):
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
__global__ void k_dct_mask(int L, const float* __restrict__ mx, float2* __restrict__ mz) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= L) return;
  const int D = 2 * L;
  auto mv = [&](int n) { return n < L ? mx[2 * n] : mx[2 * (D - 1 - n) + 1]; };
  mz[m] = make_float2(mv(2 * m), mv(2 * m + 1));
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

void launch_dct_setup(const int32_t* rows, int64_t N, int64_t D, int64_t Dp, int jacobi, float2* tw, float2* w2,
                      float2* mz, float* mx, float* theta, hipStream_t s) {
  const int L = (int)(D / 2);
  const int lg = log2_half(D) + 3, lo = (lg + 1) / 2, hi = lg - lo;
  const int n = std::max(L, 1 << lo);
  hipLaunchKernelGGL(k_dct_tables, dim3((n + 255) / 256), dim3(256), 0, s, L, lo, hi, tw, w2);
  launch_fill(mx, 0.0f, Dp, s);
  hipLaunchKernelGGL(k_dct_scatter, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, rows,
                     static_cast<const float*>(nullptr), N, mx);
  hipLaunchKernelGGL(k_dct_mask, dim3((L + 255) / 256), dim3(256), 0, s, L, mx, mz);
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

void launch_dct_operator(const DctArgs& a, int Q, hipStream_t s) { DCT_DISPATCH(k_dct_operator, Q, a, s); }

}  // namespace cofem
