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
// The complex DFT is a Stockham autosort FFT (radix 4, a final radix 2 when log2 L
// is odd) in place in LDS: each pass loads its butterflies into registers, waits
// at a barrier, and stores the results.  Twiddles, the DCT phase factors and the
// mask come from small tables built once in FP64 and rounded to FP32.
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

// Threads per workgroup for L complex points: one radix-4 butterfly per thread
// up to 1024 threads, at least one wave.
constexpr int dct_threads(int log2L) {
  return ((1 << log2L) / 4 < 64) ? 64 : (((1 << log2L) / 4 > 1024) ? 1024 : (1 << log2L) / 4);
}

// One radix-4 Stockham pass over L points with NT threads; ns = size of the
// sub-transforms already done (1, 4, 16, ...).  Butterfly j reads points
// j + r L/4, multiplies point r by W_{4 ns}^{k r} (k = j mod ns) and writes its
// 4-point DFT to (j - k) 4 + k + r ns.  MASK: the pass reads the conjugated
// output of an inverse transform and applies the sample mask to it (see the
// operator kernel).
template <int L, int NT, bool MASK>
__device__ __forceinline__ void fft_radix4_pass(float2* buf, const float2* __restrict__ tw, int ns,
                                                const float2* __restrict__ mz) {
  constexpr int Q4 = L / 4;
  constexpr int BPT = (Q4 + NT - 1) / NT;
  float2 a[BPT][4];
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int j = threadIdx.x + b * NT;
    if (j < Q4) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float2 v = buf[j + r * Q4];
        if (MASK) {
          const float2 m = mz[j + r * Q4];
          v = make_float2(m.x * v.x, -m.y * v.y);
        }
        a[b][r] = v;
      }
    }
  }
  __syncthreads();
  const int stride = Q4 / ns;  // table step of W_{4 ns} = W_L^{L / (4 ns)}
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int j = threadIdx.x + b * NT;
    if (j < Q4) {
      const int k = j & (ns - 1);
      const float2 a0 = a[b][0];
      const float2 a1 = cmul(a[b][1], tw[k * stride]);
      const float2 a2 = cmul(a[b][2], tw[2 * k * stride]);
      const float2 a3 = cmul(a[b][3], tw[3 * k * stride]);
      const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
      const float2 t2 = cadd(a1, a3), t3 = ctimes_minus_i(csub(a1, a3));
      const int o = (j - k) * 4 + k;
      buf[o] = cadd(t0, t2);
      buf[o + ns] = cadd(t1, t3);
      buf[o + 2 * ns] = csub(t0, t2);
      buf[o + 3 * ns] = csub(t1, t3);
    }
  }
  __syncthreads();
}

// The last pass when log2 L is odd: radix 2 with ns = L / 2.
template <int L, int NT>
__device__ __forceinline__ void fft_radix2_last(float2* buf, const float2* __restrict__ tw) {
  constexpr int H = L / 2;
  constexpr int BPT = (H + NT - 1) / NT;
  float2 a[BPT][2];
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int j = threadIdx.x + b * NT;
    if (j < H) {
      a[b][0] = buf[j];
      a[b][1] = buf[j + H];
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int j = threadIdx.x + b * NT;
    if (j < H) {
      const float2 t = cmul(a[b][1], tw[j]);
      buf[j] = cadd(a[b][0], t);
      buf[j + H] = csub(a[b][0], t);
    }
  }
  __syncthreads();
}

// Forward DFT of the L points in buf (natural order in and out).  Callers place a
// barrier between their last write to buf and this call.
template <int LOG2L, bool MASK_FIRST>
__device__ __forceinline__ void fft_forward(float2* buf, const float2* __restrict__ tw,
                                            const float2* __restrict__ mz) {
  constexpr int L = 1 << LOG2L, NT = dct_threads(LOG2L);
  fft_radix4_pass<L, NT, MASK_FIRST>(buf, tw, 1, mz);
  int ns = 4;
#pragma unroll 1
  for (int p = 1; p < LOG2L / 2; ++p, ns *= 4) fft_radix4_pass<L, NT, false>(buf, tw, ns, mz);
  if constexpr ((LOG2L & 1) != 0) fft_radix2_last<L, NT>(buf, tw);
}

// V(k) = (Za + conj Zb) / 2 - i wh_k (Za - conj Zb) / 2: bin k of the real DFT of
// length D from bins k and L - k of the half-length complex DFT.
__device__ __forceinline__ float2 real_split(float2 za, float2 zb, float2 whk) {
  const float2 e = cscale(cadd(za, cconj(zb)), 0.5f);
  const float2 d = cmul(whk, cscale(csub(za, cconj(zb)), 0.5f));
  return cadd(e, ctimes_minus_i(d));
}

// After fft_forward: the DCT-II of the reordered signal, C_k = sum_n x_n
// cos(pi (2n + 1) k / 2D) (unnormalised), written over buf as D floats.
template <int LOG2L>
__device__ __forceinline__ void dct_post(float2* buf, const DctArgs& a) {
  constexpr int L = 1 << LOG2L, NT = dct_threads(LOG2L);
  constexpr int IT = (L / 2 + 1 + NT - 1) / NT;
  const int D = 2 * L;
  float2 A[IT], B[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int t = threadIdx.x + i * NT;
    if (t <= L / 2) {
      A[i] = buf[t];
      B[i] = buf[(L - t) & (L - 1)];
    }
  }
  __syncthreads();
  float* cb = reinterpret_cast<float*>(buf);
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int t = threadIdx.x + i * NT;
    if (t <= L / 2) {
      float2 w = cmul(a.wq[t], real_split(A[i], B[i], a.wh[t]));
      cb[t] = w.x;
      if (t > 0) cb[D - t] = -w.y;
      if (t == 0) {
        w = cmul(a.wq[L], real_split(A[i], A[i], a.wh[L]));
        cb[L] = w.x;
      } else if (t < L / 2) {
        w = cmul(a.wq[L - t], real_split(B[i], A[i], a.wh[L - t]));
        cb[L - t] = w.x;
        cb[L + t] = -w.y;
      }
    }
  }
  __syncthreads();
}

// Operator over one column per workgroup: Psi = beta Omega diag(m) Omega^T Pd +
// alpha Pd, and the FP64 partials of pi_q = sum_j Pd_jq Psi_jq per 1024
// coordinates at pipart[q * nbx + chunk].
template <int LOG2L>
__global__ __launch_bounds__(dct_threads(LOG2L)) void k_dct_operator(DctArgs a) {
  constexpr int L = 1 << LOG2L, NT = dct_threads(LOG2L);
  __shared__ __align__(16) float2 buf[L];
  if (a.done && *a.done) return;  // a step enqueued after the stop rule fired
  const int D = 2 * L;
  const int q = blockIdx.x;
  const float* __restrict__ p = a.in + (int64_t)q * a.Dp;
  // Inverse transform, spectrum side.  With c_k = s_k Pd_k, the Hermitian
  // spectrum of the reordered output is H_0 = c_0, H_k = e^{i pi k / 2D} (c_k -
  // i c_{D-k}) / 2; its half-length form is Z_k = E_k + i O_k with E_k = H_k +
  // conj H_{L-k}, O_k = (H_k - conj H_{L-k}) e^{2 pi i k / D}.  buf gets conj Z,
  // so that a forward DFT yields the conjugate of the inverse one.
  auto hval = [&](int k) -> float2 {
    if (k == 0) return make_float2(a.s0 * p[0], 0.0f);
    const float ck = a.s1 * p[k], cm = a.s1 * p[D - k];
    return cscale(cmul(cconj(a.wq[k]), make_float2(ck, -cm)), 0.5f);
  };
  auto zval = [&](float2 h1, float2 h2, float2 whk) -> float2 {
    const float2 e = cadd(h1, cconj(h2));
    const float2 o = cmul(csub(h1, cconj(h2)), cconj(whk));
    return cadd(e, ctimes_i(o));
  };
  for (int t = threadIdx.x; t <= L / 2; t += NT) {
    const float2 h1 = hval(t), h2 = hval(L - t);
    buf[t] = cconj(zval(h1, h2, a.wh[t]));
    if (t > 0 && t < L / 2) buf[L - t] = cconj(zval(h2, h1, a.wh[L - t]));
  }
  __syncthreads();
  fft_forward<LOG2L, false>(buf, a.tw, a.mz);
  // buf = conj(z), z_m = v_2m + i v_{2m+1} the reordered Omega^T Pd.  The next
  // transform's first pass reads z' = (m_2m v_2m, m_{2m+1} v_{2m+1}).
  fft_forward<LOG2L, true>(buf, a.tw, a.mz);
  dct_post<LOG2L>(buf, a);
  const float* __restrict__ cb = reinterpret_cast<const float*>(buf);
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  float* __restrict__ out = a.out + (int64_t)q * a.Dp;
  for (int c = wv; c < a.nbx; c += NT / 64) {
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t j = (int64_t)c * VCHUNK + i * 256 + 4 * ln;
      if (j < a.Dp) {
        f32x4 ps = {0.f, 0.f, 0.f, 0.f};
        if (j < D) {
          const f32x4 pv = *reinterpret_cast<const f32x4*>(p + j);
          const f32x4 al = *reinterpret_cast<const f32x4*>(a.alpha + j);
          const f32x4 cv = *reinterpret_cast<const f32x4*>(cb + j);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float sk = (j + e == 0) ? a.s0 : a.s1;
            ps[e] = (float)(a.beta * (double)(sk * cv[e]) + (double)al[e] * (double)pv[e]);
            acc += (double)pv[e] * (double)ps[e];
          }
        }
        *reinterpret_cast<f32x4*>(out + j) = ps;
      }
    }
    acc = wave_sum(acc);
    if (ln == 0) a.pipart[(int64_t)q * a.nbx + c] = acc;
  }
}

// out = beta Omega u for one signal u of D samples (the right-hand side b = beta
// Phi^T y once y is scattered to its samples); out is zero on [D, Dp).
template <int LOG2L>
__global__ __launch_bounds__(dct_threads(LOG2L)) void k_dct_forward(DctArgs a) {
  constexpr int L = 1 << LOG2L, NT = dct_threads(LOG2L);
  __shared__ __align__(16) float2 buf[L];
  const int D = 2 * L;
  const float* __restrict__ u = a.in;
  // z_m = v_2m + i v_{2m+1} with v_n = u_2n (n < L), v_n = u_{2(D-1-n)+1} (n >= L)
  for (int m = threadIdx.x; m < L; m += NT) {
    buf[m] = (m < L / 2) ? make_float2(u[4 * m], u[4 * m + 2]) : make_float2(u[2 * D - 4 * m - 1], u[2 * D - 4 * m - 3]);
  }
  __syncthreads();
  fft_forward<LOG2L, false>(buf, a.tw, a.mz);
  dct_post<LOG2L>(buf, a);
  const float* __restrict__ cb = reinterpret_cast<const float*>(buf);
  for (int64_t j = threadIdx.x; j < a.Dp; j += NT) {
    const float sk = (j == 0) ? a.s0 : a.s1;
    a.out[j] = (j < D) ? (float)(a.beta * (double)(sk * cb[j])) : 0.0f;
  }
}

// ---------------------------------------------------------------------------
// Set-up: tables, mask, theta, right-hand side
// ---------------------------------------------------------------------------
// tw_i = e^{-2 pi i i / L} (i < L); wq_k = e^{-i pi k / 2D}, wh_k = e^{-2 pi i k / D}
// (k <= L), from FP64 sincospi (the arguments are exact binary fractions).
__global__ void k_dct_tables(int L, float2* __restrict__ tw, float2* __restrict__ wq, float2* __restrict__ wh) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > L) return;
  const double D = 2.0 * L;
  double s, c;
  if (i < L) {
    sincospi(2.0 * i / L, &s, &c);
    tw[i] = make_float2((float)c, (float)-s);
  }
  sincospi(i / (2.0 * D), &s, &c);
  wq[i] = make_float2((float)c, (float)-s);
  sincospi(2.0 * i / D, &s, &c);
  wh[i] = make_float2((float)c, (float)-s);
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

void launch_dct_setup(const int32_t* rows, int64_t N, int64_t D, int64_t Dp, int jacobi, float2* tw, float2* wq,
                      float2* wh, float2* mz, float* mx, float* theta, hipStream_t s) {
  const int L = (int)(D / 2);
  hipLaunchKernelGGL(k_dct_tables, dim3((L + 1 + 255) / 256), dim3(256), 0, s, L, tw, wq, wh);
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
