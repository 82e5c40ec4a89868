// Device helpers shared by the single-problem kernels and the serving kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace cofem {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8_t;
typedef __attribute__((ext_vector_type(4))) float f32x4;

constexpr int VCHUNK = 1024;  // coordinates per block of the per-column vector tiles (256 threads x 4)

// SplitMix64 finaliser (Steele, Lea & Flood 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// Key of EM iteration t: output t of the stream started at `seed`.
__device__ __forceinline__ uint64_t iteration_key(uint64_t seed, int t) {
  return mix64(seed + (uint64_t)t * GOLDEN_GAMMA);
}
// Word j of the stream started at the iteration key (output j + 1).
__device__ __forceinline__ uint64_t probe_word(uint64_t key, int64_t j) {
  return mix64(key + (uint64_t)(j + 1) * GOLDEN_GAMMA);
}
__device__ __forceinline__ float probe_sign(uint64_t w, int k) { return ((w >> k) & 1ull) ? -1.0f : 1.0f; }
// Entry (j, k) of the Sylvester-Hadamard matrix: (-1)^popcount(j & k).
__device__ __forceinline__ float hadamard_sign(int64_t j, int k) {
  return (__popcll((unsigned long long)j & (unsigned long long)k) & 1) ? -1.0f : 1.0f;
}

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
// The third slice of x after split_bf16: x = hi + lo + x3 exactly (x - hi - lo has at
// most 8 significant bits, so both subtractions are exact and x3 is a bf16 value).
__device__ __forceinline__ uint16_t slice3_bf16(float x, uint16_t hi, uint16_t lo) {
  return bf16_rne((x - bf16_val(hi)) - bf16_val(lo));
}
// Tile-interleaved layout of the FIR dictionary's bf16 signal slices of Q real columns
// (q < Q, j < Dp): for each 16-column tile and 32-sample block, the tile's columns' 32
// samples lie together (1 KB for a full tile), so that the filter kernels' loads of one
// block for a tile are one contiguous segment.  The last tile holds only its real columns
// (w = min(16, Q - 16 (q / 16))), so padding columns take neither space nor traffic; the
// whole layout spans Q Dp elements.
__host__ __device__ __forceinline__ int64_t sig_tile_width(int64_t q, int64_t Q) {
  const int64_t w = Q - (q & ~int64_t(15));
  return w < 16 ? w : 16;
}
__host__ __device__ __forceinline__ int64_t sig_index(int64_t q, int64_t j, int64_t Dp, int64_t Q) {
  return (q & ~int64_t(15)) * Dp + (j >> 5) * (32 * sig_tile_width(q, Q)) + (q & 15) * 32 + (j & 31);
}
// Four values' hi/lo slices (and, with X, their third slices) at offset o.  NT: stored
// non-temporally.  The dense contraction reads the right-hand-side slices that the kernel
// before it wrote (the direction, and V between the passes) through L2 by LDS DMA;
// written non-temporally, those lines are not left dirty in the writing XCD's L2 when the
// contraction starts: 386 -> 383 us per bf16 launch at N = 16384, D = 65536.
template <bool NT = false>
__device__ __forceinline__ void store_split4(uint16_t* H, uint16_t* L, int64_t o, const f32x4& v,
                                             uint16_t* X = nullptr) {
  typedef __attribute__((ext_vector_type(2))) unsigned int u32x2;
  uint16_t h[4], l[4], x[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    split_bf16(v[e], h[e], l[e]);
    x[e] = slice3_bf16(v[e], h[e], l[e]);
  }
  auto put = [](uint16_t* dst, const uint16_t (&s)[4]) {
    const u32x2 w{(uint32_t)s[0] | ((uint32_t)s[1] << 16), (uint32_t)s[2] | ((uint32_t)s[3] << 16)};
    if constexpr (NT) __builtin_nontemporal_store(w, reinterpret_cast<u32x2*>(dst));
    else *reinterpret_cast<u32x2*>(dst) = w;
  };
  put(H + o, h);
  put(L + o, l);
  if (X) put(X + o, x);
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

// Sum of p[i * stride] over i < n by one wave, in a fixed order (all lanes get it).  The
// unrolled loop issues UNR of a lane's loads together (registers permitting, 16 take
// 1024 values in one round trip); the additions keep their order whatever UNR.
template <int UNR = 8>
__device__ __forceinline__ double wave_sum_strided(const double* p, int n, int stride) {
  const int lane = threadIdx.x & 63;
  double a = 0.0;
#pragma unroll UNR
  for (int i = lane; i < n; i += 64) a += p[(int64_t)i * stride];
  return wave_sum(a);
}

// Tile order of the contractions.  Workgroups are dispatched round-robin over
// the 8 XCDs (tile L runs on XCD L % 8 when tiles are laid out from a multiple
// of 8), and each XCD has its own L2.  Blocks that share a split of the
// reduction dimension read the same slice of the right-hand-side block, so they
// are placed on the same XCD.
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

}  // namespace cofem
