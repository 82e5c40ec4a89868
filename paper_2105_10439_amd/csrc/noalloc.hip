// The FIR-dictionary operator with no device allocation (cofem_conv_apply_A_static).
//
// The same kernels and launch order as cofem_apply_A on a context of the FIR
// dictionary with the FP32 operator, but every piece of scratch memory (padded taps,
// padded alpha, the packed direction block, V = Phi P, the packed Psi, the pi partials
// and the pass state) is carved out of one file-scope device array.  Each device that
// runs this code holds its own copy of the array, at its own address, for the life of
// the process; the host side looks that address up once per device and passes it to
// the kernels as an ordinary pointer (the array's name in host code is only a
// registration handle, not a device address).
#include "cofem.h"
#include "device_common.h"
#include "kernels.h"

#include <cmath>
#include <mutex>
#include <string>

#define COFEM_API extern "C" __attribute__((visibility("default")))

using namespace cofem;

namespace {

static __device__ __align__(256) unsigned char scratch[COFEM_STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[MAX_DEVICES];  // device address of `scratch` per device, null until looked up

inline int64_t round_up(int64_t x, int64_t m) { return ((x + m - 1) / m) * m; }

cofem_status fail(cofem_status s, const std::string& msg) {
  set_error(msg);
  return s;
}

// Byte offsets of the scratch regions for one call (each 256-byte aligned).
struct StaticLayout {
  int64_t Dp, Qp, nbx;
  size_t st, hp32, hp16, alpha, Pd, V, Psi, pipart, total;
};

StaticLayout static_layout(int64_t D, int ncols) {
  StaticLayout l{};
  l.Dp = round_up(D, 256);
  l.Qp = round_up(ncols, 16);
  l.nbx = (l.Dp + VCHUNK - 1) / VCHUNK;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += (size_t)round_up((int64_t)bytes, 256);
    return at;
  };
  l.st = take(sizeof(CGState));
  l.hp32 = take(sizeof(float) * CONV_HPAD);
  l.hp16 = take(sizeof(uint16_t) * CONV_HPAD);
  l.alpha = take(sizeof(float) * (size_t)l.Dp);
  l.Pd = take(sizeof(float) * (size_t)(l.Qp * l.Dp));
  l.V = take(sizeof(float) * (size_t)(l.Qp * l.Dp));
  l.Psi = take(sizeof(float) * (size_t)(l.Qp * l.Dp));
  l.pipart = take(sizeof(double) * (size_t)(l.Qp * l.nbx));
  l.total = o;
  return l;
}

// The device address of `scratch` on the current device, looked up on the first call
// there (with that device current) and kept.
cofem_status scratch_on_current_device(unsigned char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(COFEM_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(COFEM_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(COFEM_EDEVICE, std::string("hipGetSymbolAddress of the scratch array: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return COFEM_OK;
}

}  // namespace

COFEM_API cofem_status cofem_conv_apply_A_static(const float* h, int32_t L, int64_t D, double beta,
                                                 const float* alpha, const float* P, float* Psi, int32_t ncols,
                                                 double* pi, void* stream) {
  if (!h || !alpha || !P || !Psi) return fail(COFEM_EINVAL, "NULL argument");
  if (L < 1 || L > CONV_MAX_TAPS)
    return fail(COFEM_EINVAL, "L must be in [1, " + std::to_string(CONV_MAX_TAPS) + "]");
  if (D < 1) return fail(COFEM_EINVAL, "D must be >= 1");
  if (ncols < 1 || ncols > COFEM_MAX_K + 1)
    return fail(COFEM_EINVAL, "ncols must be in [1, " + std::to_string(COFEM_MAX_K + 1) + "]");
  if (!(beta > 0.0) || !std::isfinite(beta)) return fail(COFEM_EINVAL, "beta must be positive and finite");
  if (D > ((int64_t)1 << 40)) return fail(COFEM_EINVAL, "D too large for the static scratch");
  const StaticLayout l = static_layout(D, ncols);
  if (l.total > (size_t)COFEM_STATIC_SCRATCH_BYTES)
    return fail(COFEM_EINVAL, "D = " + std::to_string(D) + " with " + std::to_string(ncols) + " columns needs " +
                                  std::to_string(l.total) + " bytes of scratch, more than the static " +
                                  std::to_string((size_t)COFEM_STATIC_SCRATCH_BYTES) + "-byte array");
  unsigned char* base = nullptr;
  cofem_status rc = scratch_on_current_device(&base);
  if (rc != COFEM_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  CGState* st = reinterpret_cast<CGState*>(base + l.st);
  float* hp32 = reinterpret_cast<float*>(base + l.hp32);
  uint16_t* hp16 = reinterpret_cast<uint16_t*>(base + l.hp16);
  float* alpha_p = reinterpret_cast<float*>(base + l.alpha);
  float* Pd = reinterpret_cast<float*>(base + l.Pd);
  float* V = reinterpret_cast<float*>(base + l.V);
  float* PsiP = reinterpret_cast<float*>(base + l.Psi);
  double* pipart = reinterpret_cast<double*>(base + l.pipart);

  // the state's done flag must read 0 for the filter passes (a previous call's state stays behind)
  launch_state_reset(st, ncols, s);
  launch_conv_taps(h, L, hp32, hp16, s);
  launch_copy_pad(alpha, D, l.Dp, 1.0f, alpha_p, s);
  launch_pack_block(P, ncols, D, (int)l.Qp, l.Dp, Pd, nullptr, nullptr, s);
  ConvArgs a{};
  a.hp32 = hp32;
  a.hp16 = hp16;
  a.L = L;
  a.D = D;
  a.Dp = l.Dp;
  a.Q = ncols;
  a.nct = (ncols + 15) / 16;
  a.nbx = (int)l.nbx;
  a.beta = beta;
  a.done = &st->done;
  ConvArgs p1 = a, p2 = a;
  p1.in32 = Pd;
  p1.out32 = V;
  p2.in32 = V;
  p2.out32 = PsiP;
  p2.alpha = alpha_p;
  p2.Pd = Pd;
  p2.pipart = pipart;
  launch_conv_pass(p1, 0, s);
  launch_conv_pass(p2, 1, s);
  launch_unpack_block(PsiP, ncols, D, l.Dp, Psi, s);
  if (pi) launch_reduce_pi(ncols, l.Dp, pipart, pi, s);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(COFEM_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  return COFEM_OK;
}
