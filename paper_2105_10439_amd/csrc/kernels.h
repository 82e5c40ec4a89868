// Internal interface between the gfx950 kernels (kernels.hip) and the host
// driver (cofem.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace cofem {

// Thread-local message of the last failing C-ABI call (shared by all entry points).
void set_error(const std::string& msg);

constexpr int QMAX = 64;          // padded right-hand-side columns per problem
constexpr int VBLOCK = 256;       // threads per block of the vector kernels
constexpr int VPART = 256;        // coordinates per partial-sum slot (sizes the reduction scratch)
constexpr uint64_t GOLDEN_GAMMA = 0x9E3779B97F4A7C15ull;

// Device-resident state of one multi-RHS PCG solve (Algorithm 2) and of the EM
// iteration around it.  All step scalars are FP64.  Scalars are written by
// single-block kernels; per-column flags by the first tile of the column.
struct CGState {
  double rho[QMAX];     // rho_q = sum_j R_jq W_jq
  double pi[QMAX];      // pi_q = sum_j P_jq Psi_jq
  double gamma[QMAX];   // gamma_q = rho_q / pi_q
  double eta[QMAX];     // eta_q = rho_q / rho_q^old
  double bn2[QMAX];     // ||B_q||^2
  double rn2[QMAX];     // ||R_q||^2 after the last update
  double bnorm2;        // ||B||_F^2 over the Q real columns
  double delta;         // ||R||_F / ||B||_F after the last update
  int active[QMAX];     // column still iterating
  int done;             // stop rule met or U steps taken
  int steps;            // operator applications in this solve
  int breakdown;        // columns frozen because pi_q <= 0 with rho_q != 0
  int clamped;          // M-step floor events (this fit)
  int phase;            // serving: 0 idle, 1 needs E-step init, 2 in CG, 3 finished
  int t;                // serving: current EM iteration (1-based)
  int total_steps;      // serving: CG steps over the fit
  int xpend;            // this step's update ran and left X += gamma P to the direction kernel
  int nonfinite;        // non-finite entries found in the last checked input (y, Phi or taps)
  double rho_prev[QMAX];  // rho_q as the update used it for gamma (the old rho of the direction)
};

struct SolveCfg {
  int Q, Qp, K, U, stop_mode;
  int nonneg;        // M-step of the non-negative model (Sec. III-E.2)
  double tol, beta;
  int hadamard = 0;  // probes: 0 the SplitMix64 hash, 1 columns 0..K-1 of the Sylvester-Hadamard matrix
  int sigblk = 0;    // bf16 slices of Pd in the tile-interleaved layout (sig_index): the FIR dictionary
  int nt_store = 0;  // launch choice: X, and P when its bf16 slices feed the operator, stored
                     // non-temporally (the operator streams more than the caches hold before
                     // they are read again)
};

// ---- setup -----------------------------------------------------------------
// Row stride (elements) of the library's padded dictionary layouts.  The transposed bf16
// copy gets 128 bytes of padding per row: row starts that are an odd multiple of 128
// bytes spread the rows a contraction tile streams at once over the HBM channels, where
// rows a multiple of 256 bytes long would land on the same few (bf16 tile at 16384 x
// 65536: 5.46 -> 5.61 TB/s on the N-long rows).  The row-major bf16 copy is stored
// split-blocked instead (see launch_dict_layouts).  FP32 rows stay unpadded: that
// contraction is bound by the FP32 matrix rate, and the pad measured 3 % slower.
constexpr int64_t DICT_ROW_PAD_BYTES = 128;
__host__ __device__ inline int64_t dict_ld(int64_t len, int elem_bytes) {
  return elem_bytes == 2 ? len + DICT_ROW_PAD_BYTES / elem_bytes : len;
}

// Copy the caller's N x D row-major FP32 dictionary into the library's layouts:
// phi32 (Np rows of dict_ld(Dp, 4)), phi32T (Dp rows of dict_ld(Np, 4)), phi16T (Dp
// rows of dict_ld(Np, 2), bf16 bits), and phi16 split-blocked: the reduction range of the
// first pass cut into the contraction's splits of kc16 columns, split s an Np x kc16
// row-major block at phi16 + s Np kc16 (cdiv(Dp, kc16) blocks).  Each split then streams
// whole contiguous rows (16 KB at the large size) instead of 16 KB pieces of 128 KB
// rows: 5.33 -> 5.73 TB/s on the first pass.  Any output pointer may be null.  Entries
// past D (or N) up to Dp (or Np) are zero; the row pad and the block tail past Dp are
// never read.
void launch_dict_layouts(const float* phi, int64_t N, int64_t D, int64_t Np, int64_t Dp, int64_t kc16, float* phi32,
                         float* phi32T, uint16_t* phi16, uint16_t* phi16T, hipStream_t s);

// theta_j = sum_i Phi_ij^2 (jacobi) or 1 from the caller's N x D matrix; padding 1.
void launch_theta(const float* phi, int64_t N, int64_t D, int64_t Dp, int jacobi, float* theta, hipStream_t s);

// b_j = beta * sum_i Phi_ij y_i from a transposed layout with rows of `ld` elements
// (FP32 if phi32T is not null, else the bf16 phi16T).
void launch_rhs(const float* phi32T, const uint16_t* phi16T, int64_t ld, int64_t Np, int64_t Dp, const float* y,
                double beta, float* b, hipStream_t s);

// x[0..n) = v.
void launch_fill(float* x, float v, int64_t n, hipStream_t s);
// *count += the number of entries of x[0..n) that are NaN or infinite.
void launch_count_nonfinite(const float* x, int64_t n, int* count, hipStream_t s);
// y[0..n) += a x[0..n).
void launch_axpy(float* y, const float* x, float a, int64_t n, hipStream_t s);

// ---- per EM iteration --------------------------------------------------------
// Probes for iteration key `key`, B = [b | p_1..p_K | 0], minv = 1/(beta theta + alpha),
// X = 0, R = B, Pd = W = minv R (FP32 and, if PdH != null, bf16 hi/lo, and if PdX != null
// the third slice: Pd = hi + lo + X exactly); then one block sets the initial rho,
// ||B_q||^2, active flags and resets done/steps (two launches).
void launch_em_init(const SolveCfg& c, uint64_t key, int64_t D, int64_t Dp, const float* b,
                    const float* theta, const float* alpha, float* minv, float* X, float* R, float* Pd,
                    uint16_t* PdH, uint16_t* PdL, double* part, CGState* st, hipStream_t s,
                    uint16_t* PdX = nullptr);

// mu = X_0, s = (1/K) sum_k p_k X_k (probes regenerated from `key`); if do_mstep,
// alpha = 1 / max(mu^2 + s, floor) and clamp events are counted in st->clamped.
void launch_mstep(const SolveCfg& c, uint64_t key, int64_t D, int64_t Dp, const float* X, float* mu,
                  float* s_out, float* alpha, double floor, int do_mstep, CGState* st, hipStream_t s);

// ---- operator A P = beta Phi^T (Phi P) + alpha P ----------------------------
struct GemmCfg {
  int rt;        // row tiles of 16 per wave (1, 2 or 4); a block has 4 waves
  int splits;    // split of the reduction dimension
  int64_t kchunk;
};
GemmCfg choose_gemm(int64_t rows, int64_t kdim, int bf16);

// Ypart[split][q][row] = sum_{k in split} M[row, k] Z[q, k] for the Q real columns (rows of
// Ypart past the column tiles are not written); Qp is the padded column count of Z and Ypart.
// bf16: M has rows of ldm elements, one block of rows (sps = 0) or split-blocked (split s at
// M + s sps, its rows holding k in [s kchunk, (s + 1) kchunk)).  FP32: rows of
// dict_ld(kdim, 4) elements.
// bf16: M, ZH, ZL are bf16 bits, products of M with ZH and ZL accumulate in FP32.
// FP32: M is FP32, Z is given as its three bf16 slices ZH + ZM + ZL (exact); the
// products are formed on the bf16 matrix cores from slices of both operands.
void launch_gemm_bf16(const GemmCfg& g, const uint16_t* M, int64_t ldm, int64_t sps, int64_t rows, int64_t kdim,
                      const uint16_t* ZH, const uint16_t* ZL, int Q, int Qp, float* Yp, const CGState* st,
                      hipStream_t s);
void launch_gemm_f32(const GemmCfg& g, const float* M, int64_t rows, int64_t kdim, const uint16_t* ZH,
                     const uint16_t* ZM, const uint16_t* ZL, int Q, int Qp, float* Ypart, const CGState* st,
                     hipStream_t s);

// V = sum_split Ypart (rows Np); writes V (FP32) and/or VH/VL (bf16 hi/lo) and VX (third slice).
void launch_finish_pass1(const float* Ypart, int splits, int Q, int Qp, int64_t Np, float* V, uint16_t* VH,
                         uint16_t* VL, const CGState* st, hipStream_t s, uint16_t* VX = nullptr);

// Psi = beta * sum_split Ypart + alpha * Pd (columns q < c.Q) and per-chunk partials of
// pi_q = sum_j Pd_jq Psi_jq into pipart ([q][chunk], chunks of 1024 coordinates).
void launch_finish_pass2(const SolveCfg& c, const float* Ypart, int splits, int64_t Dp, const float* alpha,
                         const float* Pd, float* Psi, double* pipart, const CGState* st, hipStream_t s);
// pi[q] = sum of the pi partials, q < Q (test hooks only; the CG update reduces them itself).
void launch_reduce_pi(int Q, int64_t Dp, const double* pipart, double* pi, hipStream_t s);

// ---- CG vector updates (Algorithm 2 after the operator) -----------------------
// gamma_q = rho_q / pi_q (pi reduced from pipart), X += Pd gamma, R -= Psi gamma, partials
// of ||R_q||^2 and rho'_q = sum R minv R into part; then (scalars) one block applies the stop
// rule and computes eta (a first block reduces the pi partials when a column has many).
// xdir: X += gamma Pd is left to launch_cg_direction (FIR dictionary, bf16 form: its direction
// kernel reads Pd anyway; pass 1 of the filter clears the state's flag each step).
// scalars = false leaves the scalar reductions to launch_cg_direction (when
// cg_direction_fuses_scalars), which then runs them in its own launch.
void launch_cg_update(const SolveCfg& c, int64_t Dp, const float* minv, float* X, float* R, const float* Pd,
                      const float* Psi, const double* pipart, double* part, CGState* st, hipStream_t s,
                      bool xdir = false, bool scalars = true);
// Whether launch_cg_direction runs the CG scalars too: for column-major directions (every
// form except the FIR dictionary's bf16 one).
bool cg_direction_fuses_scalars(const SolveCfg& c, const uint16_t* PdH);
// Pd = minv R + eta Pd (FP32, and bf16 hi/lo if PdH != null, and the third slice if PdX != null).
// With X (only with c.sigblk and PdH: the update's xdir form), first X += gamma Pd when the
// step's update ran, also on the step whose update met the stop rule.  When
// cg_direction_fuses_scalars, the same launch first reduces the update's partials `part`
// (the CG scalars, and eta per column; part is then required).
void launch_cg_direction(const SolveCfg& c, int64_t Dp, const float* minv, const float* R, float* Pd,
                         uint16_t* PdH, uint16_t* PdL, CGState* st, hipStream_t s, uint16_t* PdX = nullptr,
                         float* X = nullptr, const double* part = nullptr);

// Multi-task M-step over L tasks' mu and s (device arrays of L device pointers).
void launch_mt_mstep(const float* const* mus, const float* const* ss, int L, int64_t D, float* alpha, double floor,
                     int* clamped, hipStream_t s);

// ---- test-hook helpers ---------------------------------------------------------
// Copy ncols columns of length D (caller layout) into a Qp x Dp block (zero padding),
// optionally also as bf16 hi/lo (and the third slice dX), at sig_index of the ncols real
// columns when sigblk.
void launch_pack_block(const float* src, int ncols, int64_t D, int Qp, int64_t Dp, float* dst, uint16_t* dH,
                       uint16_t* dL, hipStream_t s, uint16_t* dX = nullptr, int sigblk = 0);
void launch_unpack_block(const float* src, int ncols, int64_t D, int64_t Dp, float* dst, hipStream_t s);
void launch_copy_pad(const float* src, int64_t n, int64_t np, float pad, float* dst, hipStream_t s);
void launch_state_reset(CGState* st, int Q, hipStream_t s);

// ---- convolutional dictionary (conv.hip) ----------------------------------------
// Phi_ij = h[i - j] for 0 <= i - j < L (N = D).  The taps live padded with zeros in
// hp32 / hp16 (CONV_HPAD entries, FP32 and bfloat16).
constexpr int CONV_MAX_TAPS = 256;
constexpr int CONV_HPAD = 384;

// One filter pass over the Qp x Dp blocks (columns q < Q are computed; runs of 1024
// samples per wave and 16-column tile).  dir 0: out = Phi in.  dir 1: out = beta Phi^T in
// + alpha Pd and the pi partials into pipart[q * nbx + run].  FP32 reads in32; bf16
// reads the hi/lo pair inH/inL (tile-interleaved, sig_index).  Pass 1 writes out32
// and/or outH/outL (tile-interleaved).
struct ConvArgs {
  const float* hp32;
  const uint16_t* hp16;
  int L;
  int64_t D, Dp;
  int Q, nct, nbx;
  const float* in32;
  const uint16_t *inH, *inL;
  float* out32;
  uint16_t *outH, *outL;
  double beta;
  const float* alpha;
  const float* Pd;               // FP32 form: Pd for the epilogue of pass 2
  const uint16_t *PdH, *PdL;     // bf16 form: Pd's hi/lo slices (tile-interleaved), its value there
  double* pipart;
  const int* done;
  int* xclear;  // pass 1 of a CG step zeroes the state's xpend flag (before the done test)
};
int conv_blocks_f32(int L);
int conv_blocks_bf16(int L);
// Pad the device taps h[0..L) into hp32 and hp16 (CONV_HPAD entries each).
void launch_conv_taps(const float* h, int L, float* hp32, uint16_t* hp16, hipStream_t s);
// Pad the device taps h[0..L) into hp32/hp16 and fill theta (Jacobi: column norms).
void launch_conv_setup(const float* h, int L, int64_t D, int64_t Dp, int jacobi, float* hp32, uint16_t* hp16,
                       float* theta, hipStream_t s);
// b = beta Phi^T y with the FP32 taps (hp16 null) or the bfloat16 taps.
void launch_conv_rhs(const float* hp32, const uint16_t* hp16, int L, int64_t D, int64_t Dp, const float* y,
                     double beta, float* b, hipStream_t s);
// One FP32 filter pass: dir 0, V = Phi Pd (in32 = Pd, out32 = V); dir 1, Psi = beta Phi^T V
// + alpha Pd and the pi partials (in32 = V, Pd, alpha, out32 = Psi, pipart).
void launch_conv_pass(const ConvArgs& a, int dir, hipStream_t s);
// The bf16 operator in one launch (both filters, V in registers): inH/inL = Pd's pair,
// alpha, out32 = Psi, pipart, xclear, done.
void launch_conv_op_bf16(const ConvArgs& a, hipStream_t s);

// ---- subsampled DCT dictionary (dct.hip) ----------------------------------------
// Phi = M Omega^{-1}: Omega the orthonormal DCT-II of size D, M keeps N samples.
// D is a power of two in [DCT_MIN_D, DCT_MAX_D] (the L = D / 2 point complex FFT
// of one column lives in LDS).
constexpr int64_t DCT_MIN_D = 16;
constexpr int64_t DCT_MAX_D = 32768;
constexpr int DCT_W2_SIZE = 1024;  // >= 2^lo + 2^hi for 4D = 2^(lo + hi) up to 4 DCT_MAX_D
bool dct_size_ok(int64_t D);

struct DctArgs {
  int64_t D, Dp;
  int nbx;                           // pi partial chunks per column, cdiv(Dp, 1024)
  float s0, s1;                      // orthonormal scales sqrt(1/D), sqrt(2/D)
  const float2 *tw, *mz;             // FFT twiddles (D/2 entries), mask pairs (D/2 entries)
  const float2* w2;                  // two-level table of e^{-2 pi i m / 4D} (DCT_W2_SIZE entries)
  const float* in;                   // operator: Pd (Qp x Dp); forward: one signal of D samples
  float* out;                        // operator: Psi; forward: beta Omega in
  double beta;
  const float* alpha;                // operator only
  double* pipart;                    // operator only: [q][chunk]
  const int* done;                   // operator only, may be null
  float2 *y1, *y2;                   // split operator only: exchange buffers, Qp x D/2 each
  const float2* mzt;                 // split operator only: mask pairs transposed, [k mod S][k / S]
};
// The split form of the operator (one column over several workgroups, three
// launches) exists for D = 2^11, 2^13 and 2^15; it needs y1, y2 and mzt.
bool dct_split_ok(int64_t D);
// Tables (tw: D/2, w2: DCT_W2_SIZE, mz: D/2 entries; mzt: D/2 entries or null), the mask (mx: Dp floats of
// scratch), and theta (Jacobi: column norms of Phi; else ones).  rows: N distinct
// sample indices in [0, D) on the device.
void launch_dct_setup(const int32_t* rows, int64_t N, int64_t D, int64_t Dp, int jacobi, float2* tw, float2* w2,
                      float2* mz, float2* mzt, float* mx, float* theta, hipStream_t s);
// b = beta Phi^T y = beta Omega (M^T y) into a.out (u: Dp floats of scratch).
void launch_dct_rhs(const DctArgs& a, const float* y, const int32_t* rows, int64_t N, float* u, hipStream_t s);
// Psi = A Pd for columns q < Q, one workgroup per column, with the pi partials.
void launch_dct_operator(const DctArgs& a, int Q, hipStream_t s);

}  // namespace cofem
