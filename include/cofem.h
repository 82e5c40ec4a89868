/*
 * cofem.h -- C ABI of the covariance-free EM (CoFEM) hot path for AMD gfx950.
 *
 * The problem (Eq. sparse-coding, Sec. I): y = Phi z + eps with y in R^N,
 * z in R^D, Phi in R^{N x D}.  The model (Eq. model, Sec. II-A) puts
 * z ~ N(0, diag(alpha)^-1) and y | z ~ N(Phi z, beta^-1 I) with the noise
 * precision beta fixed.  A fit runs Algorithm 1 (CovarianceFreeEM(y, Phi,
 * beta, T, K)): T EM iterations, each solving A X = B with
 * A = beta Phi^T Phi + diag(alpha) and B = [beta Phi^T y | p_1 .. p_K]
 * (Eq. mat-eq) by the multi-RHS preconditioned CG of Algorithm 2 with the
 * diagonal preconditioner M = diag(beta theta + alpha) (Sec. III-C), then
 * forming mu, the diagonal estimate s_j = (1/K) sum_k p_kj x_kj
 * (Eq. diag-estimate) and, for t < T, alpha_j = 1 / (mu_j^2 + s_j)
 * (Eq. mstep with Sigma_jj replaced by s_j).  It returns alpha^(T), mu, s.
 *
 * Conventions shared by every entry point:
 *   - Every array argument is DEVICE memory on the device that was current
 *     when the context was created, unless a comment says "host".
 *   - Matrices are row-major and contiguous.  A "block of Q columns of length
 *     L" is Q contiguous vectors of L floats each (column q starts at q * L).
 *   - The caller owns every buffer it passes; the library never frees or
 *     retains caller pointers beyond the call, reads inputs only and writes
 *     outputs only.  The library owns its workspace (copies of the
 *     dictionary in its own layouts, CG blocks, reduction scratch).
 *   - All work is enqueued on the HIP stream given at creation (NULL = the
 *     default stream).  Calls that return results block until the stream has
 *     finished them.
 *   - Functions return COFEM_OK or a negative status; the thread-local
 *     cofem_last_error() then holds a message.  Arguments are validated
 *     before any device work; no C++ exception crosses this boundary.
 *   - A context is not thread-safe: calls on one context must not overlap.
 */
#ifndef COFEM_H
#define COFEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define COFEM_ABI_VERSION 7
#define COFEM_MAX_T 512 /* longest EM run recorded in cofem_stats */
#define COFEM_MAX_K 63  /* probes per EM iteration (one 64-bit hash word per coordinate) */

typedef struct cofem_ctx cofem_ctx;

typedef enum {
  COFEM_OK = 0,
  COFEM_EINVAL = -1,     /* bad argument or parameter combination */
  COFEM_ENOMEM = -2,     /* device allocation failed */
  COFEM_EDEVICE = -3,    /* a HIP runtime call failed */
  COFEM_ESTATE = -4,     /* call out of order (e.g. fit before set_dictionary) */
  COFEM_EBREAKDOWN = -5, /* CG breakdown (pi_q <= 0) in the mu column */
  COFEM_EBUDGET = -6     /* serving: request larger than the whole memory budget */
} cofem_status;

typedef enum { COFEM_THETA_ONES = 0, COFEM_THETA_JACOBI = 1 } cofem_theta_mode;
typedef enum { COFEM_STOP_JOINT = 0, COFEM_STOP_COLUMN = 1 } cofem_stop_mode;
typedef enum { COFEM_OP_DENSE = 0, COFEM_OP_CONV = 1, COFEM_OP_DCT = 2 } cofem_op_kind;
typedef enum { COFEM_PHI_FP32 = 0, COFEM_PHI_BF16 = 1 } cofem_phi_dtype;
typedef enum { COFEM_MSTEP_GAUSSIAN = 0, COFEM_MSTEP_NONNEG = 1 } cofem_mstep_mode;
typedef enum { COFEM_PROBES_HASH = 0, COFEM_PROBES_HADAMARD = 1 } cofem_probe_mode;

/*
 * Fit parameters.  Names follow Algorithms 1 and 2.
 *   N, D        sizes of y and z (Eq. sparse-coding); for COFEM_OP_CONV N must equal D;
 *               for COFEM_OP_DCT D is a power of two in [16, 32768] and N <= D.
 *   beta        noise precision, > 0 (Eq. model).
 *   K           Rademacher probes per EM iteration, 1..COFEM_MAX_K (Alg. 1).
 *   T           EM iterations, 1..COFEM_MAX_T (Alg. 1); T E-steps and T-1 M-steps.
 *   U           maximum CG steps per E-step, >= 1 (Alg. 2).
 *   tol         epsilon_max of the CG stop test (Alg. 2), >= 0.
 *   theta_mode  preconditioner M = diag(beta theta + alpha) with theta = 1
 *               (COFEM_THETA_ONES) or theta_j = sum_i Phi_ij^2 (Jacobi), Sec. III-C.
 *   stop_mode   COFEM_STOP_JOINT: stop when ||R||_F / ||B||_F <= tol (the printed
 *               test); COFEM_STOP_COLUMN: freeze column q once ||R_q||/||B_q|| <= tol.
 *   op_kind     COFEM_OP_DENSE: Phi is a dense N x D matrix.  COFEM_OP_CONV: Phi is
 *               the D x D causal convolution Phi_ij = h[i - j], 0 <= i - j < conv_taps
 *               (the convolutional dictionary of Sec. V-A.2).  COFEM_OP_DCT: Phi =
 *               M Omega^{-1}, Omega the orthonormal DCT-II of size D and M keeping N
 *               of the D samples (the DCT dictionary of Sec. V-A.2); FP32 only.
 *   phi_dtype   arithmetic of the operator: COFEM_PHI_FP32, or COFEM_PHI_BF16 (Phi
 *               rounded to bfloat16 once, products accumulated in FP32).
 *   refine_last with COFEM_PHI_BF16: the last refine_last E-steps use the FP32 operator.
 *   conv_taps   FIR length L for COFEM_OP_CONV (1..256); ignored otherwise.
 *   seed        probe seed.  Probe entry p_{k,j} at EM iteration t is +1 if bit k of
 *               w(t, j) is 0 and -1 otherwise, where w(t, j) is output j+1 of the
 *               SplitMix64 stream started at key_t, and key_t is output t of the
 *               SplitMix64 stream started at seed (Steele, Lea & Flood 2014).
 *   alpha_floor M-step denominators below it are raised to it (> 0); with the
 *               non-negative M-step it also floors s_j used as the posterior variance.
 *   mstep_mode  COFEM_MSTEP_GAUSSIAN: alpha_j = 1 / (mu_j^2 + s_j) (Eq. mstep).
 *               COFEM_MSTEP_NONNEG: the rectified-Gaussian prior of Sec. III-E.2;
 *               alpha_j = 1 / E[z_j^2] with the second moment of Eq. (nonneg-sbl),
 *               s_j in place of Sigma_jj (the truncated-Gaussian moment carries
 *               sqrt(2 s_j / pi)).  mu and s are the Gaussian E-step's in both modes.
 *   reserved_   set to 0.
 */
typedef struct cofem_params {
  int64_t N, D;
  double beta;
  int32_t K, T, U;
  double tol;
  int32_t theta_mode;
  int32_t stop_mode;
  int32_t op_kind;
  int32_t phi_dtype;
  int32_t refine_last;
  int32_t conv_taps;
  uint64_t seed;
  double alpha_floor;
  int32_t mstep_mode;
  int32_t reserved_;
} cofem_params;

/* Per-fit record (host struct, filled by cofem_posterior). */
typedef struct cofem_stats {
  int32_t T;                       /* EM iterations run */
  int32_t cg_steps[COFEM_MAX_T];   /* operator applications in E-step t (index t-1) */
  double rel_resid[COFEM_MAX_T];   /* ||R||_F / ||B||_F at the end of E-step t */
  int32_t used_bf16[COFEM_MAX_T];  /* 1 if E-step t used the bfloat16 operator */
  int64_t clamped;                 /* M-step denominators raised to alpha_floor */
  int32_t breakdown;               /* columns that hit pi_q <= 0 */
  int32_t total_cg_steps;          /* sum of cg_steps */
  double ms_setup;                 /* host wall time of cofem_set_dictionary */
  double ms_fit;                   /* host wall time of cofem_fit */
} cofem_stats;

/* Library ABI version (COFEM_ABI_VERSION). */
int32_t cofem_abi_version(void);

/* Thread-local message for the last failing call on this thread ("" if none). */
const char* cofem_last_error(void);

/*
 * Validate *p, allocate the workspace for problems of that shape on the current
 * device and bind the context to `stream` (a hipStream_t, NULL = default).
 * On success *out owns the context; release it with cofem_destroy.
 * Errors: COFEM_EINVAL (bad parameters), COFEM_ENOMEM, COFEM_EDEVICE.
 */
cofem_status cofem_create(const cofem_params* p, void* stream, cofem_ctx** out);

/* Free the context and its workspace (NULL is a no-op). */
void cofem_destroy(cofem_ctx* c);

/*
 * Load the dictionary: for COFEM_OP_DENSE `phi` is the N x D row-major FP32 matrix;
 * for COFEM_OP_CONV it is the conv_taps FIR taps h[0..taps-1].  The library copies
 * it into its own layouts (row-major and transposed, FP32 and/or bfloat16, padded)
 * and computes theta (Sec. III-C); `phi` may be freed when the call returns.
 * Errors: COFEM_EINVAL (NULL, or a COFEM_OP_DCT context), COFEM_EDEVICE.
 */
cofem_status cofem_set_dictionary(cofem_ctx* c, const float* phi);

/*
 * Load a COFEM_OP_DCT dictionary Phi = M Omega^{-1} (Sec. V-A.2): `rows` holds N
 * int32 sample indices on the device, distinct and in [0, D); entry i of y is
 * sample rows[i] of the inverse DCT of z.  The library copies them, builds its
 * transform tables and the sample mask, and computes theta (Jacobi: theta_j =
 * sum_i Omega_{j, rows_i}^2); `rows` may be freed when the call returns.
 * Errors: COFEM_EINVAL (NULL, not a DCT context, an index out of range or
 * repeated), COFEM_EDEVICE.
 */
cofem_status cofem_set_dct_samples(cofem_ctx* c, const int32_t* rows);

/*
 * Run Algorithm 1 on observation y (N floats, device) with the loaded dictionary.
 * Results stay on the device until cofem_posterior.  Non-convergence of CG within
 * U steps is not an error (Alg. 2 returns X after U steps); it shows in the stats.
 * Errors: COFEM_ESTATE (no dictionary), COFEM_EINVAL, COFEM_EDEVICE,
 * COFEM_EBREAKDOWN (the mu column broke down; results are still written).
 */
cofem_status cofem_fit(cofem_ctx* c, const float* y);

/*
 * Copy the fit's results into caller buffers of D floats each (device; any may be
 * NULL): mu and s from the E-step of iteration T, alpha = alpha^(T).  If st is
 * non-NULL (host) it receives the fit record.  Errors: COFEM_ESTATE (no fit yet).
 */
cofem_status cofem_posterior(cofem_ctx* c, float* mu, float* s, float* alpha, cofem_stats* st);

/*
 * Post-fit posterior variance (the variance maps of the MRI appendix, with the
 * identity as the image-domain map): an estimate of diag(Sigma), Sigma = (beta
 * Phi^T Phi + diag(alpha))^{-1}, from K * batches Rademacher probes.  Batch b =
 * 1..batches solves A X = [beta Phi^T y | p_1 .. p_K] (Alg. 2 with the context's
 * stop rule and tolerance, y of the last cofem_fit) with the probes of iteration
 * key b of the SplitMix64 stream started at `seed` (the construction of the fit's
 * probes, with b in place of t), and forms the diagonal estimate of Eq.
 * (diag-estimate); the result is the mean over the batches.
 *   alpha   D floats on the device, or NULL for the fit's alpha^(T).
 *   s_out   D floats on the device: the estimate.
 *   mu_out  D floats on the device, or NULL: the posterior mean at alpha.
 *   st      optional host record: cg_steps[b-1] and rel_resid[b-1] per batch,
 *           T = batches, ms_fit = wall time of this call.
 * The operator is FP32 when the context holds the FP32 dictionary, else bf16.
 * The fit's mu, s and alpha are kept (cofem_posterior still returns them).
 * Errors: COFEM_EINVAL (NULL s_out, batches outside [1, COFEM_MAX_T]),
 * COFEM_ESTATE (no successful fit), COFEM_EDEVICE, COFEM_EBREAKDOWN.
 */
cofem_status cofem_variance(cofem_ctx* c, const float* alpha, int32_t batches, uint64_t seed, float* s_out,
                            float* mu_out, cofem_stats* st);

/*
 * One application of the operator of Alg. 2 (the product of A with the search directions):
 * Psi = beta Phi^T (Phi P) + diag(alpha) P for a block of ncols (1..COFEM_MAX_K+1)
 * columns of length D, with the loaded dictionary, alpha (D floats) and the
 * FP32 (use_bf16 = 0) or bfloat16 (use_bf16 = 1, needs phi_dtype = BF16) operator.
 * If pi is non-NULL (device, ncols doubles) it receives pi_q = sum_j P_jq Psi_jq.
 * The bfloat16 operator applies the rounded dictionary to P's hi/lo bfloat16 pair
 * (hi = RNE(P), lo = RNE(P - hi)); for the FIR dictionary that pair is also the P of
 * diag(alpha) P and of pi (the form its CG steps carry), for the others P itself is.
 * Errors: COFEM_ESTATE (no dictionary), COFEM_EINVAL.
 */
cofem_status cofem_apply_A(cofem_ctx* c, const float* alpha, const float* P, float* Psi,
                           int32_t ncols, int32_t use_bf16, double* pi);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the FP32 operator of
 * cofem_apply_A for the FIR dictionary (Phi_ij = h[i - j], 0 <= i - j < L, N = D),
 * with no context and no allocation.  Same kernels, same launch order, same
 * results as cofem_apply_A on a context with op_kind = COFEM_OP_CONV, conv_taps = L
 * and the taps h loaded, use_bf16 = 0.
 *   h       L floats on the device (1 <= L <= 256): the filter taps.
 *   D       signal length, >= 1.
 *   beta    > 0.
 *   alpha   D floats on the device.
 *   P, Psi  blocks of ncols (1..COFEM_MAX_K+1) columns of length D on the device:
 *           Psi = beta Phi^T (Phi P) + diag(alpha) P.
 *   pi      NULL, or ncols doubles on the device: pi_q = sum_j P_jq Psi_jq.
 *   stream  HIP stream (NULL = the default stream) on the current device.
 * Scratch: every intermediate lives in one static device array of
 * COFEM_STATIC_SCRATCH_BYTES per device, held until the process ends; the call
 * needs 12 Qp Dp + 4 Dp + 8 Qp cdiv(Dp, 1024) bytes plus about 6 KB (Dp = D rounded
 * up to 256, Qp = ncols rounded up to 16), e.g. D = 2^16 with up to 64 columns or
 * D = 2^18 with up to 16.  The first call on a device
 * looks up that device's copy of the array (hipGetSymbolAddress): make it outside
 * graph capture.  Calls on one device share the array: calls that overlap in time
 * on one device (other streams, other threads) race and give wrong results.
 * The call only enqueues work on `stream` and returns; it does not synchronize.
 * Errors: COFEM_EINVAL (NULL h/alpha/P/Psi, L, D, ncols or beta out of range, or a
 * size that needs more scratch than the array holds; nothing is enqueued),
 * COFEM_EDEVICE (address lookup or launch failure).
 */
#define COFEM_STATIC_SCRATCH_BYTES (64u << 20)
cofem_status cofem_conv_apply_A_static(const float* h, int32_t L, int64_t D, double beta, const float* alpha,
                                       const float* P, float* Psi, int32_t ncols, double* pi, void* stream);

/*
 * Test hook: the probes of every later E-step (fits and cofem_variance).
 *   COFEM_PROBES_HASH (default): Rademacher probes from the counter-based hash,
 *     redrawn each EM iteration (Sec. III-A, Alg. 1).
 *   COFEM_PROBES_HADAMARD: probe k (k < K) is column k of the D x D
 *     Sylvester-Hadamard matrix, entry (j, k) = (-1)^popcount(j & k), the same in
 *     every EM iteration.  With K = D the cross terms of the diagonal estimate
 *     (Eq. diag-estimate) cancel, because distinct rows of a Hadamard matrix are
 *     orthogonal, and CoFEM reproduces EM with the explicit covariance up to the CG
 *     tolerance: a check of the whole path against a closed form.
 * Errors: COFEM_EINVAL (NULL context, unknown mode; Hadamard with D not a power of
 * two or K > D).
 */
cofem_status cofem_set_probe_mode(cofem_ctx* c, int32_t mode);

/*
 * Accumulated device time of the operator's matrix kernels (the two passes of
 * Phi P and Phi^T V) since the last reset, timed with HIP events recorded on the
 * context's stream around each launch when timing is enabled.
 *   cofem_set_timing(c, 1) enables and resets; (c, 0) disables.
 *   cofem_get_timing returns total milliseconds and the number of timed launches
 *   for the bfloat16 (which = 1) or FP32 (which = 0) operator.
 */
cofem_status cofem_set_timing(cofem_ctx* c, int32_t enable);
cofem_status cofem_get_timing(cofem_ctx* c, int32_t which, double* total_ms, int64_t* launches);

/* ---------------------------------------------------------------------------
 * Multi-task CoFEM (Sec. III-E.1): L sparse-coding problems y_l = Phi_l z_l + eps_l
 * whose codes share one sparsity profile alpha.  Every EM iteration runs the
 * covariance-free E-step of each task at the shared alpha (task l draws its probes
 * with seed + l), then the joint M-step alpha_j = L / sum_l (mu_lj^2 + s_lj),
 * raised to 1 / alpha_floor like the single-task M-step.
 * ------------------------------------------------------------------------- */
typedef struct cofem_mt cofem_mt;

#define COFEM_MAX_TASKS 64

/* How the L E-steps of an EM iteration run (cofem_mt_create_mode). */
#define COFEM_MT_AUTO 0    /* batched when the settings allow it and L > 4, else streams */
#define COFEM_MT_STREAMS 1 /* one context per task, each on its own stream */
#define COFEM_MT_BATCHED 2 /* all tasks' systems together, one launch per phase */
#define COFEM_MT_AUTO_STREAMS_MAX 4 /* COFEM_MT_AUTO: the most tasks it runs as streams */

/*
 * Validate *p (the shape N x D and the settings every task shares; mstep_mode must
 * be COFEM_MSTEP_GAUSSIAN) and allocate L task workspaces on the current device.
 *
 * COFEM_MT_BATCHED solves the L (K + 1) systems of an EM iteration together, as
 * Sec. III-E.1 describes: every CG step of every task is one launch per phase (the
 * operator's two contractions over all tasks' tiles, the vector kernels over all
 * tasks' columns), captured as a graph of 8 CG steps; each task keeps its own stop
 * rule (Algorithm 2 per task), and the joint M-step runs on the device once every
 * task's E-step has ended, so the tasks advance through the EM iterations together.
 * It takes dense FP32 dictionaries (op_kind COFEM_OP_DENSE, phi_dtype
 * COFEM_PHI_FP32), refine_last 0 and K <= 31; all work runs on `stream`.
 *
 * COFEM_MT_STREAMS runs one context per task: task 0 on `stream`, every other task on
 * a stream the library creates (and destroys with the handle); the loading calls and
 * cofem_mt_fit order them after `stream` at their start and cofem_mt_fit orders
 * `stream` after them at its end, so the caller sees the fit's work on `stream` alone.
 * Dense, FIR and subsampled-DCT dictionaries, every precision form.
 *
 * COFEM_MT_AUTO takes the batched form when *p allows it and L > COFEM_MT_AUTO_STREAMS_MAX:
 * the task streams overlap only as far as the hardware queues of a process go (4 by
 * default), so beyond that the batched form is faster (measured at K = 20: L = 16 tasks of
 * 1024 x 4096, 97 against 69 EM iterations/s; L = 32 of 512 x 2048, 140 against 45), while
 * at L = 4 the streams overlap their small kernels better (L = 4 of 2048 x 8192: 66 against
 * 61).  1 <= L <= COFEM_MAX_TASKS.
 * Errors: COFEM_EINVAL (bad parameters or mode, or COFEM_MT_BATCHED with settings it
 * does not take), COFEM_ENOMEM, COFEM_EDEVICE.
 */
cofem_status cofem_mt_create_mode(const cofem_params* p, int32_t L, int32_t mode, void* stream, cofem_mt** out);

/* cofem_mt_create_mode with COFEM_MT_AUTO. */
cofem_status cofem_mt_create(const cofem_params* p, int32_t L, void* stream, cofem_mt** out);

/* 1 if the handle runs the batched form, 0 otherwise (NULL: 0). */
int32_t cofem_mt_batched(const cofem_mt* m);

/* Free the tasks and their workspaces (NULL is a no-op). */
void cofem_mt_destroy(cofem_mt* m);

/* Load task `task`'s dictionary (as cofem_set_dictionary).  Errors: COFEM_EINVAL, COFEM_EDEVICE. */
cofem_status cofem_mt_set_dictionary(cofem_mt* m, int32_t task, const float* phi);
/* Load task `task`'s kept DCT samples (as cofem_set_dct_samples; op_kind COFEM_OP_DCT;
 * the streams form only).  Errors: COFEM_EINVAL, COFEM_EDEVICE. */
cofem_status cofem_mt_set_dct_samples(cofem_mt* m, int32_t task, const int32_t* rows);

/*
 * Run the multi-task EM: `ys` is a host array of L device pointers, ys[l] holding
 * task l's N observations.  Errors: COFEM_ESTATE (a dictionary missing), COFEM_EINVAL,
 * COFEM_EDEVICE, COFEM_EBREAKDOWN (some task's mu column broke down).
 */
cofem_status cofem_mt_fit(cofem_mt* m, const float* const* ys);

/*
 * Task `task`'s mu and s from its last E-step, and the shared alpha^(T), into caller
 * device buffers of D floats (any may be NULL); st (host) receives the task's record
 * (the clamp count of the joint M-step is reported with task 0).
 * Errors: COFEM_EINVAL, COFEM_ESTATE (no fit yet).
 */
cofem_status cofem_mt_posterior(cofem_mt* m, int32_t task, float* mu, float* s, float* alpha, cofem_stats* st);


/* ---------------------------------------------------------------------------
 * Serving: continuous batching of independent fits.
 *
 * A server owns one device arena of `hbm_budget` bytes and up to `max_slots`
 * concurrent fits.  Requests are admitted first-in first-out whenever a slot is
 * free and the request's workspace fits in the arena; admitted fits advance
 * together: every tick runs `steps_per_tick` CG steps of every running fit in one
 * graph-captured sequence of persistent kernels (each kernel strides over a tile
 * table that covers all running fits), and each fit moves through its own EM
 * iterations on the device (E-step initialisation, PCG, M-step, Algorithm 1).
 * Fits are independent and their reductions run in a fixed order, so a result
 * does not depend on which other requests share the device.
 *
 * Serving requests: op_kind COFEM_OP_DENSE, phi_dtype COFEM_PHI_FP32,
 * refine_last 0, K <= 31.
 * ------------------------------------------------------------------------- */
typedef struct cofem_server cofem_server;

typedef enum {
  COFEM_REQ_PENDING = 0, /* submitted, waiting for a slot and memory */
  COFEM_REQ_RUNNING = 1, /* admitted; the caller's phi and y are no longer read */
  COFEM_REQ_DONE = 2,    /* results available through cofem_server_poll */
  COFEM_REQ_UNKNOWN = -1
} cofem_request_state;

typedef struct cofem_request_info {
  int32_t state;           /* cofem_request_state */
  int32_t T;               /* EM iterations */
  int32_t total_cg_steps;  /* CG steps over the fit */
  int32_t pad_;
  double t_submit_ms;      /* host clock, ms since the server was created */
  double t_admit_ms;
  double t_finish_ms;
  int64_t bytes;           /* device workspace of the request */
} cofem_request_info;

typedef struct cofem_server_stats {
  int64_t submitted, admitted, completed, rejected;
  int64_t ticks;
  int32_t active;        /* running fits now */
  int32_t max_active;    /* most fits running at once */
  int64_t bytes_in_use;  /* arena bytes held by running fits */
  int64_t bytes_peak;    /* never above budget */
  int64_t budget;
  double tick_ms;        /* device time of the ticks' kernel sequences (events around each) */
  double dict_bytes;     /* dictionary bytes the completed fits' CG steps read by algorithm:
                            sum over them of (CG steps) x 2 passes x N D x 4 bytes */
} cofem_server_stats;

/*
 * Create a server on the current device.  hbm_budget: arena size in bytes (allocated
 * here, once).  max_slots: 1..128 concurrent fits.  steps_per_tick: CG steps per
 * tick (>= 1).  stream: hipStream_t to run on, or NULL for a server-owned stream
 * (stream capture needs a non-default stream).  Errors: COFEM_EINVAL, COFEM_ENOMEM,
 * COFEM_EDEVICE.
 */
cofem_status cofem_server_create(size_t hbm_budget, int32_t max_slots, int32_t steps_per_tick, void* stream,
                                 cofem_server** out);
void cofem_server_destroy(cofem_server* s);

/*
 * Queue one fit.  p as for cofem_create (serving restrictions above).  phi: HOST
 * pointer to the N x D row-major FP32 dictionary; y: HOST pointer to N floats.  The
 * caller keeps phi and y alive and unchanged until cofem_server_poll reports the
 * request RUNNING or DONE (they are copied to the device at admission).
 * *id receives the request id.  Errors: COFEM_EINVAL (bad parameters or
 * arguments), COFEM_EBUDGET (the request's workspace exceeds the whole budget).
 */
cofem_status cofem_server_submit(cofem_server* s, const cofem_params* p, const float* phi, const float* y,
                                 int64_t* id);

/*
 * One scheduling tick: admit what fits, launch one tick of every running fit, then
 * collect the fits that the previous tick finished.  Ticks are pipelined: the call
 * returns while the tick it launched may still run (it waits for the previous one), so
 * a finished fit becomes DONE one call after the tick that finished it; a call with
 * nothing running collects the last tick.  n_running and n_pending (may be NULL)
 * receive the counts after the call.
 */
cofem_status cofem_server_step(cofem_server* s, int32_t* n_running, int32_t* n_pending);

/*
 * State of request `id`; when DONE, copies mu, s, alpha (HOST buffers of D floats,
 * any may be NULL) and releases the request's record on the first call that passes
 * a non-NULL mu.  info (host, may be NULL) receives the state and time stamps.
 * Errors: COFEM_EINVAL (unknown id).
 */
cofem_status cofem_server_poll(cofem_server* s, int64_t id, float* mu, float* s_out, float* alpha,
                               cofem_request_info* info);

/*
 * Withdraw request `id`: a pending request leaves the queue; a running one stops (its
 * slot and workspace bytes are free for the next admission at once); a finished one's
 * results are discarded.  The id is unknown afterwards.  Other requests are not
 * affected (their results stay bitwise the same).  Errors: COFEM_EINVAL (unknown id).
 */
cofem_status cofem_server_cancel(cofem_server* s, int64_t id);

/* Counters of the server (host struct). */
cofem_status cofem_server_get_stats(cofem_server* s, cofem_server_stats* out);

#ifdef __cplusplus
}
#endif
#endif /* COFEM_H */
