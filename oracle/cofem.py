"""Plain float64 CPU implementation of covariance-free EM (CoFEM).

TEST INFRASTRUCTURE ONLY (see the package docstring): the GPU library never
imports or runs this module.

Contents, each restating one passage of the paper (Lin, Song, Bilgic, Ba,
"Covariance-Free Sparse Bayesian Learning", arXiv:2105.10439):

* probe generator: Rademacher probes (Sec. III-A, the +-1 form of the diagonal
  estimation rule) drawn from a counter-based SplitMix64 hash, because the
  paper does not fix a random number generator;
* `pcg`: the multi-right-hand-side preconditioned conjugate gradient of
  Algorithm 2 (Sec. III-B/C), in the standard preconditioned form (see the
  reading noted in its docstring);
* `cofem`: Algorithm 1 (Sec. III) with the diagonal estimate of Eq.
  (diag-estimate) and the M-step of Eq. (mstep);
* `exact_em`: the covariance-based EM of Sec. II-B, Eqs. (estep-params) and
  (mstep), used as the reference that CoFEM approximates;
* `log_evidence`, `woodbury_sigma`: the objective of Eq. (mle2) and the
  Woodbury form of Eq. (woodbury), used only to pin `exact_em`;
* `cofem_multitask`, `nonneg_second_moment`: the extensions of Sec. III-E;
* `posterior_variance`: the post-fit estimate of diag(Sigma) at a fixed alpha
  with many probes (the variance maps of the MRI appendix);
* `DenseOperator`, `ConvOperator`, `DctOperator` (with `dct_matrix`): the three
  dictionaries of Sec. V-A.

Parity status: every function here is pinned by a test against something
other than itself (closed forms, exact EM, library solvers, invariants,
published SplitMix64 outputs); see tests/test_oracle_*.py.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
# generators", OOPSLA 2014).  State advances by the golden gamma; each output
# is the state passed through a 64-bit finaliser (shift-xor, multiply,
# shift-xor, multiply, shift-xor).
# ---------------------------------------------------------------------------
GOLDEN_GAMMA = 0x9E3779B97F4A7C15
_MIX_MUL1 = 0xBF58476D1CE4E5B9
_MIX_MUL2 = 0x94D049BB133111EB
_MASK64 = (1 << 64) - 1


def _mix64_int(z: int) -> int:
    z &= _MASK64
    z = ((z ^ (z >> 30)) * _MIX_MUL1) & _MASK64
    z = ((z ^ (z >> 27)) * _MIX_MUL2) & _MASK64
    return z ^ (z >> 31)


def splitmix64_outputs(seed: int, n: int) -> list[int]:
    """First n outputs of the SplitMix64 stream whose state starts at `seed`.

    Output i (i = 1, 2, ...) is the finaliser applied to seed + i * gamma.
    """
    return [_mix64_int(int(seed) + (i + 1) * GOLDEN_GAMMA) for i in range(int(n))]


def mix64(z: np.ndarray) -> np.ndarray:
    """The SplitMix64 finaliser on a uint64 array (arithmetic mod 2^64)."""
    z = np.asarray(z, dtype=np.uint64).copy()
    z ^= z >> np.uint64(30)
    z *= np.uint64(_MIX_MUL1)
    z ^= z >> np.uint64(27)
    z *= np.uint64(_MIX_MUL2)
    z ^= z >> np.uint64(31)
    return z


def probe_words(seed: int, t: int, D: int) -> np.ndarray:
    """64 random bits per coordinate j = 0..D-1 for EM iteration t (t >= 1).

    The iteration key is output t of the SplitMix64 stream started at `seed`;
    word j is output j + 1 of the stream started at that key.  Bit k of word j
    gives probe entry p_{k,j}, so probe sets are nested in K and every draw is
    a pure function of (seed, t, j).
    """
    key = _mix64_int(int(seed) + int(t) * GOLDEN_GAMMA)
    j = np.arange(1, int(D) + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        ctr = np.uint64(key) + j * np.uint64(GOLDEN_GAMMA)
    return mix64(ctr)


def rademacher_probes(seed: int, t: int, D: int, K: int) -> np.ndarray:
    """D x K matrix of Rademacher probes (Sec. III-A): +1 where bit k is 0, -1 where it is 1."""
    if not 1 <= K <= 64:
        raise ValueError("K must be in [1, 64]")
    w = probe_words(seed, t, D)
    bits = (w[:, None] >> np.arange(K, dtype=np.uint64)[None, :]) & np.uint64(1)
    return 1.0 - 2.0 * bits.astype(np.float64)


def hadamard_probes(D: int) -> np.ndarray:
    """The D x D Sylvester-Hadamard matrix (D a power of two), as K = D probes.

    With these probes the cross terms of Eq. (diag-expansion) cancel exactly,
    because distinct rows of a Hadamard matrix are orthogonal.
    """
    if D < 1 or D & (D - 1):
        raise ValueError("D must be a power of two")
    H = np.ones((1, 1))
    while H.shape[0] < D:
        H = np.block([[H, H], [H, -H]])
    return H


# ---------------------------------------------------------------------------
# Dictionaries.  The method only needs v -> Phi v and u -> Phi^T u
# (Sec. III-B: the cost of CG is the cost of applying Phi and its transpose).
# ---------------------------------------------------------------------------
class DenseOperator:
    """A dense N x D dictionary held in float64 (Eq. sparse-coding)."""

    def __init__(self, phi: np.ndarray):
        self.phi = np.asarray(phi, dtype=np.float64)
        self.N, self.D = self.phi.shape

    def matvec(self, V: np.ndarray) -> np.ndarray:
        return self.phi @ V

    def rmatvec(self, Uu: np.ndarray) -> np.ndarray:
        return self.phi.T @ Uu

    def col_sq_norms(self) -> np.ndarray:
        """theta_j = sum_i Phi_ij^2, the Jacobi choice of Sec. III-C."""
        return np.einsum("ij,ij->j", self.phi, self.phi)

    def dense(self) -> np.ndarray:
        return self.phi


class ConvOperator:
    """Convolutional dictionary of Sec. V-A.2: N = D, Phi_ij = h[i - j] for 0 <= i - j < L.

    Column j is the filter delayed by j samples and truncated at the end of
    the signal, so Phi is lower-triangular Toeplitz; applying it is a causal
    FIR filter and applying its transpose is the time-reversed (anti-causal)
    filter.  Both are written as direct sums over the taps.
    """

    def __init__(self, h: np.ndarray, D: int):
        self.h = np.asarray(h, dtype=np.float64)
        self.N = self.D = int(D)

    def matvec(self, V: np.ndarray) -> np.ndarray:
        V = np.asarray(V, dtype=np.float64)
        out = np.zeros_like(V)
        for t, ht in enumerate(self.h):
            if t >= self.D:
                break
            out[t:] += ht * V[:self.D - t]
        return out

    def rmatvec(self, Uu: np.ndarray) -> np.ndarray:
        Uu = np.asarray(Uu, dtype=np.float64)
        out = np.zeros_like(Uu)
        for t, ht in enumerate(self.h):
            if t >= self.D:
                break
            out[:self.D - t] += ht * Uu[t:]
        return out

    def col_sq_norms(self) -> np.ndarray:
        L = self.h.shape[0]
        csum = np.concatenate([[0.0], np.cumsum(self.h ** 2)])
        n = np.minimum(L, self.D - np.arange(self.D))
        return csum[n]

    def dense(self) -> np.ndarray:
        Phi = np.zeros((self.D, self.D))
        for t, ht in enumerate(self.h):
            if t >= self.D:
                break
            idx = np.arange(self.D - t)
            Phi[idx + t, idx] = ht
        return Phi

    def normal_rows(self, P: np.ndarray, alpha: np.ndarray, beta: float, rows) -> np.ndarray:
        """Rows `rows` of beta Phi^T Phi P + alpha P (the operator of Algorithm 2) by
        direct sums, for sizes where whole products are too slow: row j needs
        (Phi P)_i only for j <= i < j + L, and each of those is a sum over L taps."""
        P = np.asarray(P, dtype=np.float64)
        if P.ndim == 1:
            P = P[:, None]
        L = self.h.shape[0]
        taps = np.arange(L)
        out = np.empty((len(rows), P.shape[1]))
        for r, j in enumerate(rows):
            i = np.arange(j, min(j + L, self.D))              # rows of Phi P that meet column j
            src = i[:, None] - taps[None, :]                  # (Phi P)_i = sum_s h[s] P[i - s], i - s >= 0
            w = np.where(src >= 0, self.h[None, :], 0.0)
            V = np.einsum("is,isq->iq", w, P[np.clip(src, 0, None)])
            out[r] = beta * (self.h[:i.shape[0]] @ V) + float(alpha[j]) * P[j]
        return out


def dct_matrix(D: int) -> np.ndarray:
    """The orthonormal DCT-II matrix Omega of size D, entry by entry from its
    definition: Omega_kn = s_k cos(pi (2n + 1) k / (2D)), s_0 = sqrt(1/D) and
    s_k = sqrt(2/D) for k >= 1 (rows are frequencies, columns are samples)."""
    k = np.arange(D, dtype=np.float64)[:, None]
    n = np.arange(D, dtype=np.float64)[None, :]
    s = np.full((D, 1), np.sqrt(2.0 / D))
    s[0, 0] = np.sqrt(1.0 / D)
    return s * np.cos(np.pi * (2.0 * n + 1.0) * k / (2.0 * D))


class DctOperator:
    """Subsampled DCT dictionary of Sec. V-A.1: Phi = M Omega^{-1}.

    Omega is the orthonormal 1-D DCT-II of size D (so Omega^{-1} = Omega^T, the
    DCT-III), and M keeps the N samples listed in `rows` (distinct indices in
    [0, D), in the order of the entries of y).  Phi v is the inverse DCT of v read
    at those samples; Phi^T u scatters u into a zero signal of length D and takes
    its DCT.  Both use scipy's orthonormal type-II DCT as the library step.
    """

    def __init__(self, D: int, rows):
        import scipy.fft  # local: only the DCT dictionary needs it

        self._fft = scipy.fft
        self.D = int(D)
        self.rows = np.asarray(rows, dtype=np.int64).reshape(-1)
        self.N = int(self.rows.shape[0])
        if self.N < 1 or self.rows.min() < 0 or self.rows.max() >= self.D:
            raise ValueError("rows must be indices in [0, D)")
        if np.unique(self.rows).shape[0] != self.N:
            raise ValueError("rows must be distinct")

    def matvec(self, V: np.ndarray) -> np.ndarray:
        V = np.asarray(V, dtype=np.float64)
        return self._fft.idct(V, type=2, norm="ortho", axis=0)[self.rows]

    def rmatvec(self, Uu: np.ndarray) -> np.ndarray:
        Uu = np.asarray(Uu, dtype=np.float64)
        full = np.zeros((self.D,) + Uu.shape[1:])
        full[self.rows] = Uu
        return self._fft.dct(full, type=2, norm="ortho", axis=0)

    def col_sq_norms(self) -> np.ndarray:
        """theta_j = sum_i Omega_{j, rows_i}^2, summed over the kept samples in row blocks."""
        out = np.empty(self.D)
        n = self.rows.astype(np.float64)[None, :]
        for j0 in range(0, self.D, 256):
            k = np.arange(j0, min(j0 + 256, self.D), dtype=np.float64)[:, None]
            c = np.cos(np.pi * (2.0 * n + 1.0) * k / (2.0 * self.D))
            sk2 = np.where(k[:, 0] == 0, 1.0 / self.D, 2.0 / self.D)
            out[j0:j0 + k.shape[0]] = sk2 * np.sum(c * c, axis=1)
        return out

    def dense(self) -> np.ndarray:
        return dct_matrix(self.D)[:, self.rows].T


# ---------------------------------------------------------------------------
# Algorithm 2: parallel (multi-RHS) preconditioned conjugate gradient.
# ---------------------------------------------------------------------------
@dataclass
class PCGResult:
    X: np.ndarray
    steps: int                 # number of applications of A performed
    rel_resid: float           # ||R||_F / ||B||_F after the last step
    col_rel_resid: np.ndarray  # ||R_q|| / ||B_q|| per column (nan where B_q = 0)
    converged: bool
    breakdown: np.ndarray      # bool per column: pi_q <= 0 while rho_q != 0
    history: list = field(default_factory=list)


def pcg(apply_A, B: np.ndarray, minv: np.ndarray, U: int, tol: float,
        stop_mode: str = "joint", record: bool = False) -> PCGResult:
    """Solve A X = B for all Q columns of B at once (Algorithm 2).

    apply_A maps a D x Q block to A times it; minv holds the diagonal of the
    inverse preconditioner M^{-1}.

    Reading of the printed algorithm: its initialisation sets the search
    directions to B and its last line updates them from R, which is plain CG
    and ignores M; with a non-scalar M that recursion does not converge.  The
    preconditioned system of Sec. III-C (A' = M^{-1/2} A M^{-1/2}) is solved by
    standard preconditioned CG, whose directions start at W = M^{-1} B and are
    updated from W.  That is what this function does.  Everything else (the
    per-column step sizes gamma_q = rho_q / pi_q and eta_q = rho_q / rho_q^old,
    the Frobenius stop test on the recursive residual after the X and R
    updates, X starting at zero) follows Algorithm 2 as printed.

    stop_mode "joint" is the printed test ||R||_F / ||B||_F <= tol.  stop_mode
    "column" freezes each column q once ||R_q|| / ||B_q|| <= tol and stops when
    none is left.  A column whose pi_q <= 0 (impossible in exact arithmetic
    for SPD A) or whose B_q is zero gets step size 0.
    """
    B = np.asarray(B, dtype=np.float64)
    D, Q = B.shape
    minv = np.asarray(minv, dtype=np.float64).reshape(D, 1)
    X = np.zeros_like(B)
    R = B.copy()
    W = minv * R
    P = W.copy()
    rho = np.sum(R * W, axis=0)
    bnorm = np.linalg.norm(B)
    bcol = np.linalg.norm(B, axis=0)
    active = np.ones(Q, dtype=bool)
    if stop_mode == "column":
        active &= bcol > 0
    elif stop_mode != "joint":
        raise ValueError("stop_mode must be 'joint' or 'column'")
    breakdown = np.zeros(Q, dtype=bool)
    steps = 0
    converged = False
    hist = []
    if record:
        hist.append(dict(X=X.copy(), R=R.copy(), P=P.copy()))
    for u in range(1, int(U) + 1):
        if stop_mode == "column" and not active.any():
            converged = True
            break
        Psi = apply_A(P)
        pi = np.sum(P * Psi, axis=0)
        bad = active & (pi <= 0) & (rho != 0)
        breakdown |= bad
        active &= ~bad
        ok = active & (pi > 0)
        gamma = np.zeros(Q)
        gamma[ok] = rho[ok] / pi[ok]
        X = X + P * gamma
        R = R - Psi * gamma
        steps = u
        delta = np.linalg.norm(R) / bnorm
        if stop_mode == "joint":
            if delta <= tol:
                converged = True
                if record:
                    hist.append(dict(X=X.copy(), R=R.copy(), P=P.copy()))
                break
        else:
            with np.errstate(invalid="ignore", divide="ignore"):
                cd = np.linalg.norm(R, axis=0) / bcol
            active &= ~(cd <= tol)
        W = minv * R
        rho_old = rho
        rho = np.sum(R * W, axis=0)
        eta = np.zeros(Q)
        nz = rho_old != 0
        eta[nz] = rho[nz] / rho_old[nz]
        P = W + P * eta
        if record:
            hist.append(dict(X=X.copy(), R=R.copy(), P=P.copy()))
    else:
        if stop_mode == "column" and not active.any():
            converged = True
    with np.errstate(invalid="ignore", divide="ignore"):
        col_rel = np.linalg.norm(R, axis=0) / bcol
    return PCGResult(X=X, steps=steps, rel_resid=float(np.linalg.norm(R) / bnorm),
                     col_rel_resid=col_rel, converged=converged, breakdown=breakdown, history=hist)


# ---------------------------------------------------------------------------
# Diagonal estimation rule (Prop. 1) and its Rademacher form (Eq. diag-estimate).
# ---------------------------------------------------------------------------
def diag_estimate_general(P: np.ndarray, X: np.ndarray) -> np.ndarray:
    """s_j = sum_k p_{k,j} x_{k,j} / sum_k p_{k,j}^2 (Eq. single-diag-estimator); P, X are D x K."""
    return np.sum(P * X, axis=1) / np.sum(P * P, axis=1)


def diag_estimate(P: np.ndarray, X: np.ndarray) -> np.ndarray:
    """s_j = (1/K) sum_k p_{k,j} x_{k,j} for +-1 probes (Eq. diag-estimate)."""
    return np.sum(P * X, axis=1) / P.shape[1]


# ---------------------------------------------------------------------------
# Algorithm 1: covariance-free EM.
# ---------------------------------------------------------------------------
@dataclass
class CoFEMResult:
    alpha: np.ndarray          # alpha^(T) (the last M-step's output; no M-step at t = T)
    mu: np.ndarray             # mu from the E-step of iteration T
    s: np.ndarray              # diagonal estimate from the E-step of iteration T
    cg_steps: list             # CG steps per EM iteration
    rel_resid: list            # final ||R||_F/||B||_F per EM iteration
    clamped: int               # M-step denominators raised to the floor
    breakdown: int             # columns that hit pi <= 0
    alphas: list = field(default_factory=list)   # alpha^(t) for t = 1..T when record=True


def _as_operator(op):
    if isinstance(op, (DenseOperator, ConvOperator, DctOperator)):
        return op
    return DenseOperator(op)


def cofem(op, y: np.ndarray, beta: float, T: int, K: int, U: int, tol: float, seed: int = 0,
          theta_mode: str = "ones", stop_mode: str = "joint", probes=None,
          alpha_floor: float = 1e-30, alpha0=None, record: bool = False, mstep: str = "gaussian") -> CoFEMResult:
    """Algorithm 1, CovarianceFreeEM(y, Phi, beta, T, K).

    alpha starts at 1.  Each iteration t = 1..T draws K Rademacher probes
    (fresh per t), solves A X = B with A = beta Phi^T Phi + diag(alpha) and
    B = [beta Phi^T y | p_1 .. p_K] by `pcg` with the diagonal preconditioner
    M = diag(beta theta + alpha) of Sec. III-C (theta = 1, or the Jacobi
    choice theta_j = ||Phi_:j||^2), forms mu and the diagonal estimate s, and
    for t < T sets alpha_j = 1 / (mu_j^2 + s_j).  Returns alpha^(T), mu, s.

    Column order: column 0 of B and X is the mu system, columns 1..K are the
    probes (the paper lists mu last; the order does not change any column).
    `probes`, if given, is a callable t -> D x K matrix that replaces the hash
    draw (used for Hadamard probes in tests).  mu_j^2 + s_j may come out <= 0
    because s is only unbiased; such denominators are raised to alpha_floor
    and counted.

    mstep="nonneg" is the M-step of the non-negative model (Sec. III-E.2): the
    denominator is the second moment of the rectified Gaussian posterior,
    `nonneg_second_moment(mu, s)` with s in place of Sigma_jj (the paper's own
    substitution), its variance floor being alpha_floor.
    """
    if mstep not in ("gaussian", "nonneg"):
        raise ValueError("mstep must be 'gaussian' or 'nonneg'")
    op = _as_operator(op)
    D = op.D
    y = np.asarray(y, dtype=np.float64).reshape(-1, 1)
    b = beta * op.rmatvec(y)[:, 0]
    if theta_mode == "ones":
        theta = np.ones(D)
    elif theta_mode == "jacobi":
        theta = op.col_sq_norms()
    else:
        raise ValueError("theta_mode must be 'ones' or 'jacobi'")
    alpha = np.ones(D) if alpha0 is None else np.asarray(alpha0, dtype=np.float64).copy()
    steps, resid, alphas = [], [], []
    clamped = 0
    nbreak = 0
    mu = s = None
    for t in range(1, int(T) + 1):
        if record:
            alphas.append(alpha.copy())
        Pr = probes(t) if probes is not None else rademacher_probes(seed, t, D, K)
        B = np.column_stack([b, Pr])
        minv = 1.0 / (beta * theta + alpha)
        a_t = alpha

        def apply_A(Pd, a_t=a_t):
            return beta * op.rmatvec(op.matvec(Pd)) + a_t[:, None] * Pd

        res = pcg(apply_A, B, minv, U, tol, stop_mode)
        steps.append(res.steps)
        resid.append(res.rel_resid)
        nbreak += int(res.breakdown.sum())
        mu = res.X[:, 0].copy()
        s = diag_estimate(Pr, res.X[:, 1:])
        if t < T:
            denom = mu ** 2 + s if mstep == "gaussian" else nonneg_second_moment(mu, s, alpha_floor)
            low = denom < alpha_floor
            clamped += int(low.sum())
            alpha = 1.0 / np.maximum(denom, alpha_floor)
    return CoFEMResult(alpha=alpha, mu=mu, s=s, cg_steps=steps, rel_resid=resid,
                       clamped=clamped, breakdown=nbreak, alphas=alphas)


# ---------------------------------------------------------------------------
# Covariance-based EM (Sec. II-B) and the quantities used to pin it.
# ---------------------------------------------------------------------------
def exact_em(phi: np.ndarray, y: np.ndarray, beta: float, T: int, alpha0=None, record: bool = False,
             mstep: str = "gaussian", alpha_floor: float = 1e-30):
    """EM with the explicit posterior covariance.

    E-step, Eq. (estep-params): Sigma = (beta Phi^T Phi + diag(alpha))^{-1},
    mu = beta Sigma Phi^T y.  M-step, Eq. (mstep): alpha_j = 1 / (mu_j^2 +
    Sigma_jj), done for t < T to match the iteration count of Algorithm 1.
    mstep="nonneg": alpha_j = 1 / max(E[z_j^2], alpha_floor) with the second moment
    of the rectified Gaussian posterior, Eq. (nonneg-sbl), from the exact Sigma_jj.
    Returns (alpha^(T), mu, diag(Sigma), list of alpha^(t)).
    """
    phi = np.asarray(phi, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    D = phi.shape[1]
    G = phi.T @ phi
    c = phi.T @ y
    alpha = np.ones(D) if alpha0 is None else np.asarray(alpha0, dtype=np.float64).copy()
    alphas = []
    mu = dSig = None
    for t in range(1, int(T) + 1):
        if record:
            alphas.append(alpha.copy())
        A = beta * G + np.diag(alpha)
        Sigma = np.linalg.inv(A)
        Sigma = 0.5 * (Sigma + Sigma.T)
        mu = beta * Sigma @ c
        dSig = np.diag(Sigma).copy()
        if t < T:
            if mstep == "gaussian":
                alpha = 1.0 / (mu ** 2 + dSig)
            else:
                alpha = 1.0 / np.maximum(nonneg_second_moment(mu, dSig, alpha_floor), alpha_floor)
    return alpha, mu, dSig, alphas


def log_evidence(phi: np.ndarray, y: np.ndarray, beta: float, alpha: np.ndarray) -> float:
    """log p(y | alpha) of Eq. (mle2).

    Integrating z out of the model of Eq. (model) gives y ~ N(0, C) with
    C = beta^{-1} I + Phi diag(alpha)^{-1} Phi^T.
    """
    phi = np.asarray(phi, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    N = phi.shape[0]
    C = np.eye(N) / beta + (phi / alpha[None, :]) @ phi.T
    sign, logdet = np.linalg.slogdet(C)
    return float(-0.5 * (N * np.log(2 * np.pi) + logdet + y @ np.linalg.solve(C, y)))


def woodbury_sigma(phi: np.ndarray, beta: float, alpha: np.ndarray) -> np.ndarray:
    """Sigma by the Woodbury identity (Eq. woodbury), with the noise precision kept.

    Sigma = C - C Phi^T (beta^{-1} I + Phi C Phi^T)^{-1} Phi C, C = diag(alpha)^{-1}.
    (The printed identity shows I in place of beta^{-1} I, which is only right
    for beta = 1; the inverse of beta Phi^T Phi + diag(alpha) needs beta^{-1}.)
    """
    phi = np.asarray(phi, dtype=np.float64)
    N = phi.shape[0]
    Cd = 1.0 / np.asarray(alpha, dtype=np.float64)
    PC = phi * Cd[None, :]
    inner = np.eye(N) / beta + PC @ phi.T
    return np.diag(Cd) - PC.T @ np.linalg.solve(inner, PC)


# ---------------------------------------------------------------------------
# Extensions of Sec. III-E.
# ---------------------------------------------------------------------------
def nonneg_second_moment(mu: np.ndarray, var: np.ndarray, var_floor: float = 1e-30) -> np.ndarray:
    """Second moment of the rectified (zero-truncated) Gaussian posterior, Eq. (nonneg-sbl).

    E[z^2] = mu^2 + v + mu * sqrt(2 v / pi) * exp(-xi^2) / erfc(-xi), xi = mu / sqrt(2 v),
    with v the posterior variance (replaced by the estimate s in CoFEM).

    Reading: the printed formula has sqrt(v / pi); the second moment of a
    Gaussian N(mu, v) truncated to z > 0 (the rectified Gaussian defined in the
    same section) carries sqrt(2 v / pi), which is what is computed here and
    what the tests pin by numerical integration.  exp(-xi^2)/erfc(-xi) is
    evaluated as 1/erfcx(-xi), the same quantity without under/overflow.  v is
    raised to var_floor first, since s can come out non-positive.
    """
    from scipy.special import erfcx

    mu = np.asarray(mu, dtype=np.float64)
    v = np.maximum(np.asarray(var, dtype=np.float64), var_floor)
    xi = mu / np.sqrt(2.0 * v)
    return mu ** 2 + v + mu * np.sqrt(2.0 * v / np.pi) / erfcx(-xi)


def cofem_multitask(ops, ys, beta: float, T: int, K: int, U: int, tol: float, seed: int = 0,
                    theta_mode: str = "ones", stop_mode: str = "joint", alpha_floor: float = 1e-30):
    """Multi-task CoFEM (Sec. III-E.1): L problems sharing one alpha.

    Every task l runs the covariance-free E-step of Algorithm 1 with its own
    dictionary, data and probes (seed + l), and the M-step combines them as
    alpha_j = L / sum_l (mu_{l,j}^2 + s_{l,j}).  With L = 1 this is `cofem`.
    Returns (alpha^(T), list of mu_l, list of s_l, CG steps per (t, l)).
    """
    ops = [_as_operator(o) for o in ops]
    L = len(ops)
    D = ops[0].D
    bs, thetas = [], []
    for op, y in zip(ops, ys):
        bs.append(beta * op.rmatvec(np.asarray(y, dtype=np.float64).reshape(-1, 1))[:, 0])
        thetas.append(np.ones(D) if theta_mode == "ones" else op.col_sq_norms())
    alpha = np.ones(D)
    mus, ss, steps = [None] * L, [None] * L, []
    for t in range(1, int(T) + 1):
        acc = np.zeros(D)
        row = []
        for l, op in enumerate(ops):
            Pr = rademacher_probes(seed + l, t, D, K)
            B = np.column_stack([bs[l], Pr])
            minv = 1.0 / (beta * thetas[l] + alpha)
            a_t = alpha

            def apply_A(Pd, op=op, a_t=a_t):
                return beta * op.rmatvec(op.matvec(Pd)) + a_t[:, None] * Pd

            res = pcg(apply_A, B, minv, U, tol, stop_mode)
            row.append(res.steps)
            mus[l] = res.X[:, 0].copy()
            ss[l] = diag_estimate(Pr, res.X[:, 1:])
            acc += mus[l] ** 2 + ss[l]
        steps.append(row)
        if t < T:
            alpha = 1.0 / np.maximum(acc / L, alpha_floor)
    return alpha, mus, ss, steps


def posterior_variance(op, y: np.ndarray, beta: float, alpha: np.ndarray, K: int, batches: int, U: int,
                       tol: float, seed: int = 0, theta_mode: str = "ones", stop_mode: str = "joint",
                       probes=None):
    """Post-fit estimate of diag(Sigma) at a given alpha (the variance maps of the
    MRI appendix, with the identity in place of the image-domain map E).

    Sigma = (beta Phi^T Phi + diag(alpha))^{-1}.  Batch b = 1..batches draws K
    fresh Rademacher probes (the probe words of iteration key b of the stream
    started at `seed`, as in Algorithm 1), solves A X = [beta Phi^T y | probes] by
    `pcg` with the preconditioner of Sec. III-C, and forms the diagonal estimate
    of Eq. (diag-estimate); the result is the mean over the batches, i.e. the
    estimate from K * batches probes.  Returns (s, mu, CG steps per batch), mu
    being the mean of the last batch (every batch solves the same mu system).
    `probes`, if given, is a callable b -> D x K matrix replacing the hash draw.
    """
    op = _as_operator(op)
    D = op.D
    alpha = np.asarray(alpha, dtype=np.float64).reshape(-1)
    b = beta * op.rmatvec(np.asarray(y, dtype=np.float64).reshape(-1, 1))[:, 0]
    theta = np.ones(D) if theta_mode == "ones" else op.col_sq_norms()
    minv = 1.0 / (beta * theta + alpha)

    def apply_A(Pd):
        return beta * op.rmatvec(op.matvec(Pd)) + alpha[:, None] * Pd

    acc = np.zeros(D)
    steps = []
    mu = None
    for bi in range(1, int(batches) + 1):
        Pr = rademacher_probes(seed, bi, D, K) if probes is None else np.asarray(probes(bi), dtype=np.float64)
        res = pcg(apply_A, np.column_stack([b, Pr]), minv, U, tol, stop_mode)
        steps.append(res.steps)
        acc += diag_estimate(Pr, res.X[:, 1:])
        mu = res.X[:, 0].copy()
    return acc / int(batches), mu, steps
