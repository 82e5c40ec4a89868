"""Write stored oracle results used by the GPU parity tests.

Calls only the FP64 oracle and the seeded input generators, never the GPU
library.  Usage (from the repository root):

    python tests/golden/make_reference.py medium
    python tests/golden/make_reference.py large      # about an hour on 8 cores, 14 GB
    python tests/golden/make_reference.py conv16     # the FIR shape at D = 2^16

medium: the N=2048, D=8192 dense Gaussian workload (5% spikes, sigma=0.01,
K=20, T=50, tol=1e-5, U=400), probe seed 77, theta=1, joint stop rule.  The
oracle needs about a minute and a half on 8 cores, too long for a test, so its
mu, s, alpha^(T) and CG step counts are stored in medium_oracle.npz.

large: the N=16384, D=65536 benchmark workload (2% spikes, sigma=0.01, K=32,
T=30, tol=1e-5, U=400), probe seed 2024, theta=1, joint stop rule, the FP32
dictionary widened to FP64.  Besides mu, s, alpha^(T) and the CG steps, it
stores a probe-independent check of the diagonal estimate: for 64 sampled
coordinates j (32 on the support of z, 32 off it) the column c_j = A^{-1} e_j of
Sigma at alpha^(T) (A = beta Phi^T Phi + diag(alpha^(T)), the matrix of the last
E-step), solved by FP64 PCG to a relative residual of 1e-11 per column.  From
c_j it keeps Sigma_jj = c_j[j], the spread of the Rademacher estimate (Lemma 1:
Var(s_j) = (1/K) sum_{i != j} Sigma_ij^2), and the value the estimate of Eq.
(diag-estimate) takes with the probes of iteration T when every solve is exact,
(1/K) sum_k p_kj (c_j . p_k), since x_k[j] = e_j^T A^{-1} p_k = c_j . p_k.
mu_exact is A^{-1} b solved to the same precision.

conv16: the FIR workload's shape (causal filter exp(-t/50) with 256 taps,
Bernoulli(0.01) Exp(1) spikes, sigma = 0.05, K = 20, theta = 1) at D = 2^16 with
T = 5 EM iterations, probe seed 2024: every tile count and the full-length filter
runs of the D = 2^20 workload, at a size the direct-sum oracle finishes in under an
hour and a quarter.  It runs at tol 1e-8 with U = 600 instead of the workload's
1e-5 / 400: A is ill-conditioned on this dictionary (beta (sum h)^2 ~ 1e6 against
alpha ~ 1), and at 1e-5 the oracle's own mu still moves by more than the 1e-4 parity
bar with the tolerance.  The first E-step (alpha = 1) stops at U = 600 with a
residual ratio of 1.7e-7; the other four meet 1e-8.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
SEED = {"medium": 77, "large": 2024, "conv16": 2024}
CONV16 = dict(D=1 << 16, T=5, tol=1e-8, U=600)
LARGE_SAMPLES = 64
EXACT_TOL = 1e-11


def medium():
    w = workloads.WORKLOADS["medium"]
    prob = workloads.make_workload("medium")
    t0 = time.time()
    r = oracle.cofem(prob.phi, prob.y, prob.beta, T=w["T"], K=w["K"], U=w["U"], tol=w["tol"], seed=SEED["medium"])
    print(f"oracle medium: {time.time() - t0:.1f}s, CG steps {sum(r.cg_steps)}")
    np.savez_compressed(os.path.join(HERE, "medium_oracle.npz"), mu=r.mu, s=r.s, alpha=r.alpha,
                        cg_steps=np.array(r.cg_steps), rel_resid=np.array(r.rel_resid), seed=SEED["medium"])


def sampled_coordinates(z: np.ndarray, n: int, seed: int) -> np.ndarray:
    """n/2 coordinates on the support of z and n/2 off it, sorted (seeded)."""
    rng = np.random.default_rng(seed)
    on = np.flatnonzero(z)
    off = np.flatnonzero(z == 0)
    js = np.concatenate([rng.choice(on, n // 2, replace=False), rng.choice(off, n - n // 2, replace=False)])
    return np.sort(js)


def exact_columns(op, beta: float, alpha: np.ndarray, b: np.ndarray, js: np.ndarray, U: int):
    """[A^{-1} b | A^{-1} e_j for j in js] by FP64 PCG, each column to EXACT_TOL."""
    D = op.D
    E = np.zeros((D, 1 + len(js)))
    E[:, 0] = b
    E[js, 1 + np.arange(len(js))] = 1.0
    minv = 1.0 / (beta + alpha)

    def apply_A(Pd):
        return beta * op.rmatvec(op.matvec(Pd)) + alpha[:, None] * Pd

    res = oracle.pcg(apply_A, E, minv, U, EXACT_TOL, stop_mode="column")
    return res


def large():
    w = workloads.WORKLOADS["large"]
    seed = SEED["large"]
    prob = workloads.make_workload("large")
    op = oracle.DenseOperator(prob.phi)
    prob.phi = None
    t0 = time.time()
    r = oracle.cofem(op, prob.y, prob.beta, T=w["T"], K=w["K"], U=w["U"], tol=w["tol"], seed=seed)
    t_fit = time.time() - t0
    print(f"oracle large: {t_fit:.1f}s, CG steps {r.cg_steps} (total {sum(r.cg_steps)})", flush=True)
    js = sampled_coordinates(prob.z, LARGE_SAMPLES, seed=31)
    b = prob.beta * op.rmatvec(prob.y.astype(np.float64)[:, None])[:, 0]
    t1 = time.time()
    ex = exact_columns(op, prob.beta, r.alpha, b, js, U=4000)
    print(f"exact columns: {time.time() - t1:.1f}s, {ex.steps} CG steps, converged {ex.converged}, "
          f"worst column residual {np.nanmax(ex.col_rel_resid):.1e}", flush=True)
    C = ex.X[:, 1:]
    k = np.arange(len(js))
    sigma_jj = C[js, k]
    off_sq = np.sum(C * C, axis=0) - sigma_jj ** 2
    Pr = oracle.rademacher_probes(seed, w["T"], op.D, w["K"])       # probes of the last E-step
    s_exact_probes = np.array([np.mean(Pr[j] * (C[:, i] @ Pr)) for i, j in enumerate(js)])
    np.savez_compressed(os.path.join(HERE, "large_oracle.npz"), mu=r.mu, s=r.s, alpha=r.alpha,
                        cg_steps=np.array(r.cg_steps), rel_resid=np.array(r.rel_resid), seed=seed,
                        clamped=r.clamped, breakdown=r.breakdown, fit_seconds=t_fit,
                        js=js, sigma_jj=sigma_jj, sigma_offdiag_sq=off_sq, s_exact_probes=s_exact_probes,
                        mu_exact=ex.X[:, 0], exact_col_rel_resid=ex.col_rel_resid, exact_steps=ex.steps)


def conv16():
    w = dict(workloads.WORKLOADS["conv"])
    w.update(CONV16)
    seed = SEED["conv16"]
    prob = workloads.make_workload("conv", D=w["D"])
    op = oracle.ConvOperator(prob.h, prob.D)
    t0 = time.time()
    r = oracle.cofem(op, prob.y, prob.beta, T=w["T"], K=w["K"], U=w["U"], tol=w["tol"], seed=seed)
    t_fit = time.time() - t0
    print(f"oracle conv16: {t_fit:.1f}s, CG steps {r.cg_steps} (total {sum(r.cg_steps)})", flush=True)
    np.savez_compressed(os.path.join(HERE, "conv16_oracle.npz"), mu=r.mu, s=r.s, alpha=r.alpha,
                        cg_steps=np.array(r.cg_steps), rel_resid=np.array(r.rel_resid), seed=seed,
                        clamped=r.clamped, breakdown=r.breakdown, fit_seconds=t_fit, D=w["D"], T=w["T"],
                        tol=w["tol"], U=w["U"])


if __name__ == "__main__":
    for name in sys.argv[1:] or ["medium"]:
        globals()[name]()
