"""GPU checks at the full size of the benchmark workload (N=16384, D=65536, K=32, T=30,
tol 1e-5, probe seed 2024).

* The operator against the oracle on sampled output coordinates it computes one by
  one (Psi_j = beta Phi_:j^T (Phi P) + alpha_j P_j).
* Both fits of the benchmark, all-FP32 and bf16 with the last 3 EM iterations on the
  FP32 dictionary, against the stored FP64 oracle fit of the same problem
  (tests/golden/make_reference.py large): mu within 1e-4 (FP32) or the stated bf16
  bound, s within 1e-3 or its bf16 bound, and the GPU/oracle ratio of CG steps.
* diag(Sigma) independently of the E-step's solves: for 64 sampled coordinates the
  stored golden holds c_j = A^{-1} e_j at alpha^(T) (FP64 PCG to 1e-11), hence the value
  the diagonal estimate of Eq. (diag-estimate) takes with the last E-step's probes when
  every solve is exact, (1/K) sum_k p_kj (c_j . p_k), and Sigma_jj itself with the spread
  of the Rademacher estimate (Lemma 1).  The GPU's s at those coordinates is compared
  with the first; the second bounds how far any K-probe estimate can sit from Sigma_jj.
* The benchmark fit's true FP64 residual and recovery (properties at any size).
The contexts are created exactly as bench.py creates them.
"""
import os

import numpy as np
import pytest

import workloads
from bars import BF16_REFINED_MU, BF16_REFINED_S, check

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "large_oracle.npz")

pytestmark = pytest.mark.gpu

CHUNK = 1024


def _bf16_rne(x):
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF
    return (r << 16).astype(np.uint32).view(np.float32)


def _matmul64(phi32, P64):
    """Phi @ P in FP64, widening row blocks of the FP32 dictionary."""
    out = np.empty((phi32.shape[0], P64.shape[1]))
    for r in range(0, phi32.shape[0], CHUNK):
        out[r:r + CHUNK] = phi32[r:r + CHUNK].astype(np.float64) @ P64
    return out


def _rmatmul64(phi32, V64):
    out = np.zeros((phi32.shape[1], V64.shape[1]))
    for r in range(0, phi32.shape[0], CHUNK):
        out += phi32[r:r + CHUNK].astype(np.float64).T @ V64[r:r + CHUNK]
    return out


@pytest.fixture(scope="module")
def large():
    import torch

    prob = workloads.make_workload("large")
    print(f"large workload N={prob.N} D={prob.D} generated", flush=True)
    return prob, torch.from_numpy(prob.phi).cuda(), torch.from_numpy(prob.y).cuda()


@pytest.mark.parametrize("dtype", ["bf16", "fp32"])
def test_large_operator_sampled(gpu, large, dtype):
    import torch

    prob, phi_d, _ = large
    w = workloads.WORKLOADS["large"]
    rng = np.random.default_rng(11)
    Q = w["K"] + 1
    P = rng.standard_normal((Q, prob.D)).astype(np.float32)
    alpha = np.exp(rng.uniform(-3, 12, prob.D)).astype(np.float32)
    m = gpu.CoFEM(prob.N, prob.D, prob.beta, K=w["K"], T=w["T"], U=w["U"], tol=w["tol"], phi_dtype=dtype)
    m.set_dictionary(phi_d)
    Psi = m.apply_A(torch.from_numpy(alpha).cuda(), torch.from_numpy(P).cuda(), use_bf16=(dtype == "bf16"))
    Psi = Psi.cpu().numpy().astype(np.float64)
    m.close()
    phi = _bf16_rne(prob.phi) if dtype == "bf16" else prob.phi
    P64 = P.T.astype(np.float64)
    V = _matmul64(phi, P64)                                   # N x Q
    js = np.sort(rng.choice(prob.D, 64, replace=False))
    cols = phi[:, js].astype(np.float64)                      # N x 64
    ref = prob.beta * (cols.T @ V) + alpha[js, None].astype(np.float64) * P64[js]   # 64 x Q
    got = Psi[:, js].T
    # per sampled coordinate, error relative to the size of the terms that were summed
    scale = prob.beta * (np.abs(cols).T @ np.abs(V)) + np.abs(alpha[js, None] * P64[js])
    err = np.abs(got - ref) / scale
    tol = 1e-5 if dtype == "fp32" else 1e-4
    check(f"large_operator/{dtype}", err.max(), tol)


def _bench_fit(gpu, prob, phi_d, y_d, form):
    w = workloads.WORKLOADS["large"]
    kw = dict(phi_dtype="bf16", refine_last=3) if form == "bf16_refined" else dict(phi_dtype="fp32")
    m = gpu.CoFEM(prob.N, prob.D, prob.beta, K=w["K"], T=w["T"], U=w["U"], tol=w["tol"], seed=2024, **kw)
    m.set_dictionary(phi_d)
    m.fit(y_d)
    mu, s, alpha, st = m.posterior()
    m.close()
    return (mu.cpu().numpy().astype(np.float64), s.cpu().numpy().astype(np.float64),
            alpha.cpu().numpy().astype(np.float64), st)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("form", ["fp32", "bf16_refined"])
def test_large_fit_matches_stored_oracle(gpu, large, form):
    prob, phi_d, y_d = large
    if not os.path.exists(GOLDEN):
        pytest.fail(f"{GOLDEN} is missing: python tests/golden/make_reference.py large")
    g = np.load(GOLDEN)
    assert int(g["seed"]) == 2024
    mu, s, alpha, st = _bench_fit(gpu, prob, phi_d, y_d, form)
    steps, steps_or = st["total_cg_steps"], int(g["cg_steps"].sum())
    sup = np.abs(g["mu"]) > 1e-3 * np.abs(g["mu"]).max()
    print(f"large {form}: CG steps gpu {steps} oracle {steps_or} (ratio {steps / steps_or:.3f}); "
          f"support mu rel {_rel(mu[sup], g['mu'][sup]):.2e}, NRMSE gpu {_rel(mu, prob.z):.4f} "
          f"oracle {_rel(g['mu'], prob.z):.4f}")
    bar_mu, bar_s = (1e-4, 1e-3) if form == "fp32" else (BF16_REFINED_MU, BF16_REFINED_S)
    check(f"large_{form}/mu", _rel(mu, g["mu"]), bar_mu)
    check(f"large_{form}/s", _rel(s, g["s"]), bar_s)
    # the last M-step's denominators on the support, 1 / alpha_j = mu_j^2 + s_j (Eq. mstep,
    # from E-step T - 1): their error is at most that of mu^2 plus that of s
    check(f"large_{form}/mstep_denominator_support", _rel(1.0 / alpha[sup], 1.0 / g["alpha"][sup]),
          2 * bar_mu + bar_s)
    check(f"large_{form}/cg_step_ratio_minus_1", abs(steps / steps_or - 1.0), 0.05)
    # diag(Sigma) at the sampled coordinates, independent of the E-step's CG solves
    js, s_exact, sjj = g["js"], g["s_exact_probes"], g["sigma_jj"]
    spread = np.sqrt(g["sigma_offdiag_sq"] / 32.0)           # Lemma 1: std of the K = 32 estimate
    check(f"large_{form}/s_sampled_vs_exact_solves", _rel(s[js], s_exact), 10 * bar_s)
    z = (s[js] - sjj) / spread
    print(f"large {form}: s_j - Sigma_jj over the Lemma 1 spread at 64 coordinates: max |z| "
          f"{np.abs(z).max():.2f}, oracle's own {np.abs((g['s'][js] - sjj) / spread).max():.2f}")
    assert np.abs(z).max() < 5


def test_large_bench_fit_properties(gpu, large):
    prob, phi_d, y_d = large
    w = workloads.WORKLOADS["large"]
    m = gpu.CoFEM(prob.N, prob.D, prob.beta, K=w["K"], T=w["T"], U=w["U"], tol=w["tol"], seed=2024,
                  phi_dtype="bf16", refine_last=3)
    m.set_dictionary(phi_d)
    m.fit(y_d)
    mu, s, alpha, st = m.posterior()
    m.close()
    mu = mu.cpu().numpy().astype(np.float64)
    alpha = alpha.cpu().numpy().astype(np.float64)
    s = s.cpu().numpy().astype(np.float64)
    print(f"bench fit: CG steps per EM iteration {st['cg_steps']}", flush=True)
    assert st["used_bf16"] == [1] * (w["T"] - 3) + [0] * 3
    assert np.isfinite(mu).all() and np.isfinite(s).all() and np.isfinite(alpha).all()
    # Algorithm 1 returns alpha^(T), the alpha of the last E-step (no M-step at t = T), and
    # that E-step used the FP32 dictionary: mu solves (beta Phi^T Phi + diag(alpha)) mu = b.
    # The joint stop rule bounds the recursive residual by tol * ||B||_F (~ tol * ||b|| here);
    # FP32 rounding lets the true residual drift from it by a small factor (measured 0.96 tol).
    b = prob.beta * _rmatmul64(prob.phi, prob.y.astype(np.float64)[:, None])[:, 0]
    Amu = prob.beta * _rmatmul64(prob.phi, _matmul64(prob.phi, mu[:, None]))[:, 0] + alpha * mu
    true_res = np.linalg.norm(b - Amu) / np.linalg.norm(b)
    nrmse = np.linalg.norm(mu - prob.z) / np.linalg.norm(prob.z)
    check("large_bench_fit/true_residual", true_res, 3 * w["tol"])
    # end-to-end recovery (sanity, not parity).  The paper reports below 2 % after 30 EM
    # iterations for its dense Gaussian setting (Uniform(-2, 2) spikes); this workload's
    # N(0, 1) spikes include amplitudes near the noise floor (measured 2.27 %).
    check("large_bench_fit/nrmse", nrmse, 0.025)
