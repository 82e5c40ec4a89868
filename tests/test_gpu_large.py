"""GPU checks at the full size of the benchmark workload (N=16384, D=65536, K=32).

A complete FP64 oracle fit at this size takes about an hour on the host, so:
  * the operator is compared with the oracle on sampled output coordinates it
    computes one by one (Psi_j = beta Phi_:j^T (Phi P) + alpha_j P_j);
  * the benchmark's own fit (bf16 dictionary, last 3 EM iterations FP32) is
    checked by properties that hold at any size: the true FP64 residual of its
    mu column, and the end-to-end recovery (NRMSE) that the paper reports for
    dense Gaussian dictionaries after 30 EM iterations (below 2 %).
The contexts are created exactly as bench.py creates them.
"""
import numpy as np
import pytest

import workloads

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
    print(f"{dtype}: max scaled error {err.max():.2e}")
    assert err.max() < tol


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
    print(f"bench fit: CG steps per EM iteration {st['cg_steps']}")
    assert st["used_bf16"] == [1] * (w["T"] - 3) + [0] * 3
    assert np.isfinite(mu).all() and np.isfinite(s).all() and np.isfinite(alpha).all()
    # Algorithm 1 returns alpha^(T), the alpha of the last E-step (no M-step at t = T), and
    # that E-step used the FP32 dictionary: mu solves (beta Phi^T Phi + diag(alpha)) mu = b.
    # The joint stop rule bounds the recursive residual by tol * ||B||_F (~ tol * ||b|| here);
    # FP32 rounding lets the true residual drift above it by a modest factor.
    b = prob.beta * _rmatmul64(prob.phi, prob.y.astype(np.float64)[:, None])[:, 0]
    Amu = prob.beta * _rmatmul64(prob.phi, _matmul64(prob.phi, mu[:, None]))[:, 0] + alpha * mu
    true_res = np.linalg.norm(b - Amu) / np.linalg.norm(b)
    nrmse = np.linalg.norm(mu - prob.z) / np.linalg.norm(prob.z)
    print(f"true residual of mu {true_res:.2e} (tol {w['tol']:.0e}), NRMSE {100 * nrmse:.2f}%")
    assert true_res < 100 * w["tol"]
    # end-to-end recovery (sanity, not parity).  The paper reports below 2 % after 30 EM
    # iterations for its dense Gaussian setting (Uniform(-2, 2) spikes); this workload's
    # N(0, 1) spikes include amplitudes near the noise floor, so the bound is looser.
    assert nrmse < 0.05
