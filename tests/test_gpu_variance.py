"""GPU parity of the post-fit posterior variance (cofem_variance): diag(Sigma) at a
fixed alpha, Sigma = (beta Phi^T Phi + diag(alpha))^{-1}, from K * batches probes.

* Against `oracle.posterior_variance` at the same alpha (the oracle's own fitted
  alpha, rounded to FP32, so that CG converges as it does after a fit), probes,
  stop rule and tolerance 1e-8 (where the oracle's own answer moves by far less than
  the bar with the tolerance), on the dense, convolutional and DCT dictionaries: s
  within 1e-4; mu within 1e-4 or 4 kappa 2^-24, whichever is larger (alpha after 8
  EM iterations leaves the mu system with kappa up to 2.4e4, and an FP32 CG solve is
  good to about kappa 2^-24 there; fits run to convergence have far smaller kappa).
* Against the exact diag(Sigma) from the explicit inverse: the error of the GPU
  estimate falls as the probe count grows (Lemma 1: ~ 1 / sqrt(K * batches)).
* alpha = NULL means the fit's alpha^(T): the same result as passing it, bitwise;
  the fit's posterior is left untouched; bad arguments are rejected.
"""
import ctypes

import numpy as np
import pytest

import oracle
import workloads
from bars import binds, check, fp32_solve_bar

pytestmark = pytest.mark.gpu


def _t(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _ti(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.int32)).cuda()


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _model(gpu, kind, prob, K, tol, **kw):
    if kind == "dense":
        m = gpu.CoFEM(prob.N, prob.D, prob.beta, K=K, T=3, U=400, tol=tol, seed=1, **kw)
        m.set_dictionary(_t(prob.phi))
        op = oracle.DenseOperator(prob.phi)
    elif kind == "conv":
        m = gpu.CoFEM(prob.D, prob.D, prob.beta, K=K, T=3, U=400, tol=tol, seed=1, op="conv",
                      conv_taps=prob.h.shape[0], **kw)
        m.set_dictionary(_t(prob.h))
        op = oracle.ConvOperator(prob.h, prob.D)
    else:
        m = gpu.CoFEM(prob.N, prob.D, prob.beta, K=K, T=3, U=400, tol=tol, seed=1, op="dct", **kw)
        m.set_dictionary(_ti(prob.rows))
        op = oracle.DctOperator(prob.D, prob.rows)
    m.fit(_t(prob.y))
    return m, op


@pytest.mark.parametrize("kind", ["dense", "conv", "dct"])
def test_variance_matches_oracle(gpu, kind):
    if kind == "dense":
        prob = workloads.dense_problem(300, 1000, 30, 0.01, seed=71)
    elif kind == "conv":
        prob = workloads.conv_problem(1200, 64, 20.0, 0.02, 0.05, seed=72)
    else:
        prob = workloads.dct_problem(1024, 341, 60, 0.01, seed=73)
    K, tol, batches, seed = 16, 1e-8, 4, 77
    m, op = _model(gpu, kind, prob, K, tol)
    alpha = oracle.cofem(op, prob.y, prob.beta, T=8, K=K, U=400, tol=tol, seed=1).alpha.astype(np.float32)
    s, mu, st = m.variance(batches, seed=seed, alpha=_t(alpha))
    m.close()
    s, mu = _np(s), _np(mu)
    ref_s, ref_mu, ref_steps = oracle.posterior_variance(op, prob.y, prob.beta, alpha, K, batches, 400, tol, seed)
    tight_s, tight_mu, _ = oracle.posterior_variance(op, prob.y, prob.beta, alpha, K, batches, 400, tol / 100, seed)
    sens_s, sens_mu = _rel(ref_s, tight_s), _rel(ref_mu, tight_mu)
    e_s, e_mu = _rel(s, ref_s), _rel(mu, ref_mu)
    print(f"variance {kind}: CG steps gpu {st['cg_steps']} oracle {ref_steps}")
    assert st["T"] == batches and len(st["cg_steps"]) == batches
    binds(f"variance/{kind}/s", sens_s, 1e-4)
    bar_mu = fp32_solve_bar(op.dense(), prob.beta, alpha)
    binds(f"variance/{kind}/mu", sens_mu, bar_mu)
    check(f"variance/{kind}/s", e_s, 1e-4)
    check(f"variance/{kind}/mu", e_mu, bar_mu)


def test_variance_converges_to_exact_diag_sigma(gpu):
    prob = workloads.dense_problem(120, 400, 12, 0.05, seed=75)
    phi = prob.phi.astype(np.float64)
    alpha = oracle.cofem(phi, prob.y, prob.beta, T=8, K=8, U=400, tol=1e-7, seed=1).alpha.astype(np.float32)
    alpha = alpha.astype(np.float64)
    exact = np.diag(np.linalg.inv(prob.beta * phi.T @ phi + np.diag(alpha)))
    m, _ = _model(gpu, "dense", prob, 8, 1e-7)
    err = {}
    for batches in (1, 64):
        s, _, _ = m.variance(batches, seed=3, alpha=_t(alpha))
        err[batches] = _rel(_np(s), exact)
    m.close()
    print(f"variance error vs exact diag(Sigma): 8 probes {err[1]:.3f}, 512 probes {err[64]:.3f}")
    assert err[64] < 0.3 * err[1]


def test_variance_default_alpha_is_the_fit_alpha(gpu):
    prob = workloads.dense_problem(200, 600, 20, 0.01, seed=78)
    m, _ = _model(gpu, "dense", prob, 8, 1e-6)
    mu0, s0, a0, _ = m.posterior()
    s1, mu1, _ = m.variance(3, seed=9)
    s2, mu2, _ = m.variance(3, seed=9, alpha=a0.clone())
    mu3, s3, a3, _ = m.posterior()
    m.close()
    assert np.array_equal(_np(s1), _np(s2)) and np.array_equal(_np(mu1), _np(mu2))
    assert np.array_equal(_np(mu0), _np(mu3)) and np.array_equal(_np(s0), _np(s3)) and np.array_equal(_np(a0), _np(a3))


def test_variance_rejects_bad_arguments(gpu):
    import torch

    so = gpu.load()
    prob = workloads.dense_problem(64, 256, 5, 0.01, seed=79)
    m = gpu.CoFEM(prob.N, prob.D, prob.beta, K=4, T=2, U=50, tol=1e-6)
    m.set_dictionary(_t(prob.phi))
    s = torch.empty(prob.D, dtype=torch.float32, device="cuda")
    sp = ctypes.c_void_p(s.data_ptr())
    assert so.cofem_variance(m._h, None, 2, 0, sp, None, None) == -4  # before a fit
    m.fit(_t(prob.y))
    assert so.cofem_variance(m._h, None, 0, 0, sp, None, None) == -1
    assert so.cofem_variance(m._h, None, 513, 0, sp, None, None) == -1
    assert so.cofem_variance(m._h, None, 2, 0, None, None, None) == -1
    assert so.cofem_variance(m._h, None, 2, 0, sp, None, None) == 0
    m.close()
