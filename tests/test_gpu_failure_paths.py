"""Failure paths of the GPU path, each forced from the inputs (no kernel is made to fault):

* a NaN or an infinity in y, in the dictionary or in the FIR taps: the call returns
  COFEM_EINVAL before any EM work, says what was wrong, and the context stays usable;
* U = 1: Algorithm 2 returns X after U steps without error (non-convergence is not a
  failure); every E-step reports one CG step and its residual ratio, which matches the
  oracle's;
* breakdown: with alpha = -1e9 the matrix A is negative definite, so every column hits
  pi_q < 0 at its first step with rho_q != 0; the GPU, like the oracle's PCG, freezes
  every column (X stays 0), counts the breakdowns and reports COFEM_EBREAKDOWN for the mu
  column.
"""
import ctypes

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _t(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def test_non_finite_observation_is_rejected(gpu):
    prob = workloads.dense_problem(64, 256, 10, 0.01, seed=3)
    m = gpu.CoFEM(prob.N, prob.D, prob.beta, K=8, T=3, U=100, tol=1e-6, seed=1)
    m.set_dictionary(_t(prob.phi))
    for bad in (np.nan, np.inf, -np.inf):
        y = prob.y.copy()
        y[[5, 40]] = bad
        with pytest.raises(gpu.CofemError) as e:
            m.fit(_t(y))
        assert e.value.status == -1 and "y has 2 non-finite" in str(e.value)
        with pytest.raises(gpu.CofemError) as e:
            m.posterior()
        assert e.value.status == -4                      # no successful fit
    m.fit(_t(prob.y))                                    # still usable
    mu, _, _, st = m.posterior()
    assert np.isfinite(_np(mu)).all() and st["total_cg_steps"] > 0
    m.close()


def test_non_finite_dictionary_and_taps_are_rejected(gpu):
    prob = workloads.dense_problem(64, 256, 10, 0.01, seed=4)
    m = gpu.CoFEM(prob.N, prob.D, prob.beta, K=8, T=2, U=100, tol=1e-6)
    phi = prob.phi.copy()
    phi[17, 200] = np.inf
    with pytest.raises(gpu.CofemError) as e:
        m.set_dictionary(_t(phi))
    assert e.value.status == -1 and "dictionary has 1 non-finite" in str(e.value)
    with pytest.raises(gpu.CofemError) as e:
        m.fit(_t(prob.y))
    assert e.value.status == -4                          # no dictionary loaded
    m.set_dictionary(_t(prob.phi))
    m.fit(_t(prob.y))
    m.close()
    h = workloads.exp_filter(32, 10.0)
    h[3] = np.nan
    c = gpu.CoFEM(300, 300, 400.0, K=4, T=2, U=50, tol=1e-6, op="conv", conv_taps=32)
    with pytest.raises(gpu.CofemError) as e:
        c.set_dictionary(_t(h))
    assert e.value.status == -1 and "taps" in str(e.value)
    c.close()


def test_non_finite_task_observation_is_rejected(gpu):
    probs = workloads.multitask_problems(2, N=60, D=200, d=6, sigma=0.01, seed=8)
    m = gpu.MultiTask(2, 60, 200, probs[0].beta, K=4, T=2, U=50, tol=1e-6)
    for l, p in enumerate(probs):
        m.set_dictionary(l, _t(p.phi))
    y1 = probs[1].y.copy()
    y1[0] = np.nan
    with pytest.raises(gpu.CofemError) as e:
        m.fit([_t(probs[0].y), _t(y1)])
    assert e.value.status == -1 and "ys[1]" in str(e.value)
    m.close()


def test_u1_reports_non_convergence_like_the_oracle(gpu):
    prob = workloads.dense_problem(128, 512, 12, 0.01, seed=6)
    K, T = 8, 5
    m = gpu.CoFEM(prob.N, prob.D, prob.beta, K=K, T=T, U=1, tol=1e-6, seed=21)
    m.set_dictionary(_t(prob.phi))
    m.fit(_t(prob.y))                                    # not an error (Alg. 2 returns X after U steps)
    mu, s, alpha, st = m.posterior()
    m.close()
    ref = oracle.cofem(prob.phi, prob.y, prob.beta, T=T, K=K, U=1, tol=1e-6, seed=21)
    assert st["cg_steps"] == [1] * T and ref.cg_steps == [1] * T
    got, exp = np.array(st["rel_resid"]), np.array(ref.rel_resid)
    print(f"U = 1: residual ratios gpu {got} oracle {exp}")
    assert np.all(got > 1e-6)                            # none met the tolerance
    assert np.allclose(got, exp, rtol=1e-4)
    assert np.linalg.norm(_np(mu) - ref.mu) <= 1e-4 * np.linalg.norm(ref.mu)


def test_breakdown_freezes_columns_and_is_reported(gpu):
    prob = workloads.dense_problem(64, 256, 10, 0.01, seed=7)
    K, U, batches = 8, 12, 2
    m = gpu.CoFEM(prob.N, prob.D, prob.beta, K=K, T=2, U=U, tol=1e-6, seed=1)
    m.set_dictionary(_t(prob.phi))
    m.fit(_t(prob.y))
    so = gpu.load()
    neg = _t(np.full(prob.D, -1e9))                      # A = beta Phi^T Phi - 1e9 I is negative definite
    s_out = _t(np.full(prob.D, 7.0))
    mu_out = _t(np.full(prob.D, 7.0))
    st = gpu.Stats()
    rc = so.cofem_variance(m._h, ctypes.c_void_p(neg.data_ptr()), batches, 5, ctypes.c_void_p(s_out.data_ptr()),
                           ctypes.c_void_p(mu_out.data_ptr()), ctypes.byref(st))
    msg = so.cofem_last_error().decode()
    m.close()
    assert rc == -5 and "breakdown" in msg
    assert st.breakdown == batches * (K + 1)            # every column of every batch, once
    assert list(st.cg_steps[:batches]) == [U] * batches  # frozen columns never meet the stop rule
    assert np.all(_np(s_out) == 0.0) and np.all(_np(mu_out) == 0.0)   # X stayed 0
    # the oracle's PCG on the same system: every column breaks down, X = 0
    a = np.full(prob.D, -1e9)
    phi = prob.phi.astype(np.float64)
    B = np.column_stack([prob.beta * phi.T @ prob.y.astype(np.float64), oracle.rademacher_probes(3, 1, prob.D, K)])
    res = oracle.pcg(lambda P: prob.beta * phi.T @ (phi @ P) + a[:, None] * P, B, 1.0 / (prob.beta + a), U, 1e-6)
    assert res.breakdown.all() and np.all(res.X == 0.0) and res.steps == U
