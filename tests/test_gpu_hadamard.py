"""The whole GPU path against a closed form: with the D columns of a Sylvester-Hadamard
matrix as probes (cofem_set_probe_mode), the cross terms of the diagonal estimate
(Eq. diag-estimate) cancel, so CoFEM reproduces EM with the explicit posterior
covariance (Eq. estep-params, Eq. mstep) up to the CG tolerance.  This pins the GPU
fit to exact EM with no random probes involved (the oracle's exact_em is the plain
matrix-inverse definition, itself pinned against the closed forms of the oracle's
tests).

* dense FP32 (K = D = 32, T = 10) against exact EM, the bf16-refined fit against
  exact EM run with the same precision schedule (E-steps 1 .. T-3 on the
  bf16-rounded dictionary, the last three on the FP32 one), and the DCT dictionary
  (D = 32, all FP32);
* the FP32 fits against the oracle's CoFEM with the same Hadamard probes and stop
  rule (the same algorithm step for step);
* bad probe modes rejected.

Bars: mu within 1e-4 and s, alpha within 1e-3 relative of exact EM at tol 1e-7 (FP32
CG stops at a residual of about 1e-7 relative, and T = 10 EM iterations propagate it;
measured 8e-6 / 6e-5); 3e-3 for s and alpha of the bf16-refined fit.
"""
import ctypes

import numpy as np
import pytest

import oracle
import workloads
from bars import check

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


def _bf16_rne(x):
    """FP32 -> bfloat16 by round to nearest even, back to FP64."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("kind", ["fp32", "bf16_refined", "dct"])
def test_hadamard_fit_equals_exact_em(gpu, kind):
    D, T = 32, 10
    if kind == "dct":
        prob = workloads.dct_problem(D, 16, 4, 0.01, seed=91)
        m = gpu.CoFEM(prob.N, D, prob.beta, K=D, T=T, U=400, tol=1e-7, seed=5, op="dct")
        m.set_dictionary(_ti(prob.rows))
        phi = oracle.DctOperator(D, prob.rows).dense()
    else:
        prob = workloads.dense_problem(16, D, 4, 0.01, seed=92)
        kw = dict(phi_dtype="bf16", refine_last=3) if kind == "bf16_refined" else {}
        m = gpu.CoFEM(prob.N, D, prob.beta, K=D, T=T, U=400, tol=1e-7, seed=5, **kw)
        m.set_dictionary(_t(prob.phi))
        phi = prob.phi.astype(np.float64)
    m.set_probe_mode("hadamard")
    m.fit(_t(prob.y))
    mu, s, alpha, st = m.posterior()
    m.close()
    mu, s, alpha = _np(mu), _np(s), _np(alpha)
    if kind == "bf16_refined":
        # the same precision schedule in exact EM: E-steps 1 .. T - 3 on the bf16-rounded
        # dictionary (b from it too), the last three on the FP32 one
        a_mid, _, _, _ = oracle.exact_em(_bf16_rne(prob.phi), prob.y, prob.beta, T=T - 2)
        a_em, mu_em, dS_em, _ = oracle.exact_em(phi, prob.y, prob.beta, T=3, alpha0=a_mid)
    else:
        a_em, mu_em, dS_em, _ = oracle.exact_em(phi, prob.y, prob.beta, T=T)
    H = oracle.hadamard_probes(D)
    op = oracle.DctOperator(D, prob.rows) if kind == "dct" else phi
    ref = oracle.cofem(op, prob.y, prob.beta, T=T, K=D, U=400, tol=1e-7, probes=lambda t: H)
    e = dict(mu=_rel(mu, mu_em), s=_rel(s, dS_em), alpha=_rel(alpha, a_em))
    print(f"hadamard {kind}: CG steps {st['cg_steps']}")
    # bf16 phase: the GPU applies the rounded dictionary to P carried as hi/lo bf16 pieces
    # (2^-17), exact EM to the exact P; alpha^(T-2) carries that into s
    tol_s = 3e-3 if kind == "bf16_refined" else 1e-3
    check(f"hadamard_{kind}/mu_vs_exact_em", e["mu"], 1e-4)
    check(f"hadamard_{kind}/s_vs_exact_em", e["s"], tol_s)
    check(f"hadamard_{kind}/alpha_vs_exact_em", e["alpha"], tol_s)
    if kind != "bf16_refined":
        check(f"hadamard_{kind}/mu_vs_oracle", _rel(mu, ref.mu), 1e-4)
        check(f"hadamard_{kind}/s_vs_oracle", _rel(s, ref.s), 1e-4)


def test_probe_mode_rejects_bad_arguments(gpu):
    so = gpu.load()
    for D, K, mode, ok in ((32, 8, 1, True), (48, 8, 1, False), (16, 20, 1, False), (32, 8, 2, False),
                           (32, 8, 0, True), (48, 8, 0, True)):
        p = gpu.make_params(N=8, D=D, beta=1e4, K=K, T=1, U=1, tol=0.0)
        h = ctypes.c_void_p()
        assert so.cofem_create(ctypes.byref(p), None, ctypes.byref(h)) == 0
        try:
            assert (so.cofem_set_probe_mode(h, mode) == 0) == ok, (D, K, mode)
        finally:
            so.cofem_destroy(h)
