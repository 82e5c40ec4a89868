"""The no-allocation entry point cofem_conv_apply_A_static (the FIR operator with its
scratch in a static device array) against the existing entry point it varies,
cofem_apply_A on a context of the FIR dictionary (FP32 operator): the same kernels in the
same order, so the outputs must agree bitwise, on two calls in a row (the second with a
smaller signal and fewer columns, over the scratch the first one left behind), and both
within the FP32 operator's bar of the oracle's direct FIR sums (2e-5 per column).
"""
import ctypes

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _t(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


CASES = [(5000, 256, 21, 1), (1234, 37, 5, 2)]  # (D, taps, columns, seed): the second call is smaller


def test_static_conv_operator_matches_apply_A(gpu):
    import torch

    for D, L, ncols, seed in CASES:
        print(f"static conv operator D={D} L={L} ncols={ncols}", flush=True)
        rng = np.random.default_rng(seed)
        h = rng.standard_normal(L).astype(np.float32)
        beta = 400.0
        alpha = np.exp(rng.uniform(-3, 8, D)).astype(np.float32)
        P = rng.standard_normal((ncols, D)).astype(np.float32)
        m = gpu.CoFEM(D, D, beta, K=max(ncols - 1, 1), T=1, U=1, tol=0.0, op="conv", conv_taps=L, phi_dtype="fp32")
        m.set_dictionary(_t(h))
        Psi_ref, pi_ref = m.apply_A(_t(alpha), _t(P), use_bf16=False, want_pi=True)
        m.close()
        Psi, pi = gpu.conv_apply_A_static(_t(h), _t(alpha), _t(P), beta, want_pi=True)
        torch.cuda.synchronize()
        assert torch.equal(Psi, Psi_ref)
        assert torch.equal(pi, pi_ref)
        op = oracle.ConvOperator(h, D)
        Pt = P.T.astype(np.float64)
        ref = (beta * op.rmatvec(op.matvec(Pt)) + alpha.astype(np.float64)[:, None] * Pt).T
        got = Psi.cpu().numpy().astype(np.float64)
        err = max(_rel(got[q], ref[q]) for q in range(ncols))
        print(f"  bitwise equal to cofem_apply_A; max column error vs oracle {err:.2e}")
        assert err < 2e-5


def test_static_conv_operator_rejects_oversized_and_bad_arguments(gpu):
    import torch

    so = gpu.load()
    z = torch.zeros(16, dtype=torch.float32, device="cuda")
    p = ctypes.c_void_p(z.data_ptr())
    # 2^20 samples with 33 columns need about 600 MB of scratch: rejected before any work
    assert so.cofem_conv_apply_A_static(p, 256, 1 << 20, 400.0, p, p, p, 33, None, None) == -1
    assert "scratch" in so.cofem_last_error().decode()
    assert so.cofem_conv_apply_A_static(None, 4, 16, 400.0, p, p, p, 1, None, None) == -1
    assert so.cofem_conv_apply_A_static(p, 0, 16, 400.0, p, p, p, 1, None, None) == -1
    assert so.cofem_conv_apply_A_static(p, 4, 16, 0.0, p, p, p, 1, None, None) == -1
    assert so.cofem_conv_apply_A_static(p, 4, 16, 400.0, p, p, p, 65, None, None) == -1
