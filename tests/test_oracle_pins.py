"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these tests re-types an oracle formula and compares it with itself:
each checks the oracle against a published value, a closed form, a library
solver, an invariant of conjugate gradients, or exact EM, chosen so that a
dropped term, a wrong sign or index, or a transposed operand fails one of them.
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import (ConvOperator, DctOperator, DenseOperator, cofem, cofem_multitask, dct_matrix, diag_estimate,
                    diag_estimate_general, exact_em, hadamard_probes, log_evidence,
                    nonneg_second_moment, pcg, probe_words, rademacher_probes,
                    splitmix64_outputs, woodbury_sigma)
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# Probe generator
# ---------------------------------------------------------------------------
def test_splitmix64_published_vector():
    lines = [l.split("#")[0].strip() for l in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt"))]
    lines = [l for l in lines if l]
    seed = int(lines[0].split()[1])
    expect = [int(v) for v in lines[1:]]
    assert splitmix64_outputs(seed, len(expect)) == expect


def test_probe_words_are_nested_splitmix_streams():
    seed, t, D = 0xC0FFEE, 7, 300
    key = splitmix64_outputs(seed, t)[t - 1]
    expect = np.array(splitmix64_outputs(key, D), dtype=np.uint64)
    assert np.array_equal(probe_words(seed, t, D), expect)


def test_rademacher_probe_statistics():
    D, K = 8192, 64
    P = rademacher_probes(123, 1, D, K)
    assert P.shape == (D, K)
    assert set(np.unique(P)) == {-1.0, 1.0}
    # balanced: each column mean is within 5 standard errors of 0
    assert np.all(np.abs(P.mean(axis=0)) < 5 / math.sqrt(D))
    # columns (bits) and iterations are uncorrelated
    C = (P.T @ P) / D
    off = C[~np.eye(K, dtype=bool)]
    assert np.max(np.abs(off)) < 5.5 / math.sqrt(D)
    P2 = rademacher_probes(123, 2, D, K)
    assert abs(np.mean(P * P2)) < 5 / math.sqrt(D * K)
    # nested in K: the first k columns do not depend on K
    assert np.array_equal(rademacher_probes(123, 1, D, 8), P[:, :8])


# ---------------------------------------------------------------------------
# Algorithm 2 (PCG)
# ---------------------------------------------------------------------------
def _spd_problem(D=40, Q=5, seed=0, spread=1e3):
    rng = np.random.default_rng(seed)
    N = D // 2
    Phi = rng.standard_normal((N, D)) / math.sqrt(N)
    beta = 50.0
    alpha = np.exp(rng.uniform(0, math.log(spread), D))
    A = beta * Phi.T @ Phi + np.diag(alpha)
    B = rng.standard_normal((D, Q))
    minv = 1.0 / (beta + alpha)
    return A, B, minv


@pytest.mark.parametrize("mode", ["joint", "column"])
def test_pcg_matches_direct_solve(mode):
    A, B, minv = _spd_problem()
    res = pcg(lambda P: A @ P, B, minv, U=500, tol=1e-13, stop_mode=mode)
    Xs = np.linalg.solve(A, B)
    assert res.converged
    assert np.linalg.norm(res.X - Xs) / np.linalg.norm(Xs) < 1e-10


def test_pcg_invariants():
    A, B, minv = _spd_problem(D=30, Q=3, seed=1)
    Xs = np.linalg.solve(A, B)
    res = pcg(lambda P: A @ P, B, minv, U=200, tol=1e-14, record=True)
    H = res.history
    # finite termination (exact arithmetic: at most D steps; allow rounding slack)
    assert res.converged and res.steps <= 30 + 10
    Minv = np.diag(minv)
    Ainv = np.linalg.inv(A)
    lam = np.linalg.eigvalsh(np.sqrt(Minv) @ A @ np.sqrt(Minv))
    kappa = lam[-1] / lam[0]
    rate = (math.sqrt(kappa) - 1) / (math.sqrt(kappa) + 1)
    for q in range(B.shape[1]):
        Rs = [h["R"][:, q] for h in H]
        Ps = [h["P"][:, q] for h in H]
        Xq = [h["X"][:, q] for h in H]
        b = B[:, q]
        nb = math.sqrt(b @ Ainv @ b)
        prev = float("inf")
        for u in range(min(12, len(H) - 1)):
            # recursive residual equals the true residual
            assert np.linalg.norm(Rs[u] - (b - A @ Xq[u])) <= 1e-10 * np.linalg.norm(b)
            # A-norm of the error decreases and obeys the CG convergence lemma
            e = Xs[:, q] - Xq[u]
            ea = math.sqrt(e @ A @ e)
            assert ea <= prev * (1 + 1e-12)
            prev = ea
            assert ea / nb <= 2 * rate ** u * (1 + 1e-9)
            for v in range(u):
                # preconditioned residuals are M^-1-orthogonal
                ru, rv = Rs[u], Rs[v]
                assert abs(ru @ Minv @ rv) <= 1e-8 * math.sqrt((ru @ Minv @ ru) * (rv @ Minv @ rv))
                # directions are A-conjugate
                pu, pv = Ps[u], Ps[v]
                assert abs(pu @ A @ pv) <= 1e-8 * math.sqrt((pu @ A @ pu) * (pv @ A @ pv))


def test_pcg_multi_rhs_equals_single_rhs():
    A, B, minv = _spd_problem(D=40, Q=4, seed=2)
    res = pcg(lambda P: A @ P, B, minv, U=300, tol=1e-8, stop_mode="column")
    for q in range(B.shape[1]):
        r1 = pcg(lambda P: A @ P, B[:, q:q + 1], minv, U=300, tol=1e-8, stop_mode="column")
        # equal up to the rounding of a blocked versus an unblocked product
        assert np.abs(res.X[:, q] - r1.X[:, 0]).max() <= 1e-7 * np.abs(r1.X).max()
        assert res.col_rel_resid[q] <= 1e-8
    # joint rule: every column equals a single-column run with the same step count
    rj = pcg(lambda P: A @ P, B, minv, U=300, tol=1e-6, stop_mode="joint")
    assert rj.converged and rj.rel_resid <= 1e-6
    for q in range(B.shape[1]):
        r1 = pcg(lambda P: A @ P, B[:, q:q + 1], minv, U=rj.steps, tol=0.0, stop_mode="joint")
        assert r1.steps == rj.steps
        assert np.abs(rj.X[:, q] - r1.X[:, 0]).max() <= 1e-7 * np.abs(r1.X).max()


def test_pcg_joint_stop_is_first_crossing():
    A, B, minv = _spd_problem(D=40, Q=3, seed=3)
    res = pcg(lambda P: A @ P, B, minv, U=300, tol=1e-7)
    before = pcg(lambda P: A @ P, B, minv, U=res.steps - 1, tol=1e-7)
    assert res.rel_resid <= 1e-7 < before.rel_resid


def test_printed_recursion_without_preconditioned_directions_fails():
    """The printed directions (P <- B, P <- R + P H) do not converge for a
    non-scalar M, while standard PCG does; this is why the oracle reads the
    algorithm as standard PCG."""
    A, B, minv = _spd_problem(D=60, Q=1, seed=4, spread=1e5)

    def printed(U):
        X = np.zeros_like(B)
        R = B.copy()
        P = B.copy()
        W = minv[:, None] * B
        rho = np.sum(R * W, 0)
        for _ in range(U):
            Psi = A @ P
            g = rho / np.sum(P * Psi, 0)
            X = X + P * g
            R = R - Psi * g
            W = minv[:, None] * R
            rho_old, rho = rho, np.sum(R * W, 0)
            P = R + P * (rho / rho_old)
        return np.linalg.norm(B - A @ X) / np.linalg.norm(B)

    good = pcg(lambda P: A @ P, B, minv, U=200, tol=1e-10)
    assert good.converged
    assert printed(200) > 1e-3


# ---------------------------------------------------------------------------
# Exact EM (the reference CoFEM approximates)
# ---------------------------------------------------------------------------
def _small_dense(N=24, D=48, d=4, seed=5, sigma=0.05):
    p = workloads.dense_problem(N, D, d, sigma, seed)
    return p.phi.astype(np.float64), p.y.astype(np.float64), 1.0 / sigma ** 2


def test_woodbury_equals_inverse():
    phi, y, beta = _small_dense()
    alpha = np.exp(np.random.default_rng(0).uniform(-2, 6, phi.shape[1]))
    Sig = np.linalg.inv(beta * phi.T @ phi + np.diag(alpha))
    assert np.allclose(woodbury_sigma(phi, beta, alpha), Sig, rtol=1e-8, atol=1e-12)


def test_log_evidence_by_bayes_rule_over_z():
    """log p(y | alpha) without the N x N marginal covariance: for any z, Bayes' rule gives
    log p(y) = log p(y | z) + log p(z) - log p(z | y), each a Gaussian density (noise
    N(Phi z, I / beta), prior N(0, diag(alpha)^-1), posterior N(mu, Sigma) with Sigma the
    explicit inverse of beta Phi^T Phi + diag(alpha) and mu = beta Sigma Phi^T y), evaluated
    by scipy at two different z; and the scalar case N = D = 1 against the normal density
    with variance 1 / beta + phi^2 / alpha."""
    from scipy.stats import multivariate_normal, norm

    phi, y, beta = _small_dense()
    N, D = phi.shape
    rng = np.random.default_rng(12)
    alpha = np.exp(rng.uniform(-2, 6, D))
    Sig = np.linalg.inv(beta * phi.T @ phi + np.diag(alpha))
    mu = beta * Sig @ phi.T @ y
    for z in (np.zeros(D), rng.standard_normal(D)):
        via_z = (multivariate_normal(phi @ z, np.eye(N) / beta).logpdf(y)
                 + multivariate_normal(np.zeros(D), np.diag(1.0 / alpha)).logpdf(z)
                 - multivariate_normal(mu, Sig).logpdf(z))
        assert log_evidence(phi, y, beta, alpha) == pytest.approx(via_z, rel=1e-9, abs=1e-7)
    p1, y1, b1, a1 = np.array([[0.7]]), np.array([-1.3]), 4.0, np.array([2.5])
    assert log_evidence(p1, y1, b1, a1) == pytest.approx(norm(0.0, math.sqrt(1 / b1 + 0.49 / 2.5)).logpdf(-1.3),
                                                         rel=1e-12)


def test_exact_em_increases_evidence():
    phi, y, beta = _small_dense()
    _, _, _, alphas = exact_em(phi, y, beta, T=25, record=True)
    ev = [log_evidence(phi, y, beta, a) for a in alphas]
    assert all(b >= a - 1e-8 * abs(a) for a, b in zip(ev, ev[1:]))
    assert ev[-1] > ev[0] + 1.0


def _orthonormal(N, D, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((N, D)))
    return Q  # N x D with orthonormal columns


def test_exact_em_orthonormal_closed_form():
    N, D, beta = 40, 16, 400.0
    phi = _orthonormal(N, D, 6)
    rng = np.random.default_rng(7)
    z = np.zeros(D)
    z[:5] = rng.uniform(1, 2, 5) * rng.choice([-1, 1], 5)
    y = phi @ z + 0.05 * rng.standard_normal(N)
    c = phi.T @ y
    alpha, mu, dS, alphas = exact_em(phi, y, beta, T=3, record=True)
    a2 = alphas[1]
    assert np.allclose(mu, beta * c / (beta + a2 * 0 + alphas[2]), rtol=1e-10)
    assert np.allclose(dS, 1.0 / (beta + alphas[2]), rtol=1e-10)
    # one M-step from alpha^(1) = 1
    assert np.allclose(alphas[1], 1.0 / ((beta * c / (beta + 1)) ** 2 + 1.0 / (beta + 1)), rtol=1e-10)
    # fixed point: alpha* = 1/(c^2 - 1/beta) where c^2 > 1/beta
    alpha_inf, _, _, _ = exact_em(phi, y, beta, T=400)
    big = c ** 2 > 4.0 / beta
    assert np.allclose(alpha_inf[big], 1.0 / (c[big] ** 2 - 1.0 / beta), rtol=1e-6)


# ---------------------------------------------------------------------------
# Algorithm 1 (CoFEM)
# ---------------------------------------------------------------------------
def test_cofem_orthonormal_is_exact():
    """For Phi^T Phi = I, A is diagonal: PCG with theta = 1 ends in one step,
    s equals diag(Sigma) for any K, and CoFEM reproduces exact EM."""
    N, D, beta = 40, 16, 400.0
    phi = _orthonormal(N, D, 8)
    rng = np.random.default_rng(9)
    z = np.zeros(D)
    z[:4] = rng.uniform(1, 2, 4)
    y = phi @ z + 0.05 * rng.standard_normal(N)
    r = cofem(phi, y, beta, T=20, K=3, U=50, tol=1e-12, seed=11, record=True)
    assert all(s == 1 for s in r.cg_steps)
    a_em, mu_em, dS_em, alphas_em = exact_em(phi, y, beta, T=20, record=True)
    for a, b in zip(r.alphas, alphas_em):
        assert np.allclose(a, b, rtol=1e-9)
    assert np.allclose(r.mu, mu_em, rtol=1e-9, atol=1e-14)
    assert np.allclose(r.s, dS_em, rtol=1e-9)
    assert np.allclose(r.alpha, a_em, rtol=1e-9)


def test_cofem_hadamard_probes_reproduce_exact_em():
    """With K = D Hadamard probes the cross terms of Eq. (diag-expansion) vanish,
    so CoFEM equals EM up to the CG tolerance."""
    phi, y, beta = _small_dense(N=16, D=32, d=3, seed=12)
    H = hadamard_probes(32)
    r = cofem(phi, y, beta, T=15, K=32, U=400, tol=1e-13, probes=lambda t: H, record=True)
    a_em, mu_em, dS_em, alphas_em = exact_em(phi, y, beta, T=15, record=True)
    for a, b in zip(r.alphas, alphas_em):
        assert np.allclose(a, b, rtol=1e-6)
    assert np.linalg.norm(r.mu - mu_em) <= 1e-8 * np.linalg.norm(mu_em)
    assert np.allclose(r.s, dS_em, rtol=1e-6)


def test_cofem_nonneg_hadamard_probes_reproduce_exact_nonneg_em():
    """The non-negative M-step (Sec. III-E.2) on top of the covariance-free E-step: with
    K = D Hadamard probes s equals diag(Sigma), so CoFEM equals the explicit-covariance
    EM with the same M-step."""
    phi, y, beta = _small_dense(N=16, D=32, d=3, seed=17)
    H = hadamard_probes(32)
    r = cofem(phi, y, beta, T=10, K=32, U=400, tol=1e-13, probes=lambda t: H, record=True, mstep="nonneg")
    a_em, mu_em, dS_em, alphas_em = exact_em(phi, y, beta, T=10, record=True, mstep="nonneg")
    for a, b in zip(r.alphas, alphas_em):
        # compare the second moments 1/alpha (alpha can be huge where E[z^2] is tiny)
        assert np.allclose(1.0 / a, 1.0 / b, rtol=1e-6, atol=1e-9 * np.max(1.0 / b))
    assert np.linalg.norm(r.mu - mu_em) <= 1e-8 * np.linalg.norm(mu_em)


def test_nonneg_mstep_moves_alpha_by_the_sign_of_mu():
    """One EM step from alpha = 1: the rectified second moment exceeds mu^2 + Sigma_jj where
    mu_j > 0 and falls below it where mu_j < 0, so the non-negative alpha is smaller,
    resp. larger, than the Gaussian one."""
    phi, y, beta = _small_dense(N=24, D=48, d=5, seed=18)
    _, mu, _, _ = exact_em(phi, y, beta, T=1)             # the E-step at alpha = 1
    a_g = exact_em(phi, y, beta, T=2)[0]                  # alpha after one M-step of each kind
    a_n = exact_em(phi, y, beta, T=2, mstep="nonneg")[0]
    pos, neg = mu > 1e-6, mu < -1e-6
    assert pos.any() and neg.any()
    assert np.all(a_n[pos] < a_g[pos])
    assert np.all(a_n[neg] > a_g[neg])


def test_cofem_t1_is_one_estep_at_alpha_one():
    phi, y, beta = _small_dense(seed=13)
    r = cofem(phi, y, beta, T=1, K=8, U=500, tol=1e-13, seed=3)
    _, mu_em, _, _ = exact_em(phi, y, beta, T=1)
    assert np.array_equal(r.alpha, np.ones(phi.shape[1]))
    assert np.linalg.norm(r.mu - mu_em) <= 1e-9 * np.linalg.norm(mu_em)


def test_cofem_approaches_em_as_k_grows():
    phi, y, beta = _small_dense(N=32, D=96, d=5, seed=14)
    _, mu_em, _, _ = exact_em(phi, y, beta, T=10)
    errs = {}
    for K in (2, 8, 64):
        e = []
        for seed in range(4):
            r = cofem(phi, y, beta, T=10, K=K, U=500, tol=1e-10, seed=100 + seed)
            e.append(np.linalg.norm(r.mu - mu_em) / np.linalg.norm(mu_em))
        errs[K] = float(np.mean(e))
    assert errs[64] < errs[8] < errs[2]
    assert errs[64] < 0.5 * errs[2]


def test_lemma1_mean_and_std_of_diag_estimate():
    """Lemma 1: s_j has mean M_jj and std sqrt((1/K) sum_{j' != j} M_jj'^2)."""
    rng = np.random.default_rng(15)
    D, K, trials = 12, 4, 4000
    G = rng.standard_normal((D, D))
    M = G @ G.T / D + np.eye(D)
    S = np.empty((trials, D))
    for i in range(trials):
        P = rademacher_probes(1000 + i, 1, D, K)
        S[i] = diag_estimate(P, M @ P)
    nu = np.sqrt((np.sum(M ** 2, axis=1) - np.diag(M) ** 2) / K)
    mean_err = np.abs(S.mean(0) - np.diag(M))
    assert np.all(mean_err < 4.5 * nu / math.sqrt(trials))
    assert np.allclose(S.std(0), nu, rtol=0.08)


def test_prop1_general_probes_unbiased():
    rng = np.random.default_rng(16)
    D, K, trials = 8, 3, 20000
    M = rng.standard_normal((D, D))
    acc = np.zeros(D)
    for _ in range(trials):
        P = rng.standard_normal((D, K))
        acc += diag_estimate_general(P, M @ P)
    # Gaussian probes: unbiased, but heavier tails than Rademacher
    assert np.allclose(acc / trials, np.diag(M), atol=0.08)
    # Rademacher probes: the general form equals the 1/K form
    P = rademacher_probes(5, 1, D, K)
    assert np.allclose(diag_estimate_general(P, M @ P), diag_estimate(P, M @ P), rtol=0, atol=1e-15)


def test_cofem_floor_clamps_and_counts():
    phi, y, beta = _small_dense(seed=17)
    r0 = cofem(phi, y, beta, T=2, K=4, U=300, tol=1e-10, seed=1)
    r1 = cofem(phi, y, beta, T=2, K=4, U=300, tol=1e-10, seed=1, alpha_floor=1e-3)
    r_e = cofem(phi, y, beta, T=1, K=4, U=300, tol=1e-10, seed=1)
    denom = r_e.mu ** 2 + r_e.s
    low = denom < 1e-3
    assert r1.clamped == int(low.sum()) > 0
    assert np.allclose(r1.alpha[low], 1e3)
    assert np.allclose(r1.alpha[~low], r0.alpha[~low])


def test_cofem_jacobi_preconditioner_same_solution():
    phi, y, beta = _small_dense(N=32, D=64, d=4, seed=18)
    phi = phi * np.linspace(0.2, 3.0, phi.shape[1])[None, :]
    a = cofem(phi, y, beta, T=3, K=6, U=1000, tol=1e-11, seed=2, theta_mode="ones")
    b = cofem(phi, y, beta, T=3, K=6, U=1000, tol=1e-11, seed=2, theta_mode="jacobi")
    assert np.linalg.norm(a.mu - b.mu) <= 1e-7 * np.linalg.norm(a.mu)
    # the Jacobi choice of theta makes M equal to the diagonal of A (Sec. III-C)
    alpha = np.exp(np.random.default_rng(1).uniform(0, 5, phi.shape[1]))
    A = beta * phi.T @ phi + np.diag(alpha)
    assert np.allclose(beta * DenseOperator(phi).col_sq_norms() + alpha, np.diag(A), rtol=1e-13)


def test_cofem_small_workload_recovers_sparse_code():
    """End-to-end sanity on the small workload (not a parity check)."""
    w = workloads.WORKLOADS["small"]
    p = workloads.make_workload("small")
    r = cofem(p.phi, p.y, p.beta, T=w["T"], K=w["K"], U=w["U"], tol=w["tol"], seed=7)
    nrmse = np.linalg.norm(r.mu - p.z) / np.linalg.norm(p.z)
    assert nrmse < 0.05
    assert r.clamped == 0 and r.breakdown == 0


# ---------------------------------------------------------------------------
# Dictionaries and extensions
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("D,L", [(40, 7), (5, 9)])
def test_conv_operator_is_lower_triangular_toeplitz(D, L):
    rng = np.random.default_rng(19)
    h = rng.standard_normal(L)
    op = ConvOperator(h, D)
    Phi = np.zeros((D, D))
    for i in range(D):
        for j in range(D):
            if 0 <= i - j < L:
                Phi[i, j] = h[i - j]
    V = rng.standard_normal((D, 3))
    assert np.allclose(op.matvec(V), Phi @ V, atol=1e-13)
    assert np.allclose(op.rmatvec(V), Phi.T @ V, atol=1e-13)
    assert np.allclose(op.col_sq_norms(), np.sum(Phi ** 2, axis=0), atol=1e-13)
    assert np.allclose(op.dense(), Phi)


@pytest.mark.parametrize("D,L", [(40, 7), (30, 30), (9, 20)])
def test_conv_normal_rows_match_explicit_matrix(D, L):
    # sampled rows of beta Phi^T Phi P + alpha P against the explicit band matrix
    rng = np.random.default_rng(23)
    h = rng.standard_normal(L)
    Phi = np.zeros((D, D))
    for i in range(D):
        for j in range(D):
            if 0 <= i - j < L:
                Phi[i, j] = h[i - j]
    P = rng.standard_normal((D, 4))
    alpha = rng.uniform(0.5, 2.0, D)
    beta = 3.5
    full = beta * Phi.T @ (Phi @ P) + alpha[:, None] * P
    rows = [0, 1, D // 2, D - 2, D - 1]
    got = ConvOperator(h, D).normal_rows(P, alpha, beta, rows)
    assert np.allclose(got, full[rows], atol=1e-12)


def _dct_by_cosine_sums(D):
    """Omega_kn = s_k cos(pi (2n+1) k / 2D), one math.cos per entry."""
    Om = np.zeros((D, D))
    for k in range(D):
        sk = math.sqrt((1.0 if k == 0 else 2.0) / D)
        for n in range(D):
            Om[k, n] = sk * math.cos(math.pi * (2 * n + 1) * k / (2 * D))
    return Om


@pytest.mark.parametrize("D,N", [(16, 5), (24, 24), (64, 21)])
def test_dct_operator_matches_cosine_definition(D, N):
    """Phi = M Omega^{-1} (Sec. V-A.1): the library-DCT matvec / rmatvec, the column
    norms and the explicit matrix against the DCT-II written as cosine sums."""
    rng = np.random.default_rng(D + N)
    rows = rng.permutation(D)[:N]
    Om = _dct_by_cosine_sums(D)
    Phi = Om.T[rows]                                    # rows of Omega^{-1} = Omega^T
    op = DctOperator(D, rows)
    V = rng.standard_normal((D, 3))
    Uu = rng.standard_normal((N, 3))
    assert np.allclose(op.matvec(V), Phi @ V, atol=1e-12)
    assert np.allclose(op.rmatvec(Uu), Phi.T @ Uu, atol=1e-12)
    assert np.allclose(op.col_sq_norms(), np.sum(Phi ** 2, axis=0), atol=1e-12)
    assert np.allclose(op.dense(), Phi, atol=1e-12)
    assert np.allclose(dct_matrix(D), Om, atol=1e-12)


def test_dct_orthonormality_and_cosine_closed_form():
    """Omega is orthogonal, so Phi Phi^T = I_N for distinct samples; and the DCT of the
    sampled cosine x_n = cos(pi (2n+1) k0 / 2D) is s_k0 D / 2 at k0 (D s_0 at k0 = 0)."""
    D = 48
    Om = dct_matrix(D)
    assert np.allclose(Om @ Om.T, np.eye(D), atol=1e-12)
    rng = np.random.default_rng(3)
    rows = rng.permutation(D)[:16]
    Phi = DctOperator(D, rows).dense()
    assert np.allclose(Phi @ Phi.T, np.eye(16), atol=1e-12)
    full = DctOperator(D, np.arange(D))
    n = np.arange(D)
    for k0 in (0, 1, 7, D - 1):
        x = np.cos(np.pi * (2 * n + 1) * k0 / (2 * D))
        want = np.zeros(D)
        want[k0] = math.sqrt(D) if k0 == 0 else math.sqrt(2.0 / D) * D / 2
        assert np.allclose(full.rmatvec(x), want, atol=1e-12)
        assert np.allclose(full.matvec(want), x, atol=1e-12)


def test_cofem_dct_hadamard_probes_reproduce_exact_em():
    """On the DCT dictionary with N = D/3 samples, K = D Hadamard probes make CoFEM's
    E-step exact, so it follows covariance-based EM on the explicit matrix."""
    D, N, beta = 32, 10, 1e4
    rng = np.random.default_rng(29)
    op = DctOperator(D, np.sort(rng.permutation(D)[:N]))
    z = np.zeros(D)
    z[rng.permutation(D)[:3]] = rng.normal(0.0, math.sqrt(5.0), 3)
    y = op.matvec(z) + 0.01 * rng.standard_normal(N)
    H = hadamard_probes(D)
    r = cofem(op, y, beta, T=12, K=D, U=400, tol=1e-13, probes=lambda t: H, record=True)
    a_em, mu_em, dS_em, alphas_em = exact_em(op.dense(), y, beta, T=12, record=True)
    for a, b in zip(r.alphas, alphas_em):
        assert np.allclose(a, b, rtol=1e-6)
    assert np.linalg.norm(r.mu - mu_em) <= 1e-8 * np.linalg.norm(mu_em)
    assert np.allclose(r.s, dS_em, rtol=1e-6)


def test_nonneg_second_moment_matches_truncated_gaussian_integral():
    from scipy.integrate import quad

    for mu, v in [(0.7, 0.2), (-0.5, 0.1), (0.0, 1.0), (-3.0, 0.04), (2.0, 1e-4)]:
        sd = math.sqrt(v)
        top = max(mu, 0.0)
        off = -0.5 * ((top - mu) / sd) ** 2  # log-density maximum on z >= 0

        def dens(z):
            return math.exp(-0.5 * ((z - mu) / sd) ** 2 - off)

        hi = top + 40 * sd
        kw = dict(limit=400, epsabs=0.0, epsrel=1e-12)
        Z = quad(dens, 0.0, hi, points=[top] if top > 0 else None, **kw)[0]
        m2 = quad(lambda z: z * z * dens(z), 0.0, hi, points=[top] if top > 0 else None, **kw)[0]
        got = float(nonneg_second_moment(np.array([mu]), np.array([v]))[0])
        assert got == pytest.approx(m2 / Z, rel=1e-7)


def test_multitask_reduces_and_matches_exact_multitask_em():
    N, D, beta = 30, 12, 400.0
    rng = np.random.default_rng(20)
    phis = [_orthonormal(N, D, 21 + l) for l in range(3)]
    z = np.zeros(D)
    z[:3] = rng.uniform(1, 2, 3)
    ys = [p @ z + 0.05 * rng.standard_normal(N) for p in phis]
    # L = 1 is single-task CoFEM
    a1, mu1, s1, _ = cofem_multitask(phis[:1], ys[:1], beta, T=6, K=4, U=50, tol=1e-12, seed=9)
    r = cofem(phis[0], ys[0], beta, T=6, K=4, U=50, tol=1e-12, seed=9)
    assert np.allclose(a1, r.alpha, rtol=1e-12) and np.allclose(mu1[0], r.mu, rtol=1e-12)
    # orthonormal tasks: the shared-alpha EM has a closed-form E-step per task
    aL, muL, sL, _ = cofem_multitask(phis, ys, beta, T=8, K=4, U=50, tol=1e-12, seed=9)
    cs = [p.T @ y for p, y in zip(phis, ys)]
    alpha = np.ones(D)
    for t in range(1, 9):
        mus = [beta * c / (beta + alpha) for c in cs]
        sig = 1.0 / (beta + alpha)
        if t < 8:
            alpha = 3.0 / sum(m ** 2 + sig for m in mus)
    assert np.allclose(aL, alpha, rtol=1e-9)
    for m, mm in zip(muL, mus):
        assert np.allclose(m, mm, rtol=1e-9)


def test_posterior_variance_hadamard_is_exact_diag_sigma():
    """K = D Hadamard probes make the diagonal estimate exact: the post-fit variance
    equals diag((beta Phi^T Phi + diag(alpha))^{-1}) from the explicit inverse, and
    mu equals the explicit posterior mean."""
    phi, y, beta = _small_dense(N=16, D=32, d=3, seed=61)
    rng = np.random.default_rng(62)
    alpha = np.exp(rng.uniform(-2, 6, 32))
    H = hadamard_probes(32)
    s, mu, steps = oracle.posterior_variance(phi, y, beta, alpha, K=32, batches=2, U=400, tol=1e-13,
                                             probes=lambda b: H)
    Sigma = np.linalg.inv(beta * phi.T @ phi + np.diag(alpha))
    assert np.allclose(s, np.diag(Sigma), rtol=1e-8)
    assert np.allclose(mu, beta * Sigma @ phi.T @ y, rtol=1e-8, atol=1e-12)
    assert len(steps) == 2


def test_posterior_variance_converges_with_probe_count():
    """Rademacher probes: the estimate is unbiased and its error falls like
    1 / sqrt(K * batches) (Lemma 1), so 64 batches beat 1 batch by a wide margin."""
    phi, y, beta = _small_dense(N=24, D=48, d=4, seed=63)
    alpha = np.exp(np.random.default_rng(64).uniform(-2, 4, 48))
    exact = np.diag(np.linalg.inv(beta * phi.T @ phi + np.diag(alpha)))
    err = {}
    for B in (1, 64):
        s, _, _ = oracle.posterior_variance(phi, y, beta, alpha, K=8, batches=B, U=400, tol=1e-12, seed=5)
        err[B] = np.linalg.norm(s - exact) / np.linalg.norm(exact)
    assert err[64] < 0.3 * err[1]
    # batch b uses the probes of iteration key b: one batch at key 1 equals the T = 1 fit's s at that alpha
    s1, mu1, _ = oracle.posterior_variance(phi, y, beta, alpha, K=8, batches=1, U=400, tol=1e-12, seed=5)
    r = cofem(phi, y, beta, T=1, K=8, U=400, tol=1e-12, seed=5, alpha0=alpha)
    assert np.allclose(s1, r.s, rtol=1e-9, atol=1e-15) and np.allclose(mu1, r.mu, rtol=1e-9, atol=1e-15)
