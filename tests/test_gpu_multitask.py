"""GPU parity of multi-task CoFEM (Sec. III-E.1, cofem_mt_*): L problems sharing one
alpha, each task's E-step covariance-free with its own dictionary and probes (seed + l),
the joint M-step alpha_j = L / sum_l (mu_lj^2 + s_lj), against the oracle's
`cofem_multitask` at the same probes, stop rule and tolerance (FP32 bar as for single
fits: mu within 1e-4, s within 1e-3, alpha on the support within 1e-3 in log).  Both
forms: "batched" (all tasks' systems in one launch per phase) and "streams" (one context
per task on its own stream)."""
import numpy as np
import pytest

import oracle
import workloads
from bars import BF16_ROUNDED_MU, binds, check, fp32_fit_bar

pytestmark = pytest.mark.gpu


def _t(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("mode", ["streams", "batched"])
@pytest.mark.parametrize("L", [1, 3])
def test_multitask_matches_oracle(gpu, L, mode):
    probs = workloads.multitask_problems(L, N=120, D=400, d=12, sigma=0.01, seed=61)
    K, T, U, tol, seed = 8, 30, 300, 1e-6, 21
    m = gpu.MultiTask(L, 120, 400, probs[0].beta, K=K, T=T, U=U, tol=tol, seed=seed, mode=mode)
    assert m.batched == (mode == "batched")
    for l, p in enumerate(probs):
        m.set_dictionary(l, _t(p.phi))
    m.fit([_t(p.y) for p in probs])
    out = [m.posterior(l) for l in range(L)]
    m.close()
    a_ref, mus_ref, ss_ref, steps_ref = oracle.cofem_multitask([p.phi for p in probs], [p.y for p in probs],
                                                               probs[0].beta, T=T, K=K, U=U, tol=tol, seed=seed)
    alpha = _np(out[0][2])
    sup = np.abs(mus_ref[0]) > 1e-3 * np.abs(mus_ref[0]).max()
    key = "multitask" if mode == "streams" else "multitask_batched"
    for l in range(L):
        mu, s, a, st = out[l]
        e_mu, e_s = _rel(_np(mu), mus_ref[l]), _rel(_np(s), ss_ref[l])
        print(f"{mode} L={L} task {l}: CG steps {st['total_cg_steps']} (oracle {sum(r[l] for r in steps_ref)})")
        check(f"{key}_L{L}/task{l}/mu", e_mu, 1e-4)
        check(f"{key}_L{L}/task{l}/s", e_s, 1e-3)
        assert np.array_equal(_np(a), alpha)        # every task reports the shared alpha
        # the record: one CG step count and residual ratio per E-step
        assert st["T"] == T and sum(st["cg_steps"]) == st["total_cg_steps"]
        assert all(1 <= n <= U for n in st["cg_steps"])
        assert all(0.0 < r <= tol or n == U for r, n in zip(st["rel_resid"], st["cg_steps"]))
    assert np.max(np.abs(np.log(alpha[sup] / a_ref[sup]))) < 1e-3
    if L == 1:
        # one task is plain CoFEM
        ref1 = oracle.cofem(probs[0].phi, probs[0].y, probs[0].beta, T=T, K=K, U=U, tol=tol, seed=seed)
        assert _rel(_np(out[0][0]), ref1.mu) <= 1e-4


def test_multitask_shares_support_better_than_single_tasks(gpu):
    """The point of sharing alpha: with few measurements per task, the joint fit recovers
    the common support better than the tasks fitted one by one."""
    L, N, D, d = 4, 60, 400, 20
    probs = workloads.multitask_problems(L, N=N, D=D, d=d, sigma=0.01, seed=62)
    kw = dict(K=8, T=30, U=300, tol=1e-5, seed=3)
    m = gpu.MultiTask(L, N, D, probs[0].beta, **kw)
    for l, p in enumerate(probs):
        m.set_dictionary(l, _t(p.phi))
    m.fit([_t(p.y) for p in probs])
    joint = [_np(m.posterior(l)[0]) for l in range(L)]
    m.close()
    single = []
    for p in probs:
        c = gpu.CoFEM(N, D, p.beta, **kw)
        c.set_dictionary(_t(p.phi))
        c.fit(_t(p.y))
        single.append(_np(c.posterior()[0]))
        c.close()
    err = lambda mus: np.mean([np.linalg.norm(mu - p.z) / np.linalg.norm(p.z) for mu, p in zip(mus, probs)])
    print(f"NRMSE joint {err(joint):.3f}, single {err(single):.3f}")
    assert err(joint) < err(single)


@pytest.mark.parametrize("mode", ["streams", "batched"])
def test_multitask_concurrent_fit_is_deterministic(gpu, mode):
    """The tasks' E-steps run concurrently (on their own streams, or as the tiles of one
    launch per phase); every task's reductions are in a fixed order and the shared alpha
    is formed after all of them, so two fits on the same inputs agree bitwise (and the
    caller's stream sees the finished fit)."""
    import torch

    L, N, D = 3, 200, 800
    probs = workloads.multitask_problems(L, N=N, D=D, d=20, sigma=0.01, seed=63)
    m = gpu.MultiTask(L, N, D, probs[0].beta, K=8, T=12, U=300, tol=1e-6, seed=4, mode=mode)
    for l, p in enumerate(probs):
        m.set_dictionary(l, _t(p.phi))
    ys = [_t(p.y) for p in probs]
    runs = []
    for _ in range(2):
        m.fit(ys)
        torch.cuda.current_stream().synchronize()
        runs.append([tuple(_np(x) for x in m.posterior(l)[:3]) for l in range(L)])
    m.close()
    for l in range(L):
        for a, b in zip(runs[0][l], runs[1][l]):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("dtype", ["fp32", "bf16"])
def test_multitask_conv_matches_oracle(gpu, dtype):
    """Multi-task fits on FIR dictionaries (each task its own filter and data, one shared
    alpha): FP32, and all-bf16 E-steps against the oracle on the bf16-rounded taps (the
    right-hand side b formed from the same taps).  mu within 1e-4 (FP32) or the bf16 bound
    (the signals travel as hi/lo bf16 pairs); tol 1e-8, where the oracle's own mu moves by
    far less than that with the tolerance (the FIR systems are ill-conditioned)."""
    D, taps, L = 1200, 64, 2
    probs = [workloads.conv_problem(D, taps, tau, 0.02, 0.05, seed=64 + l) for l, tau in enumerate((20.0, 30.0))]
    K, T, U, tol, seed = 8, 12, 600, 1e-8, 5
    kw = dict(phi_dtype="bf16", refine_last=0) if dtype == "bf16" else {}
    m = gpu.MultiTask(L, D, D, probs[0].beta, K=K, T=T, U=U, tol=tol, seed=seed, op="conv", conv_taps=taps, **kw)
    for l, p in enumerate(probs):
        m.set_dictionary(l, _t(p.h))
    m.fit([_t(p.y) for p in probs])
    out = [m.posterior(l) for l in range(L)]
    m.close()

    def rne(x):
        u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
        u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
        return u.astype(np.uint32).view(np.float32).astype(np.float64)

    ops = [oracle.ConvOperator(rne(p.h) if dtype == "bf16" else p.h, D) for p in probs]
    ys = [p.y for p in probs]
    _, mus, ss, _ = oracle.cofem_multitask(ops, ys, probs[0].beta, T=T, K=K, U=U, tol=tol, seed=seed)
    _, mus_t, _, _ = oracle.cofem_multitask(ops, ys, probs[0].beta, T=T, K=K, U=U, tol=tol / 100, seed=seed)
    bar = BF16_ROUNDED_MU if dtype == "bf16" else 1e-4
    for l in range(L):
        binds(f"multitask_conv_{dtype}/task{l}", _rel(mus[l], mus_t[l]), bar)
        check(f"multitask_conv_{dtype}/task{l}/mu", _rel(_np(out[l][0]), mus[l]), bar)
        check(f"multitask_conv_{dtype}/task{l}/s", _rel(_np(out[l][1]), ss[l]), 10 * bar)


def test_multitask_dct_matches_oracle(gpu):
    """Multi-task fits on subsampled DCT dictionaries (each task its own kept samples and
    data, one shared alpha; D = 2^11 takes the split DCT operator) against the oracle."""
    D, N, L = 2048, 682, 3
    probs = [workloads.dct_problem(D, N, 150, 0.01, seed=66 + l) for l in range(L)]
    # tol 1e-9: at 1e-8 the oracle's mu still moves by 1.0e-5 with the tolerance here
    K, T, U, tol, seed = 8, 10, 400, 1e-9, 6
    m = gpu.MultiTask(L, N, D, probs[0].beta, K=K, T=T, U=U, tol=tol, seed=seed, op="dct")
    for l, p in enumerate(probs):
        import torch

        m.set_dictionary(l, torch.from_numpy(np.ascontiguousarray(p.rows, dtype=np.int32)).cuda())
    m.fit([_t(p.y) for p in probs])
    out = [m.posterior(l) for l in range(L)]
    m.close()
    ops = [oracle.DctOperator(D, p.rows) for p in probs]
    ys = [p.y for p in probs]
    a_ref, mus, ss, _ = oracle.cofem_multitask(ops, ys, probs[0].beta, T=T, K=K, U=U, tol=tol, seed=seed)
    _, mus_t, _, _ = oracle.cofem_multitask(ops, ys, probs[0].beta, T=T, K=K, U=U, tol=tol / 100, seed=seed)
    for l in range(L):
        # E-step 1 (alpha = 1) solves a system with kappa ~ 1e4 here (N = D/3, theta = 1); its
        # FP32 floor of about kappa 2^-24 is still partly in mu after 10 EM iterations
        bar = fp32_fit_bar(ops[l].dense(), probs[0].beta, [np.ones(D), a_ref])
        binds(f"multitask_dct/task{l}", _rel(mus[l], mus_t[l]), 1e-4)
        check(f"multitask_dct/task{l}/mu", _rel(_np(out[l][0]), mus[l]), bar)
        check(f"multitask_dct/task{l}/s", _rel(_np(out[l][1]), ss[l]), 10 * bar)


def test_batched_tasks_with_different_step_counts(gpu):
    """Tasks whose E-steps need very different numbers of CG steps (one task's dictionary
    scaled down, which makes its systems far better conditioned) finish their solves at
    different launches: the early ones wait for the group, the joint M-step sees every
    task's final mu and s, and the fit matches the oracle; the record shows the different
    counts.  tol 1e-8, where the oracle's mu moves by under 3e-7 to tol 1e-10; the bar is
    the FP32 floor of the fit's systems (kappa up to 2.3e3 at alpha = 1)."""
    L, N, D = 3, 250, 500
    probs = workloads.multitask_problems(L, N=N, D=D, d=15, sigma=0.05, seed=68)
    K, T, U, tol, seed = 8, 8, 600, 1e-8, 9
    # the tasks share beta; task 2's dictionary scaled by 0.01 brings its A close to diag(alpha)
    # (the oracle takes 1333, 1378 and 504 CG steps over the fit)
    phis = [p.phi if l < 2 else 0.01 * p.phi for l, p in enumerate(probs)]
    m = gpu.MultiTask(L, N, D, probs[0].beta, K=K, T=T, U=U, tol=tol, seed=seed, mode="batched")
    for l in range(L):
        m.set_dictionary(l, _t(phis[l]))
    m.fit([_t(p.y) for p in probs])
    out = [m.posterior(l) for l in range(L)]
    m.close()
    ys = [p.y for p in probs]
    a_ref, mus, ss, steps = oracle.cofem_multitask(phis, ys, probs[0].beta, T=T, K=K, U=U, tol=tol, seed=seed)
    _, mus_t, _, _ = oracle.cofem_multitask(phis, ys, probs[0].beta, T=T, K=K, U=U, tol=tol / 100, seed=seed)
    totals = [out[l][3]["total_cg_steps"] for l in range(L)]
    print(f"CG steps per task: gpu {totals}, oracle {[sum(r[l] for r in steps) for l in range(L)]}")
    assert max(totals) >= 2 * min(totals)
    for l in range(L):
        bar = fp32_fit_bar(phis[l], probs[0].beta, [np.ones(D), a_ref])
        binds(f"multitask_batched_uneven/task{l}", _rel(mus[l], mus_t[l]), bar)
        check(f"multitask_batched_uneven/task{l}/mu", _rel(_np(out[l][0]), mus[l]), bar)
        check(f"multitask_batched_uneven/task{l}/s", _rel(_np(out[l][1]), ss[l]), 10 * bar)


def test_auto_mode_takes_batched_beyond_four_tasks(gpu):
    """The automatic choice: streams up to 4 tasks (the hardware queues a process gets by
    default), batched beyond, and streams whenever the batched form cannot take the
    settings (here a bf16 dictionary)."""
    for L, kw, want in ((4, {}, False), (5, {}, True), (8, dict(phi_dtype="bf16"), False)):
        m = gpu.MultiTask(L, 64, 256, 1e4, K=4, T=2, U=10, tol=1e-5, **kw)
        got = m.batched
        m.close()
        assert got == want, (L, kw)
