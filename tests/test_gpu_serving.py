"""GPU tests of the continuous-batching server (cofem_server_*).

* a request's result is bitwise the same alone and in a mix of requests of other
  sizes, submitted at different times (each fit's arithmetic is independent of
  the batch and its reductions run in a fixed order);
* a served fit matches the FP64 oracle to the same bar as a single fit;
* admission never exceeds the memory budget; a request larger than the whole
  budget is rejected;
* requests that arrive while others run are admitted and overlap with them;
* cancelling a pending or a running request frees its queue place, slot and bytes
  at once and leaves the other requests' results bitwise unchanged;
* an observation with a NaN is rejected at submission.
"""
import numpy as np
import pytest

import oracle
import workloads
from bars import check

pytestmark = pytest.mark.gpu

GiB = 1 << 30


def _req(D, seed, sigma=0.01, frac=0.05):
    N = max(D // 4, 1)
    return workloads.dense_problem(N, D, max(int(frac * D), 1), sigma, seed)


def _run(gpu, probs, kw, budget=4 * GiB, max_slots=16, stagger=0, steps=4):
    srv = gpu.Server(budget, max_slots=max_slots, steps_per_tick=steps)
    ids = []
    queue = list(probs)
    ticks = 0
    out = {}
    while queue or len(out) < len(probs):
        # submit one request every `stagger` ticks (all at once when 0)
        while queue and (stagger == 0 or ticks % stagger == 0):
            p = queue.pop(0)
            ids.append(srv.submit(p.phi, p.y, beta=p.beta, **kw))
            if stagger:
                break
        srv.step()
        ticks += 1
        for i, rid in enumerate(ids):
            if i not in out:
                r = srv.result(rid)
                if r is not None:
                    out[i] = r
        assert ticks < 100000
    stats = srv.stats()
    srv.close()
    return [out[i] for i in range(len(probs))], stats


def test_alone_equals_mix_bitwise(gpu):
    sizes = [300, 512, 777, 1024, 1500, 2048]
    probs = [_req(D, 50 + i) for i, D in enumerate(sizes)]
    kw = dict(K=16, T=8, U=300, tol=1e-5, seed=99)
    mixed, st = _run(gpu, probs, kw, stagger=3)
    assert st["max_active"] >= 2
    for i, p in enumerate(probs):
        alone, _ = _run(gpu, [p], kw)
        for a, b in zip(alone[0][:3], mixed[i][:3]):
            assert np.array_equal(a, b), f"request {i} (D={p.D}) differs alone vs mixed"
        assert alone[0][3]["total_cg_steps"] == mixed[i][3]["total_cg_steps"]


@pytest.mark.parametrize("K", [8, 16])
def test_served_fit_matches_oracle(gpu, K):
    # K = 16 runs the 17th column on the vector ALU
    w = dict(workloads.WORKLOADS["small"], K=K)
    prob = workloads.make_workload("small")
    kw = dict(K=w["K"], T=w["T"], U=w["U"], tol=w["tol"], seed=1234)
    (res,), _ = _run(gpu, [prob], kw)
    mu, s = res[0].astype(np.float64), res[1].astype(np.float64)
    ref = oracle.cofem(prob.phi, prob.y, prob.beta, T=w["T"], K=w["K"], U=w["U"], tol=w["tol"], seed=1234)
    e_mu = np.linalg.norm(mu - ref.mu) / np.linalg.norm(ref.mu)
    e_s = np.linalg.norm(s - ref.s) / np.linalg.norm(ref.s)
    check(f"served_small_K{K}/mu", e_mu, 1e-4)
    check(f"served_small_K{K}/s", e_s, 1e-3)


def test_budget_is_never_exceeded(gpu):
    probs = [_req(D, 70 + i) for i, D in enumerate([2048, 1800, 2048, 1900, 2048, 1700])]
    kw = dict(K=16, T=4, U=200, tol=1e-5, seed=5)
    # measure one request's workspace, then give the server room for two of them
    probe = gpu.Server(1 * GiB, max_slots=1, steps_per_tick=1)
    one = probe.info(probe.submit(probs[0].phi, probs[0].y, beta=probs[0].beta, **kw))["bytes"]
    probe.close()
    budget = int(2.5 * one)
    srv = gpu.Server(budget, max_slots=8, steps_per_tick=4)
    ids = [srv.submit(p.phi, p.y, beta=p.beta, **kw) for p in probs]
    done = set()
    peak = 0
    for _ in range(100000):
        srv.step()
        st = srv.stats()
        peak = max(peak, st["bytes_in_use"])
        assert st["bytes_in_use"] <= st["budget"]
        for rid in ids:
            if rid not in done and srv.result(rid) is not None:
                done.add(rid)
        if len(done) == len(ids):
            break
    st = srv.stats()
    assert st["bytes_peak"] <= st["budget"] and st["completed"] == len(ids)
    assert st["max_active"] >= 2
    # larger than the whole budget: rejected at submit
    big = _req(8192, 3)
    with pytest.raises(gpu.CofemError) as e:
        srv.submit(big.phi, big.y, beta=big.beta, **kw)
    assert e.value.status == -6
    with pytest.raises(gpu.CofemError) as e:
        srv.submit(big.phi, big.y, beta=big.beta, K=40, T=4, U=10, tol=1e-5)
    assert e.value.status == -1
    srv.close()


def test_arrivals_overlap_running_requests(gpu):
    probs = [_req(D, 90 + i) for i, D in enumerate([4096, 1024, 2048, 3072])]
    kw = dict(K=16, T=10, U=300, tol=1e-5, seed=7)
    srv = gpu.Server(4 * GiB, max_slots=8, steps_per_tick=2)
    first = srv.submit(probs[0].phi, probs[0].y, beta=probs[0].beta, **kw)
    srv.step()
    srv.step()
    assert srv.info(first)["state"] == "running"
    later = [srv.submit(p.phi, p.y, beta=p.beta, **kw) for p in probs[1:]]
    infos = {}
    for _ in range(100000):
        srv.step()
        for rid in [first] + later:
            if rid not in infos:
                inf = srv.info(rid)
                if inf["state"] == "done":
                    infos[rid] = inf
        if len(infos) == len(probs):
            break
    # the later requests were admitted while the first was still running
    assert all(infos[r]["t_admit_ms"] < infos[first]["t_finish_ms"] for r in later)
    assert srv.stats()["max_active"] == len(probs)
    srv.close()


def test_cancel_pending_and_running_requests(gpu):
    probs = [_req(D, 80 + i) for i, D in enumerate([700, 900, 1100, 1300])]
    kw = dict(K=8, T=6, U=300, tol=1e-5, seed=17)
    alone = [_run(gpu, [p], kw)[0][0] for p in (probs[0], probs[3])]
    srv = gpu.Server(GiB, max_slots=2, steps_per_tick=2)
    ids = [srv.submit(p.phi, p.y, beta=p.beta, **kw) for p in probs]
    srv.step()                                   # two slots: requests 0 and 1 run, 2 and 3 wait
    assert [srv.info(r)["state"] for r in ids] == ["running", "running", "pending", "pending"]
    before = srv.stats()["bytes_in_use"]
    b1 = srv.info(ids[1])["bytes"]
    srv.cancel(ids[1])                           # running: its slot and bytes come back at once
    assert srv.stats()["bytes_in_use"] == before - b1
    srv.cancel(ids[2])                           # pending: leaves the queue
    for r in (ids[1], ids[2]):
        with pytest.raises(gpu.CofemError) as e:
            srv.info(r)
        assert e.value.status == -1
    out = {}
    for _ in range(100000):
        srv.step()
        for i in (0, 3):
            if i not in out:
                res = srv.result(ids[i])
                if res is not None:
                    out[i] = res
        if len(out) == 2:
            break
    st = srv.stats()
    srv.close()
    assert st["completed"] == 2 and st["bytes_in_use"] == 0 and st["admitted"] == 3
    for k, i in enumerate((0, 3)):
        for a, b in zip(out[i][:3], alone[k][:3]):
            assert np.array_equal(a, b), f"request {i} changed by the cancellations"


def test_submit_rejects_non_finite_observation(gpu):
    p = _req(512, 5)
    y = p.y.copy()
    y[7] = np.nan
    srv = gpu.Server(GiB, max_slots=2)
    with pytest.raises(gpu.CofemError) as e:
        srv.submit(p.phi, y, beta=p.beta, K=8, T=2, U=10, tol=1e-5)
    assert e.value.status == -1 and "y[7]" in str(e.value)
    assert srv.stats()["rejected"] == 1
    srv.close()


def test_stats_count_dictionary_bytes_and_tick_time(gpu):
    """The serving roofline's inputs: dict_bytes is the algorithmic dictionary traffic of the
    completed fits (each CG step reads the N x D FP32 dictionary twice) and tick_ms the device
    time of the ticks."""
    probs = [_req(D, 90 + i) for i, D in enumerate([600, 1000, 1400])]
    kw = dict(K=8, T=4, U=200, tol=1e-5, seed=23)
    res, st = _run(gpu, probs, kw, budget=GiB, max_slots=4)
    expect = sum(r[3]["total_cg_steps"] * 2.0 * p.N * p.D * 4 for r, p in zip(res, probs))
    assert st["dict_bytes"] == expect
    assert st["tick_ms"] > 0.0 and st["ticks"] > 0
