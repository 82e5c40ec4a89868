#!/usr/bin/env python3
"""CoFEM throughput on one MI355X.

One step = one whole fit (Algorithm 1) on the large dense Gaussian workload:
N = 16384, D = 65536, K = 32 probes, T = 30 EM iterations, PCG tol 1e-5, at
most 400 CG steps; the dictionary is held in bfloat16 (FP32 accumulation,
FP64 CG scalars) and the last 3 EM iterations use the FP32 dictionary.  A step
includes loading the dictionary into the library's layouts.  Inputs are
synthetic (seeded), already resident in HBM when the timed region starts.

Prints one JSON line.  `value` is EM iterations per second.  Beside it:
  roofline      the operator's matrix kernel (bf16), algorithmic bytes per
                launch / average launch time from HIP events on the library's
                stream over the timed steps, against 8 TB/s;
  fp32          the same fit with the FP32 dictionary throughout;
  cpu_baseline  the FP64 oracle on a bounded sample of the same workload;
  conv          the convolutional dictionary (D = 2^20 causal FIR, 256 taps,
                K = 20): EM iterations/s with bf16 taps (+ 3 FP32 iterations) and
                FP32, and the filter passes against the MFMA and HBM peaks;
  serving       the continuous-batching server on a stream of independent
                requests (D uniform in [512, 16384], N = D/4, 5 % spikes, sigma in
                {0.01, 0.05}, K = 16, T = 30, FP32): saturated request rate from a
                pilot batch, then Poisson arrivals at 0.8x that rate (the 512-request
                stream) and at 0.5x and 0.95x (shorter streams); p50/p99 latency from
                submission to completion; the serving contraction's dictionary bytes
                (CG steps x 2 passes x N D x 4 per request) over the device time of
                the ticks, against 8 TB/s.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "CoFEM EM-iters/s + HBM GB/s at D=65536 (BF16 vs FP32); serving p50/p99"


# HBM traffic of the bf16 operator kernel (k_gemm_bf16<4,2,2,true>) at N=16384, D=65536,
# from two rocprofv3 --pmc passes over `bench.py --pmc-probe` (FETCH_SIZE, then
# WRITE_SIZE; KiB per dispatch, averaged over 6 dispatches), each scaled by what the
# same counter reads for a plain 1 GiB device copy.  It holds only for the kernel
# source it was taken on: the hash covers the tile function and the launch shape choice.
GEMM_TRAFFIC = dict(src_sha="372cee0ad138146f", fetch_kib=1058560.4, write_kib=16913.4,
                    copy_kib=1048576.0, copy_fetch_kib=524302.4, copy_write_kib=1048576.0,
                    profile="profiles/hbm_traffic_k_gemm_bf16_dense_N16384_D65536.md")


def gemm_source_sha() -> str:
    """Hash of the sources the bf16 operator kernel is built from: its tile, its kernel
    wrapper, the tiling choice and launch code, and the dictionary row padding."""
    import hashlib

    csrc = os.path.join(ROOT, "paper_2105_10439_amd", "csrc")
    tiles = open(os.path.join(csrc, "tiles.h")).read()
    kern = open(os.path.join(csrc, "kernels.hip")).read()
    hdr = open(os.path.join(csrc, "kernels.h")).read()

    def cut(s, a, b):
        i = s.index(a)
        return s[i:s.index(b, i)]

    parts = [cut(tiles, "constexpr int GEMM_WAVES", "// FP32: v_mfma_f32_16x16x4_f32."),
             cut(kern, "template <int RT, int CT, int KS, bool X1>\n__global__ __launch_bounds__(64 * GEMM_WAVES, 2) "
                       "void k_gemm_bf16(", "\n}\n"),
             cut(kern, "GemmCfg choose_gemm(", "constexpr int KS_F32"),
             cut(kern, "static inline void gemm_cols(", "#define GEMM_F32("),
             cut(kern, "template <int RT>\nstatic void gemm_bf16_rt(", "template <int RT>\nstatic void gemm_f32_rt("),
             cut(hdr, "constexpr int64_t DICT_ROW_PAD_BYTES", "\n}")]
    return hashlib.sha256("".join(parts).encode()).hexdigest()[:16]


def gemm_traffic(N: int, D: int, dom: str):
    """Scaled HBM bytes per launch of the bf16 operator kernel, or None when the
    counters were not taken on this workload or on this kernel source."""
    g = GEMM_TRAFFIC
    if dom != "bf16" or (N, D) != (16384, 65536) or gemm_source_sha() != g["src_sha"]:
        return None
    rd = g["fetch_kib"] * (g["copy_kib"] / g["copy_fetch_kib"]) * 1024
    wr = g["write_kib"] * (g["copy_kib"] / g["copy_write_kib"]) * 1024
    return dict(total=rd + wr, read=rd, write=wr)


def stream_peaks():
    """Measured HBM rates on this GPU for context, best of 10, timed with events: a 1 GiB
    device copy (read + write bytes) and a read-only stream, the row sums of a 2 GiB FP32
    matrix of 16384 x 32768 (torch's reduction over the last dimension; read bytes only,
    the fastest read of the torch reductions tried: a full sum, a column sum, amax, a
    norm, a dot product and an FP32 matrix-vector product read at 3.7-5.6 TB/s)."""
    import torch

    n = (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    big = torch.ones(2 * n, dtype=torch.float32, device="cuda")
    res = {}
    rows = big.view(1 << 14, -1)
    for name, fn, nbytes in (("copy", lambda: b.copy_(a), 2 * 4 * n), ("read", lambda: rows.sum(1), 8 * n)):
        fn()
        best = None
        for _ in range(10):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        res[name] = round(nbytes / (best * 1e-3) / 1e9, 1)
    del a, b, big
    torch.cuda.empty_cache()
    return res


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large", choices=["large", "medium", "small"])
    ap.add_argument("--no-fp32", action="store_true", help="skip the all-FP32 comparison fit")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=12, help="CG steps in the oracle sample")
    ap.add_argument("--serve-requests", type=int, default=512, help="requests in the serving stream (0: skip)")
    ap.add_argument("--serve-pilot", type=int, default=32, help="requests of the saturation pilot")
    ap.add_argument("--serve-budget-gib", type=float, default=8.0)
    ap.add_argument("--serve-load", type=float, default=0.8, help="arrival rate as a fraction of saturation")
    ap.add_argument("--serve-side-loads", default="0.5,0.95",
                    help="further load points, as fractions of saturation ('' for none)")
    ap.add_argument("--serve-side-requests", type=int, default=160, help="requests per further load point")
    ap.add_argument("--no-conv", action="store_true", help="skip the convolutional-dictionary fits")
    ap.add_argument("--conv-only", action="store_true", help="only the convolutional-dictionary fits (for profiling)")
    ap.add_argument("--no-dct", action="store_true", help="skip the DCT-dictionary fits")
    ap.add_argument("--no-multitask", action="store_true", help="skip the multi-task fit")
    ap.add_argument("--multitask-only", action="store_true", help="only the multi-task fit (for profiling)")
    ap.add_argument("--dct-only", action="store_true", help="only the DCT-dictionary fits (for profiling)")
    ap.add_argument("--dct-fits", type=int, default=5, help="timed DCT-dictionary fits")
    ap.add_argument("--serve-only", action="store_true", help="only the serving phase (for profiling)")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="only run a 1 GiB copy and three operator applications (for rocprofv3 --pmc)")
    ap.add_argument("--pmc-probe-conv", action="store_true",
                    help="only run a 1 GiB copy and three bf16 FIR operator applications at D=2^20 "
                         "(for rocprofv3 --pmc)")
    ap.add_argument("--pmc-probe-dct", action="store_true",
                    help="only run ten DCT operator applications at D=2^15 and one fit with eager launches "
                         "(for rocprofv3 --pmc)")
    return ap.parse_args()


def pmc_probe():
    """Kernels for the HBM traffic counters: a plain 1 GiB device copy (known bytes,
    to calibrate FETCH_SIZE / WRITE_SIZE) and three applications of the bf16
    operator at the large size."""
    import numpy as np
    import torch

    import paper_2105_10439_amd as lib
    import workloads

    torch.cuda.set_device(0)
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    w = workloads.WORKLOADS["large"]
    prob = workloads.make_workload("large")
    m = lib.CoFEM(prob.N, prob.D, prob.beta, K=w["K"], T=w["T"], U=w["U"], tol=w["tol"], phi_dtype="bf16")
    m.set_dictionary(torch.from_numpy(prob.phi).cuda())
    rng = np.random.default_rng(0)
    P = torch.from_numpy(rng.standard_normal((w["K"] + 1, prob.D)).astype(np.float32)).cuda()
    al = torch.ones(prob.D, dtype=torch.float32, device="cuda")
    for _ in range(3):
        m.apply_A(al, P, use_bf16=True)
    torch.cuda.synchronize()
    m.close()
    log("pmc probe done")


def pmc_probe_conv():
    """As pmc_probe, for the FIR dictionary: the 1 GiB copy, then three applications of the
    bf16 operator at D = 2^20, 256 taps, K = 20 (one k_conv_bf16_op launch each, both filters
    with V in registers)."""
    import numpy as np
    import torch

    import paper_2105_10439_amd as lib
    import workloads

    torch.cuda.set_device(0)
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    w = workloads.WORKLOADS["conv"]
    prob = workloads.make_workload("conv")
    m = lib.CoFEM(prob.D, prob.D, prob.beta, K=w["K"], T=w["T"], U=w["U"], tol=w["tol"], op="conv",
                  conv_taps=prob.h.shape[0], phi_dtype="bf16")
    m.set_dictionary(torch.from_numpy(prob.h).cuda())
    rng = np.random.default_rng(0)
    P = torch.from_numpy(rng.standard_normal((w["K"] + 1, prob.D)).astype(np.float32)).cuda()
    al = torch.ones(prob.D, dtype=torch.float32, device="cuda")
    for _ in range(3):
        m.apply_A(al, P, use_bf16=True)
    torch.cuda.synchronize()
    m.close()
    log("pmc probe (FIR) done")


def pmc_probe_dct():
    """The DCT workload's kernels for the wave-state counters: ten applications of the split
    operator (three launches each) at D = 2^15, Q = 21, then one fit with per-launch events, so
    that its CG steps run as eager launches (the counters see every dispatch)."""
    import numpy as np
    import torch

    import paper_2105_10439_amd as lib
    import workloads

    torch.cuda.set_device(0)
    w = workloads.WORKLOADS["dct"]
    prob = workloads.make_workload("dct")
    m = lib.CoFEM(prob.N, prob.D, prob.beta, K=w["K"], T=w["T"], U=w["U"], tol=w["tol"], seed=2024, op="dct")
    m.set_dictionary(torch.from_numpy(prob.rows).cuda())
    rng = np.random.default_rng(0)
    P = torch.from_numpy(rng.standard_normal((w["K"] + 1, prob.D)).astype(np.float32)).cuda()
    al = torch.ones(prob.D, dtype=torch.float32, device="cuda")
    for _ in range(10):
        m.apply_A(al, P)
    torch.cuda.synchronize()
    m.set_timing(True)
    m.fit(torch.from_numpy(prob.y).cuda())
    torch.cuda.synchronize()
    m.close()
    log("pmc probe (DCT) done")


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; run with --gpus 1 (multi-GPU sharding is a design, not an implementation)"}))
        sys.exit(2)
    if args.pmc_probe:
        pmc_probe()
        return
    if args.pmc_probe_conv:
        pmc_probe_conv()
        return
    if args.pmc_probe_dct:
        pmc_probe_dct()
        return
    if args.serve_only:
        import torch

        torch.cuda.set_device(0)
        print(json.dumps({"serving": serving(args)}), flush=True)
        return
    if args.conv_only:
        import torch

        torch.cuda.set_device(0)
        print(json.dumps({"conv": conv_bench()}), flush=True)
        return
    if args.dct_only:
        import torch

        torch.cuda.set_device(0)
        print(json.dumps({"dct": dct_bench(args.dct_fits)}), flush=True)
        return
    if args.multitask_only:
        import torch

        torch.cuda.set_device(0)
        print(json.dumps({"multitask": multitask_bench()}), flush=True)
        return
    import numpy as np
    import torch

    import paper_2105_10439_amd as lib
    import workloads

    lib.load()
    torch.cuda.set_device(0)
    w = dict(workloads.WORKLOADS[args.workload])
    refine = 3 if args.workload == "large" else 0
    t0 = time.time()
    prob = workloads.make_workload(args.workload)
    log(f"generated {args.workload} N={prob.N} D={prob.D} in {time.time() - t0:.1f}s")
    phi_d = torch.from_numpy(prob.phi).cuda()
    y_d = torch.from_numpy(prob.y).cuda()
    torch.cuda.synchronize()

    def run(phi_dtype, refine_last, steps, warmup, timing, var_batches=0, theta="ones"):
        m = lib.CoFEM(prob.N, prob.D, prob.beta, K=w["K"], T=w["T"], U=w["U"], tol=w["tol"], seed=2024,
                      phi_dtype=phi_dtype, refine_last=refine_last, theta=theta)
        for i in range(warmup):
            m.set_dictionary(phi_d)
            m.fit(y_d)
            log(f"warmup {i + 1}/{warmup} done")
        if timing:
            m.set_timing(True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(steps):
            m.set_dictionary(phi_d)
            m.fit(y_d)
            log(f"step {i + 1}/{steps} done")
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        mu, s, alpha, st = m.posterior()
        tim = {k: m.get_timing(k) for k in ("bf16", "fp32")} if timing else None
        var = None
        if var_batches:
            m.set_timing(False)
            torch.cuda.synchronize()
            tv = time.perf_counter()
            _, _, vst = m.variance(var_batches, seed=7)
            torch.cuda.synchronize()
            ev = time.perf_counter() - tv
            var = dict(batches=var_batches, probes=var_batches * w["K"], ms=round(1e3 * ev, 1),
                       cg_steps=vst["cg_steps"], operator="fp32" if not vst["used_bf16"][0] else "bf16")
            log(f"post-fit variance: {var}")
        m.close()
        run.var = var
        return el, st, tim, mu

    el, st, tim, mu = run("bf16" if args.workload == "large" else "fp32", refine, args.steps, args.warmup, True,
                          var_batches=2)
    em_iters = w["T"] * args.steps
    value = em_iters / el
    nbytes_launch = {"bf16": prob.N * prob.D * 2, "fp32": prob.N * prob.D * 4}
    ops = {}
    for k, (ms, n) in tim.items():
        if n:
            avg_ms = ms / n
            ops[k] = dict(launches=n, avg_ms=avg_ms, gbps=nbytes_launch[k] / (avg_ms * 1e-3) / 1e9)
    dom = "bf16" if "bf16" in ops else "fp32"
    traf = gemm_traffic(prob.N, prob.D, dom)
    roof = dict(bound="hbm", achieved=round(ops[dom]["gbps"], 1), peak=HBM_PEAK_GBPS, unit="GB/s",
                frac=round(ops[dom]["gbps"] / HBM_PEAK_GBPS, 4), traffic=round(traf["total"]) if traf else None,
                kernel=f"k_gemm_{dom}", bytes_per_launch=nbytes_launch[dom], avg_launch_ms=ops[dom]["avg_ms"])
    if traf:
        roof.update(traffic_read=round(traf["read"]), traffic_write=round(traf["write"]),
                    traffic_over_algorithmic=round(traf["total"] / nbytes_launch[dom], 4))
    peaks = stream_peaks()
    roof.update(measured_copy_gbps=peaks["copy"], frac_of_measured_copy=round(ops[dom]["gbps"] / peaks["copy"], 4),
                measured_read_gbps=peaks["read"], frac_of_measured_read=round(ops[dom]["gbps"] / peaks["read"], 4))
    log(f"measured stream rates: {peaks}")
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "EM-iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * el / args.steps, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16" if refine else "fp32", "data": "synthetic",
        "config": {"workload": f"dense Gaussian {args.workload}: N={prob.N} D={prob.D} K={w['K']} T={w['T']} "
                               f"tol={w['tol']} U={w['U']}" + (f" bf16 dictionary, last {refine} EM iterations FP32"
                                                               if refine else " FP32"),
                   "N": prob.N, "D": prob.D, "K": w["K"], "T": w["T"]},
        "roofline": roof,
        "operator": ops,
        "cg_steps_per_fit": st["total_cg_steps"],
        "cg_steps_per_em_iter": st["cg_steps"],
        "posterior_variance": run.var,
        "arithmetic": "operator: bf16 (or FP32) dictionary, FP32 accumulation; CG dot products, gamma, eta, rho, pi "
                      "and the stop test in FP64; X, R, P, Psi stored in FP32, their element-wise updates "
                      "computed in FP64 with the FP64 step scalars and rounded to FP32 once (an all-FP32 form "
                      "measured less accurate at no speed gain)",
    }
    if not args.no_fp32 and args.workload == "large":
        el32, st32, tim32, mu32 = run("fp32", 0, 1, 0, True)
        ms, n = tim32["fp32"]
        out["fp32"] = dict(em_iters_per_s=round(w["T"] / el32, 3), ms_per_fit=round(1e3 * el32, 1),
                           cg_steps=st32["total_cg_steps"],
                           operator_gbps=round(nbytes_launch["fp32"] / (ms / n * 1e-3) / 1e9, 1) if n else None,
                           mu_rel_diff_bf16_refined_vs_fp32=float(
                               (torch.linalg.vector_norm(mu.double() - mu32.double()) /
                                torch.linalg.vector_norm(mu32.double())).item()))
        log(f"fp32 comparison fit: {out['fp32']}")
    if args.workload == "large":
        # the Jacobi preconditioner of Sec. III-C (theta_j = ||Phi_:j||^2) beside the default theta = 1
        elj, stj, _, _ = run("bf16", refine, 1, 0, False, theta="jacobi")
        out["jacobi"] = dict(em_iters_per_s=round(w["T"] / elj, 3), cg_steps=stj["total_cg_steps"],
                             cg_steps_per_em_iter=stj["cg_steps"], theta_ones_cg_steps=st["total_cg_steps"])
        log(f"jacobi fit: {out['jacobi']}")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, w, st, args.cpu_steps)
    del phi_d, y_d, prob
    torch.cuda.empty_cache()
    if not args.no_conv:
        out["conv"] = conv_bench()
    if not args.no_dct:
        out["dct"] = dct_bench(args.dct_fits)
    if not args.no_multitask:
        out["multitask"] = multitask_bench()
    if args.serve_requests > 0:
        out["serving"] = serving(args)
    print(json.dumps(out), flush=True)


def conv_bench():
    """The convolutional dictionary (D = 2^20 causal FIR, 256 taps): one warm-up and
    one timed fit with bf16 taps and the last 3 EM iterations on FP32 taps, one timed
    all-FP32 fit, and one timed bf16-refined fit with the non-negative M-step of
    Sec. III-E.2 (the model of the calcium-deconvolution application); NRMSE of mu
    against the true spikes for each.  Per operator application: algorithmic flops
    4 L D Q (Q = K + 1 real columns) against the MFMA peak of the dtype, and algorithmic
    bytes against 8 TB/s: FP32, two filter launches moving 20 D Q + 4 D bytes (pass 1
    reads Pd and writes V, pass 2 reads V, Pd, alpha and writes Psi); bf16, one launch
    with V kept in registers, 8 D Q + 4 D bytes (Pd as its hi/lo pair, alpha, Psi)."""
    import torch

    import paper_2105_10439_amd as lib
    import workloads

    w = dict(workloads.WORKLOADS["conv"])
    prob = workloads.make_workload("conv")
    L, D, Q = prob.h.shape[0], prob.D, w["K"] + 1
    h_d = torch.from_numpy(prob.h).cuda()
    y_d = torch.from_numpy(prob.y).cuda()
    flops_app = 4.0 * L * D * Q
    # FP32: two filter launches, pass 1 reads Pd and writes V, pass 2 reads V, Pd and alpha
    # and writes Psi; bf16: one launch with V in registers, reading Pd's hi/lo pair and alpha
    # and writing Psi (the epilogue takes Pd from the causal filter's window)
    bytes_app = {"fp32": 20.0 * D * Q + 4.0 * D, "bf16": 8.0 * D * Q + 4.0 * D}
    per_app = {"fp32": 2, "bf16": 1}
    peak = {"bf16": 2500.0, "fp32": 157.3}
    res = dict(workload=f"causal FIR dictionary: D=N={D}, {L} taps of exp(-t/{w['tau']:g}), Bernoulli({w['p']})*Exp(1) "
                        f"spikes, sigma={w['sigma']}, K={w['K']} T={w['T']} tol={w['tol']} U={w['U']}",
               signal_storage="bf16 forms: taps rounded to bf16; the direction P travels as its hi/lo bf16 "
                              "pair (4 bytes per value, the bytes of FP32) and V = Phi P stays in registers in "
                              "the one-launch operator, so the bf16 gain is the matrix rate and the V round trip, "
                              "not halved signal bytes (a 2-byte signal form measured no net gain in emulation)")
    z = torch.from_numpy(prob.z)
    for name, dt, refine, mstep, theta in (("bf16_refined", "bf16", 3, "gaussian", "ones"),
                                           ("fp32", "fp32", 0, "gaussian", "ones"),
                                           ("bf16_refined_nonneg", "bf16", 3, "nonneg", "ones"),
                                           ("bf16_refined_jacobi", "bf16", 3, "gaussian", "jacobi")):
        m = lib.CoFEM(D, D, prob.beta, K=w["K"], T=w["T"], U=w["U"], tol=w["tol"], seed=2024, op="conv",
                      conv_taps=L, phi_dtype=dt, refine_last=refine, mstep=mstep, theta=theta)
        if dt == "bf16":
            m.set_dictionary(h_d)
            m.fit(y_d)
        m.set_timing(True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        m.set_dictionary(h_d)
        m.fit(y_d)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        mu, _, _, st = m.posterior()
        nrmse = float(torch.linalg.vector_norm(mu.double().cpu() - z) / torch.linalg.vector_norm(z))
        passes = {}
        for k in ("bf16", "fp32"):
            ms, n = m.get_timing(k)
            if n:
                app_s = per_app[k] * ms / n * 1e-3
                passes[k] = dict(launches=n, launches_per_application=per_app[k],
                                 avg_launch_us=round(1e3 * ms / n, 1), us_per_application=round(1e6 * app_s, 1),
                                 tflops=round(flops_app / app_s / 1e12, 1),
                                 mfma_frac=round(flops_app / app_s / 1e12 / peak[k], 4),
                                 algorithmic_bytes=bytes_app[k], gbps=round(bytes_app[k] / app_s / 1e9, 1),
                                 hbm_frac=round(bytes_app[k] / app_s / 1e9 / HBM_PEAK_GBPS, 4))
        m.close()
        res[name] = dict(em_iters_per_s=round(w["T"] / el, 3), ms_per_fit=round(1e3 * el, 1),
                         cg_steps=st["total_cg_steps"], ms_per_cg_step=round(1e3 * el / st["total_cg_steps"], 4),
                         nrmse=round(nrmse, 4), passes=passes)
        res[name]["cg_steps_per_em_iter"] = st["cg_steps"]
        log(f"conv {name}: {res[name]}")
    return res


def multitask_bench():
    """Multi-task CoFEM (Sec. III-E.1): L = 4 tasks of the medium shape (N = 2048,
    D = 8192, FP32 dictionaries, 64 MiB each) sharing one support of 5 % spikes, K = 20,
    T = 30, tol 1e-5: one warm-up and one timed fit in each form, batched (all tasks'
    systems in one launch per phase) and streams (one context per task on its own stream;
    the automatic choice at L = 4 and the reported value); then both forms on 32 smaller
    tasks (N = 512, D = 2048), where the streams no longer fit the hardware queues.  The value is shared-alpha EM iterations per
    second (each = L covariance-free E-steps and one joint M-step)."""
    import torch

    import paper_2105_10439_amd as lib
    import workloads

    w = dict(workloads.WORKLOADS["multitask"])
    probs = workloads.make_workload("multitask")
    L, N, D = w["L"], w["N"], w["D"]
    phis = [torch.from_numpy(p.phi).cuda() for p in probs]
    ys = [torch.from_numpy(p.y).cuda() for p in probs]

    def one(mode):
        m = lib.MultiTask(L, N, D, probs[0].beta, K=w["K"], T=w["T"], U=w["U"], tol=w["tol"], seed=2024, mode=mode)
        for l in range(L):
            m.set_dictionary(l, phis[l])
        m.fit(ys)
        torch.cuda.synchronize()
        t = time.perf_counter()
        m.fit(ys)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        steps, nrmse = [], []
        for l in range(L):
            mu, _, _, st = m.posterior(l)
            steps.append(st["total_cg_steps"])
            z = torch.from_numpy(probs[l].z)
            nrmse.append(round(float(torch.linalg.vector_norm(mu.double().cpu() - z) / torch.linalg.vector_norm(z)), 4))
        m.close()
        return el, steps, nrmse

    el, steps, nrmse = one("batched")
    el_s, steps_s, nrmse_s = one("streams")
    # many small tasks: L = 32 of N = 512, D = 2048 (same recipe, same K, T, tol)
    many = {}
    Lm, Nm, Dm = 32, 512, 2048
    mprobs = workloads.multitask_problems(Lm, N=Nm, D=Dm, d=Dm // 20, sigma=w["sigma"], seed=w["seed"] + 1)
    mphis = [torch.from_numpy(p.phi).cuda() for p in mprobs]
    mys = [torch.from_numpy(p.y).cuda() for p in mprobs]
    for mode in ("batched", "streams"):
        m = lib.MultiTask(Lm, Nm, Dm, mprobs[0].beta, K=w["K"], T=w["T"], U=w["U"], tol=w["tol"], seed=2024,
                          mode=mode)
        for l in range(Lm):
            m.set_dictionary(l, mphis[l])
        m.fit(mys)
        torch.cuda.synchronize()
        t = time.perf_counter()
        m.fit(mys)
        torch.cuda.synchronize()
        el_m = time.perf_counter() - t
        m.close()
        many[mode] = round(w["T"] / el_m, 3)
    op_bytes = 2.0 * N * D * 4 * sum(steps)  # two FP32 dictionary passes per CG step of each task
    auto = "batched" if L > 4 else "streams"  # cofem_mt_create's automatic choice
    el_a = el if auto == "batched" else el_s
    res = dict(workload=f"multi-task dense: L={L} tasks of N={N} D={D}, shared support of {w['d']} spikes, "
                        f"sigma={w['sigma']}, K={w['K']} T={w['T']} tol={w['tol']} U={w['U']}, FP32",
               form=auto, em_iters_per_s=round(w["T"] / el_a, 3), ms_per_fit=round(1e3 * el_a, 1),
               batched=dict(em_iters_per_s=round(w["T"] / el, 3), ms_per_fit=round(1e3 * el, 1),
                            cg_steps_per_task=steps, ms_per_cg_step=round(1e3 * el / max(steps), 4),
                            nrmse_per_task=nrmse, dictionary_gbps_whole_fit=round(op_bytes / el / 1e9, 1)),
               streams=dict(em_iters_per_s=round(w["T"] / el_s, 3), ms_per_fit=round(1e3 * el_s, 1),
                            cg_steps_per_task=steps_s, nrmse_per_task=nrmse_s),
               many_tasks=dict(workload=f"L={Lm} tasks of N={Nm} D={Dm}, {Dm // 20} shared spikes, same settings",
                               em_iters_per_s_batched=many["batched"], em_iters_per_s_streams=many["streams"]),
               note="ms_per_cg_step: fit time over the most CG steps of any task (the tasks advance "
                    "together); dictionaries (4 x 64 MiB) and their transposed copies are 512 MiB, about "
                    "twice the 256 MB Infinity Cache")
    log(f"multitask: {res}")
    return res


def dct_bench(fits):
    """The subsampled DCT dictionary at the largest DCT size of the paper's scalability
    study (D = 2^15, N = D/3, d = 0.12 D spikes, K = 20, T = 30, U = 400, tol 1e-4):
    one warm-up fit, then `fits` timed fits (sample set loaded once per fit), then one fit
    with per-launch events for the operator's own time.  Per
    operator application (Q = K + 1 columns): algorithmic bytes 8 D Q + 4 D (read Pd
    and alpha, write Psi), and the conventional 5 L log2 L flops of each of the 2 Q
    complex FFTs of length L = D / 2."""
    import math

    import torch

    import paper_2105_10439_amd as lib
    import workloads

    w = dict(workloads.WORKLOADS["dct"])
    prob = workloads.make_workload("dct")
    D, N, Q = prob.D, prob.N, w["K"] + 1
    L = D // 2
    rows_d = torch.from_numpy(prob.rows).cuda()
    y_d = torch.from_numpy(prob.y).cuda()
    bytes_app = 8.0 * D * Q + 4.0 * D
    flops_app = 2.0 * Q * 5.0 * L * math.log2(L)
    m = lib.CoFEM(N, D, prob.beta, K=w["K"], T=w["T"], U=w["U"], tol=w["tol"], seed=2024, op="dct")
    m.set_dictionary(rows_d)
    m.fit(y_d)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(fits):
        m.set_dictionary(rows_d)
        m.fit(y_d)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    mu, _, _, st = m.posterior()
    # the operator's launches timed with events in one more fit (kept out of the fit timing:
    # at ~27 us per application the event pairs are a visible share of a CG step)
    m.set_timing(True)
    m.fit(y_d)
    ms, n = m.get_timing("fp32")
    m.close()
    app_s = ms / n * 1e-3
    nrmse = float(torch.linalg.vector_norm(mu.double().cpu() - torch.from_numpy(prob.z)) /
                  torch.linalg.vector_norm(torch.from_numpy(prob.z)))
    res = dict(workload=f"subsampled DCT dictionary: D={D}, N={N} kept samples, {prob.meta['d']} spikes N(0,5), "
                        f"sigma={w['sigma']}, K={w['K']} T={w['T']} tol={w['tol']} U={w['U']}, FP32",
               em_iters_per_s=round(w["T"] * fits / el, 2), ms_per_fit=round(1e3 * el / fits, 2),
               cg_steps=st["total_cg_steps"], ms_per_cg_step=round(1e3 * el / fits / st["total_cg_steps"], 4),
               nrmse=round(nrmse, 4),
               operator=dict(launches=n, avg_us=round(1e6 * app_s, 2), gbps=round(bytes_app / app_s / 1e9, 1),
                             hbm_frac=round(bytes_app / app_s / 1e9 / HBM_PEAK_GBPS, 4),
                             fft_tflops=round(flops_app / app_s / 1e12, 3)),
               paper_context="the paper reports about 2 s per CoFEM fit at this size on an NVIDIA T4 (Sec. V-C)")
    log(f"dct: {res}")
    return res


SERVE_KW = dict(K=16, T=30, U=400, tol=1e-5)


class Prepared:
    """Generates request inputs in arrival order on a background thread, a bounded
    number ahead (NumPy releases the GIL while it fills the arrays)."""

    def __init__(self, descs, ahead=48):
        import queue
        import threading

        import workloads

        self.q = queue.Queue(maxsize=ahead)

        def run():
            for d in descs:
                self.q.put((d, workloads.serving_request(d)))

        self.t = threading.Thread(target=run, daemon=True)
        self.t.start()

    def get(self, block=True):
        import queue

        try:
            return self.q.get(block=block)
        except queue.Empty:
            return None


def serving(args):
    import numpy as np

    import paper_2105_10439_amd as lib
    import workloads

    budget = int(args.serve_budget_gib * (1 << 30))
    descs = workloads.serving_stream(args.serve_requests, seed=4242)

    def submit(srv, d, p):
        return srv.submit(p.phi, p.y, beta=p.beta, seed=d["seed"], **SERVE_KW)

    def drain(srv, ids, done):
        for rid in ids:
            if rid not in done:
                r = srv.result(rid)
                if r is not None:
                    done[rid] = r[3]

    # 1. saturated rate: a pilot batch submitted at once
    pilot = descs[:min(args.serve_pilot, len(descs))]
    prep = Prepared(pilot)
    items = [prep.get() for _ in pilot]
    srv = lib.Server(budget, max_slots=128, steps_per_tick=4)
    t0 = time.perf_counter()
    ids = [submit(srv, d, p) for d, p in items]
    done = {}
    while len(done) < len(ids):
        srv.step()
        drain(srv, ids, done)
    sat_s = time.perf_counter() - t0
    sat_rps = len(ids) / sat_s
    srv.close()
    del items
    log(f"serving pilot: {len(ids)} requests in {sat_s:.2f}s = {sat_rps:.2f} req/s")

    # 2. Poisson arrivals at fractions of saturation
    def stream(load, descs, seed):
        rate = load * sat_rps
        arrivals = workloads.poisson_arrivals(len(descs), rate, seed=seed)
        prep = Prepared(descs)
        srv = lib.Server(budget, max_slots=128, steps_per_tick=4)
        ids, done = [], {}
        nxt = prep.get()
        k = 0
        late = 0.0
        t0 = time.perf_counter()
        last_log = t0
        while len(done) < len(descs):
            now = time.perf_counter() - t0
            while nxt is not None and k < len(descs) and arrivals[k] <= now:
                late = max(late, now - arrivals[k])
                ids.append(submit(srv, *nxt))
                k += 1
                nxt = prep.get() if k < len(descs) else None
            running, pending = srv.step()
            drain(srv, ids, done)
            if running == 0 and pending == 0 and k < len(descs):
                time.sleep(max(0.0, min(0.002, arrivals[k] - (time.perf_counter() - t0))))
            if time.perf_counter() - last_log > 10:
                last_log = time.perf_counter()
                log(f"serving at {load}x: {len(done)}/{len(descs)} done, {running} running, {pending} pending")
        el = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        lat = np.array([inf["t_finish_ms"] - inf["t_submit_ms"] for inf in done.values()])
        steps = sum(inf["total_cg_steps"] for inf in done.values())
        gbps = st["dict_bytes"] / (st["tick_ms"] * 1e-3) / 1e9
        res = dict(load=load, requests=len(descs), arrival_rps=round(rate, 3),
                   throughput_rps=round(len(descs) / el, 3), em_iters_per_s=round(len(descs) * SERVE_KW["T"] / el, 2),
                   p50_ms=round(float(np.percentile(lat, 50)), 2), p99_ms=round(float(np.percentile(lat, 99)), 2),
                   mean_ms=round(float(lat.mean()), 2), max_active=st["max_active"], ticks=st["ticks"],
                   cg_steps_total=int(steps), max_submit_delay_ms=round(1e3 * late, 1),
                   bytes_peak_gib=round(st["bytes_peak"] / (1 << 30), 3),
                   tick_device_s=round(st["tick_ms"] * 1e-3, 2), busy_frac=round(st["tick_ms"] * 1e-3 / el, 3),
                   dict_gbps_over_ticks=round(gbps, 1))
        log(f"serving at {load}x: {res}")
        return res

    main_pt = stream(args.serve_load, descs, 777)
    side = []
    for i, ld in enumerate(float(x) for x in args.serve_side_loads.split(",") if x.strip()):
        side.append(stream(ld, descs[:min(args.serve_side_requests, len(descs))], 778 + i))
    res = dict(main_pt, workload="dense Gaussian requests, D uniform in [512, 16384], N = D/4, 5% spikes, "
                                 "sigma in {0.01, 0.05}, K=16, T=30, tol=1e-5, FP32",
               budget_gib=args.serve_budget_gib, saturated_rps=round(sat_rps, 3))
    res["roofline"] = dict(bound="hbm", kernel="serving tick (ks_gemm and the vector kernels)",
                           achieved=main_pt["dict_gbps_over_ticks"], peak=HBM_PEAK_GBPS, unit="GB/s",
                           frac=round(main_pt["dict_gbps_over_ticks"] / HBM_PEAK_GBPS, 4),
                           note="dictionary bytes of the completed fits' CG steps (2 passes x N D x 4 each) over "
                                "the device time of every tick, so the other kernels of a tick count against it")
    res["load_points"] = [dict((k, p[k]) for k in ("load", "requests", "arrival_rps", "throughput_rps", "p50_ms",
                                                   "p99_ms", "max_active", "dict_gbps_over_ticks"))
                          for p in sorted([main_pt] + side, key=lambda p: p["load"])]
    return res


def cpu_baseline(prob, w, st, cg_steps):
    """The FP64 oracle on a bounded sample: one E-step capped at `cg_steps` CG
    steps (tol = 0 so it runs them all), scaled to EM iterations/s with the
    oracle's own mean CG steps per EM iteration on this workload (from its stored
    full fit, tests/golden/large_oracle.npz), or the GPU fit's when that is absent."""
    import numpy as np

    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    op = oracle.DenseOperator(prob.phi)
    t_conv = time.perf_counter() - t0
    t1 = time.perf_counter()
    oracle.cofem(op, prob.y, prob.beta, T=1, K=w["K"], U=cg_steps, tol=0.0, seed=2024)
    el = time.perf_counter() - t1
    per_step = el / cg_steps
    golden = os.path.join(ROOT, "tests", "golden", "large_oracle.npz")
    if prob.N == 16384 and prob.D == 65536 and os.path.exists(golden):
        g = np.load(golden)
        mean_steps = float(g["cg_steps"].mean())
        whose = f"the oracle's own mean {mean_steps:.1f} CG steps per EM iteration (its stored full fit)"
    else:
        mean_steps = st["total_cg_steps"] / max(st["T"], 1)
        whose = f"the GPU fit's mean {mean_steps:.1f} CG steps per EM iteration"
    v = 1.0 / (per_step * mean_steps)
    log(f"cpu baseline: {cg_steps} CG steps in {el:.1f}s ({per_step:.3f}s/step), widening {t_conv:.1f}s")
    return dict(value=round(v, 5), unit="EM-iters/s", cores=threads, kind="oracle",
                sample=f"one E-step of the same workload capped at {cg_steps} CG steps ({el:.1f}s), scaled by "
                       f"{whose}; NumPy FP64 with {threads} BLAS threads")


if __name__ == "__main__":
    main()
