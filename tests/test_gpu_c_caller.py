"""The C ABI from a plain C program: `tests/c/fit_smoke.c` (C99, built by the package
build step with gcc against include/cofem.h, libcofem.so and the HIP runtime, no
Python binding in the loop) fits the small dense workload; its mu and s are
compared with the FP64 oracle at the same probes, stop rule and tolerance, to the
same bar as the Python-driven fits: 1e-4 (mu) and 1e-3 (s) relative.  At T = 20 the
oracle's own mu still moves by 2e-4 between tol 1e-6 and 1e-8 on this workload, so
the fit runs at tol 1e-8, where that change is far below the bar.
"""
import os
import struct
import subprocess

import numpy as np
import pytest

import oracle
import workloads
from bars import binds, check

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "c", "fit_smoke")


def test_plain_c_caller_matches_oracle(gpu, tmp_path):
    if not os.path.exists(EXE):
        pytest.fail(f"{EXE} is missing: run the package build (python -m paper_2105_10439_amd.build)")
    w = dict(workloads.WORKLOADS["small"], tol=1e-8)
    T, seed = 20, 77
    prob = workloads.make_workload("small")
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        f.write(struct.pack("<qqd", prob.N, prob.D, prob.beta))
        f.write(np.ascontiguousarray(prob.phi, dtype=np.float32).tobytes())
        f.write(np.ascontiguousarray(prob.y, dtype=np.float32).tobytes())
    env = dict(os.environ)
    env["LD_LIBRARY_PATH"] = os.path.join(ROOT, "paper_2105_10439_amd") + ":" + env.get("LD_LIBRARY_PATH", "")
    print(f"C caller: N={prob.N} D={prob.D} K={w['K']} T={T}", flush=True)
    res = subprocess.run([EXE, str(inp), str(out), str(w["K"]), str(T), str(w["U"]), repr(w["tol"]), str(seed)],
                         capture_output=True, text=True, timeout=120, env=env)
    print(res.stdout, res.stderr)
    assert res.returncode == 0
    raw = open(out, "rb").read()
    D = prob.D
    vals = np.frombuffer(raw[:12 * D], dtype=np.float32).astype(np.float64)
    mu, s, alpha = vals[:D], vals[D:2 * D], vals[2 * D:]
    steps = struct.unpack("<i", raw[12 * D:12 * D + 4])[0]
    ref = oracle.cofem(prob.phi, prob.y, prob.beta, T=T, K=w["K"], U=w["U"], tol=w["tol"], seed=seed)
    tight = oracle.cofem(prob.phi, prob.y, prob.beta, T=T, K=w["K"], U=w["U"], tol=w["tol"] / 100, seed=seed)

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    e_mu, e_s = rel(mu, ref.mu), rel(s, ref.s)
    sens_mu, sens_s = rel(ref.mu, tight.mu), rel(ref.s, tight.s)
    print(f"C caller: CG steps {steps} (oracle {sum(ref.cg_steps)})")
    binds("c_caller", sens_mu, 1e-4)
    check("c_caller/mu", e_mu, 1e-4)
    check("c_caller/s", e_s, 1e-3)
    assert np.all(np.isfinite(alpha)) and steps > 0
