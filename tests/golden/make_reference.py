"""Write stored oracle results used by the GPU parity tests.

Calls only the FP64 oracle and the seeded input generators, never the GPU
library.  Usage (from the repository root):

    python tests/golden/make_reference.py medium

medium: the N=2048, D=8192 dense Gaussian workload (5% spikes, sigma=0.01,
K=20, T=50, tol=1e-5, U=400), probe seed 77, theta=1, joint stop rule.  The
oracle needs about a minute and a half on 8 cores, too long for a test, so its
mu, s, alpha^(T) and CG step counts are stored in medium_oracle.npz.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
SEED = {"medium": 77}


def medium():
    w = workloads.WORKLOADS["medium"]
    prob = workloads.make_workload("medium")
    t0 = time.time()
    r = oracle.cofem(prob.phi, prob.y, prob.beta, T=w["T"], K=w["K"], U=w["U"], tol=w["tol"], seed=SEED["medium"])
    print(f"oracle medium: {time.time() - t0:.1f}s, CG steps {sum(r.cg_steps)}")
    np.savez_compressed(os.path.join(HERE, "medium_oracle.npz"), mu=r.mu, s=r.s, alpha=r.alpha,
                        cg_steps=np.array(r.cg_steps), rel_resid=np.array(r.rel_resid), seed=SEED["medium"])


if __name__ == "__main__":
    for name in sys.argv[1:] or ["medium"]:
        globals()[name]()
