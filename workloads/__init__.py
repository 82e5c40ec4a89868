"""Seeded synthetic inputs for covariance-free EM (CoFEM) problems.

This module only draws inputs; it holds none of the method's arithmetic and
imports neither the oracle nor the GPU library, so both sides can consume the
same arrays.  The recipes follow the simulation setup of Sec. V-A (ground-truth
spikes at uniformly random positions, y = Phi z + noise with noise std sigma)
and the dictionary types of Sec. V-A.2 (dense Gaussian with entries N(0, 1/N);
convolutional = lower-triangular Toeplitz built from a decaying filter).  Sizes
and value laws are the ones of the workloads this library is measured on.

All generators are deterministic functions of their arguments: large arrays
are drawn in fixed-size blocks, each block from its own PCG64 stream keyed by
(seed, tag, block index), so the result does not depend on the thread count.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

_BLOCK_ELEMS = 1 << 22  # elements per independently seeded block


def _stream(seed: int, tag: int, idx: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(tag), int(idx)])))


def _threads() -> int:
    n = os.cpu_count() or 1
    return max(1, min(16, n))


def gaussian_dictionary(N: int, D: int, seed: int) -> np.ndarray:
    """Dense N x D dictionary, entries i.i.d. N(0, 1/N), row-major float32.

    Drawn in blocks of whole rows; block b uses stream (seed, 0xD1C7, b).
    """
    N, D = int(N), int(D)
    phi = np.empty((N, D), dtype=np.float32)
    rows_per_block = max(1, _BLOCK_ELEMS // max(D, 1))
    nblocks = (N + rows_per_block - 1) // rows_per_block
    scale = np.float32(1.0 / math.sqrt(N))

    def fill(b: int) -> None:
        r0 = b * rows_per_block
        r1 = min(N, r0 + rows_per_block)
        blk = phi[r0:r1]
        _stream(seed, 0xD1C7, b).standard_normal(out=blk, dtype=np.float32)
        blk *= scale

    if nblocks == 1:
        fill(0)
    else:
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(fill, range(nblocks)))
    return phi


def sparse_code(D: int, d: int, seed: int, law: str = "normal") -> np.ndarray:
    """Ground-truth code z in R^D with d nonzeros at uniformly random positions.

    law = "normal": values N(0, 1); "normal5": values N(0, 5), read as variance 5 (the
    DCT setting of Sec. V-A.2); "exp1": values Exp(1) (non-negative spikes).
    """
    rng = _stream(seed, 0x5A11)
    z = np.zeros(int(D), dtype=np.float64)
    pos = rng.choice(int(D), size=int(d), replace=False)
    if law == "normal":
        z[pos] = rng.standard_normal(int(d))
    elif law == "normal5":
        z[pos] = math.sqrt(5.0) * rng.standard_normal(int(d))
    elif law == "exp1":
        z[pos] = rng.exponential(1.0, int(d))
    else:
        raise ValueError(f"unknown spike law {law!r}")
    return z


def bernoulli_spikes(D: int, p: float, seed: int) -> np.ndarray:
    """z_j = Bernoulli(p) * Exp(1), the calcium-trace spike law."""
    rng = _stream(seed, 0xB3E1)
    on = rng.random(int(D)) < p
    z = np.zeros(int(D), dtype=np.float64)
    z[on] = rng.exponential(1.0, int(on.sum()))
    return z


def dense_observation(phi: np.ndarray, z: np.ndarray, sigma: float, seed: int) -> np.ndarray:
    """y = Phi z + sigma * N(0, I), formed in float64 and rounded to float32."""
    supp = np.flatnonzero(z)
    y = phi[:, supp].astype(np.float64) @ z[supp]
    y += sigma * _stream(seed, 0x7015E).standard_normal(phi.shape[0])
    return y.astype(np.float32)


def exp_filter(taps: int, tau: float) -> np.ndarray:
    """Causal filter h[t] = exp(-t / tau), t = 0..taps-1, float32."""
    return np.exp(-np.arange(int(taps), dtype=np.float64) / float(tau)).astype(np.float32)


def geometric_filter(taps: int, rho: float) -> np.ndarray:
    """Causal filter h[t] = (1 - rho)^t, the decaying filter of Sec. V-A.2."""
    return ((1.0 - float(rho)) ** np.arange(int(taps), dtype=np.float64)).astype(np.float32)


def conv_observation(h: np.ndarray, z: np.ndarray, sigma: float, seed: int) -> np.ndarray:
    """y = Phi z + noise for the causal convolution Phi (N = D), float64 -> float32.

    Phi_{ij} = h[i - j] for 0 <= i - j < len(h).  Only the nonzero spikes are
    expanded, so this is cheap for sparse z at any D.
    """
    D = z.shape[0]
    y = np.zeros(D, dtype=np.float64)
    hh = h.astype(np.float64)
    L = hh.shape[0]
    for j in np.flatnonzero(z):
        n = min(L, D - j)
        y[j:j + n] += z[j] * hh[:n]
    y += sigma * _stream(seed, 0xC0417).standard_normal(D)
    return y.astype(np.float32)


def dct_rows(D: int, N: int, seed: int) -> np.ndarray:
    """The N of D sample positions kept by the undersampling operator M of the DCT
    dictionary (Sec. V-A.2): distinct, uniformly random, sorted, int32."""
    rng = _stream(seed, 0xDC7)
    return np.sort(rng.choice(int(D), size=int(N), replace=False)).astype(np.int32)


def dct_observation(rows: np.ndarray, z: np.ndarray, sigma: float, seed: int) -> np.ndarray:
    """y = M Omega^{-1} z + sigma * N(0, I) with Omega the orthonormal DCT-II of size D
    (inverse DCT by scipy in float64, then the kept samples), rounded to float32."""
    import scipy.fft

    x = scipy.fft.idct(np.asarray(z, dtype=np.float64), type=2, norm="ortho")
    y = x[np.asarray(rows, dtype=np.int64)]
    y += float(sigma) * _stream(seed, 0x0B5E).standard_normal(y.shape[0])
    return y.astype(np.float32)


@dataclass
class Problem:
    """One sparse-coding problem y = Phi z + eps with its generation recipe."""
    name: str
    N: int
    D: int
    beta: float
    sigma: float
    y: np.ndarray
    z: np.ndarray
    phi: np.ndarray | None = None     # dense dictionary (N x D float32), or None
    h: np.ndarray | None = None       # FIR taps for a convolutional dictionary
    rows: np.ndarray | None = None    # kept sample positions of a subsampled DCT dictionary
    meta: dict = field(default_factory=dict)


def dense_problem(N: int, D: int, d: int, sigma: float, seed: int, name: str = "dense",
                  law: str = "normal") -> Problem:
    phi = gaussian_dictionary(N, D, seed)
    z = sparse_code(D, d, seed, law)
    y = dense_observation(phi, z, sigma, seed)
    return Problem(name=name, N=N, D=D, beta=1.0 / sigma ** 2, sigma=sigma, y=y, z=z, phi=phi,
                   meta={"d": int(d), "seed": int(seed), "law": law})


def multitask_problems(L: int, N: int, D: int, d: int, sigma: float, seed: int) -> list:
    """L dense problems whose codes share one support of d positions (Sec. III-E.1's
    setting): task l has its own dictionary and values, drawn with seed * 1009 + l."""
    pos = _stream(seed, 0x3A5C).choice(int(D), size=int(d), replace=False)
    out = []
    for l in range(int(L)):
        s = int(seed) * 1009 + l
        phi = gaussian_dictionary(N, D, s)
        z = np.zeros(int(D), dtype=np.float64)
        z[pos] = _stream(s, 0x5A11).standard_normal(int(d))
        y = dense_observation(phi, z, sigma, s)
        out.append(Problem(name=f"task{l}", N=N, D=D, beta=1.0 / sigma ** 2, sigma=sigma, y=y, z=z, phi=phi,
                           meta={"d": int(d), "seed": s, "law": "normal", "shared_support": True}))
    return out


def conv_problem(D: int, taps: int, tau: float, p_spike: float, sigma: float, seed: int,
                 name: str = "conv") -> Problem:
    h = exp_filter(taps, tau)
    z = bernoulli_spikes(D, p_spike, seed)
    y = conv_observation(h, z, sigma, seed)
    return Problem(name=name, N=D, D=D, beta=1.0 / sigma ** 2, sigma=sigma, y=y, z=z, h=h,
                   meta={"taps": int(taps), "tau": float(tau), "p": float(p_spike), "seed": int(seed)})


def dct_problem(D: int, N: int, d: int, sigma: float, seed: int, name: str = "dct") -> Problem:
    """Subsampled DCT dictionary Phi = M Omega^{-1} with N of D samples kept, d spikes
    N(0, 5) at uniformly random positions, noise std sigma."""
    rows = dct_rows(D, N, seed)
    z = sparse_code(D, d, seed, "normal5")
    y = dct_observation(rows, z, sigma, seed)
    return Problem(name=name, N=int(N), D=int(D), beta=1.0 / sigma ** 2, sigma=sigma, y=y, z=z, rows=rows,
                   meta={"d": int(d), "seed": int(seed), "law": "normal5"})


# ---------------------------------------------------------------------------
# Named workloads.  "small": N=64, D=256, 10 spikes, sigma=0.01, K=8, T=50,
# tol=1e-6, U=256.  "medium": N=2048, D=8192, 5% spikes, K=20, T=50, tol=1e-5,
# U=400.  "large": N=16384, D=65536, 2% spikes, K=32, T=30, tol=1e-5, U=400.
# "conv": D=2^20 causal FIR with 256 taps of exp(-t/50), Bernoulli(0.01)*Exp(1)
# spikes, sigma=0.05, K=20, T=30.  "dct": the DCT scalability setting of Sec. V-C at
# its largest size, D=2^15, N=floor(D/3), d=floor(0.12 D) spikes N(0, 5), sigma=0.01,
# K=20, T=30, U=400, tol=1e-4.  "multitask": L=4 tasks of the medium shape (N=2048,
# D=8192) sharing one support of 5% spikes (multitask_problems), K=20, T=30, tol=1e-5.
# ---------------------------------------------------------------------------
WORKLOADS = {
    "small": dict(N=64, D=256, d=10, sigma=0.01, K=8, T=50, tol=1e-6, U=256, seed=1001),
    "medium": dict(N=2048, D=8192, d=409, sigma=0.01, K=20, T=50, tol=1e-5, U=400, seed=1002),
    "large": dict(N=16384, D=65536, d=1310, sigma=0.01, K=32, T=30, tol=1e-5, U=400, seed=1003),
    "conv": dict(D=1 << 20, taps=256, tau=50.0, p=0.01, sigma=0.05, K=20, T=30, tol=1e-5, U=400, seed=1005),
    "dct": dict(D=1 << 15, N=(1 << 15) // 3, d=int(0.12 * (1 << 15)), sigma=0.01, K=20, T=30, tol=1e-4, U=400,
                seed=1006, dictionary="dct"),
    "multitask": dict(L=4, N=2048, D=8192, d=409, sigma=0.01, K=20, T=30, tol=1e-5, U=400, seed=1007),
}


def make_workload(name: str, **override):
    """The named workload's Problem (a list of L Problems for "multitask")."""
    w = dict(WORKLOADS[name])
    w.update(override)
    if name == "multitask":
        return multitask_problems(w["L"], w["N"], w["D"], w["d"], w["sigma"], w["seed"])
    if name == "conv" or "taps" in w:
        return conv_problem(w["D"], w["taps"], w["tau"], w["p"], w["sigma"], w["seed"], name=name)
    if w.get("dictionary") == "dct":
        return dct_problem(w["D"], w["N"], w["d"], w["sigma"], w["seed"], name=name)
    return dense_problem(w["N"], w["D"], w["d"], w["sigma"], w["seed"], name=name)


def serving_stream(n: int, seed: int, d_lo: int = 512, d_hi: int = 16384, frac: float = 0.05,
                   sigmas=(0.01, 0.05)):
    """Request descriptors for the serving workload.

    D_i ~ uniform integer in [d_lo, d_hi], N_i = floor(D_i / 4), d_i = floor(frac * D_i),
    sigma_i drawn from `sigmas` with equal probability, per-request data seed.
    Returns a list of dicts (no arrays; draw them with `serving_request`).
    """
    rng = _stream(seed, 0x5E7E)
    out = []
    for i in range(int(n)):
        D = int(rng.integers(d_lo, d_hi + 1))
        out.append(dict(idx=i, D=D, N=D // 4, d=int(frac * D), sigma=float(sigmas[int(rng.integers(len(sigmas)))]),
                        seed=int(seed) * 100003 + i))
    return out


def serving_request(desc: dict) -> Problem:
    return dense_problem(desc["N"], desc["D"], desc["d"], desc["sigma"], desc["seed"], name=f"req{desc['idx']}")


def poisson_arrivals(n: int, rate_per_s: float, seed: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process with the given rate."""
    gaps = _stream(seed, 0xA221).exponential(1.0 / float(rate_per_s), int(n))
    return np.cumsum(gaps) - gaps[0]
