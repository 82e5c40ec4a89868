"""Python binding of the gfx950 CoFEM library (include/cofem.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
libcofem.so.  PyTorch supplies device memory and the current stream.  There is
no CPU fallback: if the shared library is missing, `load()` raises.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libcofem.so")

COFEM_MAX_T = 512
COFEM_MAX_K = 63

STATUS = {0: "COFEM_OK", -1: "COFEM_EINVAL", -2: "COFEM_ENOMEM", -3: "COFEM_EDEVICE", -4: "COFEM_ESTATE",
          -5: "COFEM_EBREAKDOWN", -6: "COFEM_EBUDGET"}
THETA = {"ones": 0, "jacobi": 1}
STOP = {"joint": 0, "column": 1}
OPS = {"dense": 0, "conv": 1, "dct": 2}
DTYPES = {"fp32": 0, "bf16": 1}
MSTEP = {"gaussian": 0, "nonneg": 1}
PROBE_MODES = {"hash": 0, "hadamard": 1}
ABI_VERSION = 7  # COFEM_ABI_VERSION of include/cofem.h

# every symbol include/cofem.h declares
EXPORTS = [
    "cofem_abi_version", "cofem_last_error", "cofem_create", "cofem_destroy", "cofem_set_dictionary",
    "cofem_set_dct_samples",
    "cofem_fit", "cofem_posterior", "cofem_variance", "cofem_apply_A", "cofem_conv_apply_A_static",
    "cofem_set_probe_mode", "cofem_set_timing", "cofem_get_timing",
    "cofem_server_create", "cofem_server_destroy", "cofem_server_submit", "cofem_server_step",
    "cofem_server_poll", "cofem_server_cancel", "cofem_server_get_stats",
    "cofem_mt_create", "cofem_mt_destroy", "cofem_mt_set_dictionary", "cofem_mt_set_dct_samples", "cofem_mt_fit",
    "cofem_mt_posterior", "cofem_mt_create_mode", "cofem_mt_batched",
]
REQ_STATE = {0: "pending", 1: "running", 2: "done", -1: "unknown"}


class CofemError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int64), ("D", ctypes.c_int64), ("beta", ctypes.c_double),
        ("K", ctypes.c_int32), ("T", ctypes.c_int32), ("U", ctypes.c_int32), ("tol", ctypes.c_double),
        ("theta_mode", ctypes.c_int32), ("stop_mode", ctypes.c_int32), ("op_kind", ctypes.c_int32),
        ("phi_dtype", ctypes.c_int32), ("refine_last", ctypes.c_int32), ("conv_taps", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("alpha_floor", ctypes.c_double),
        ("mstep_mode", ctypes.c_int32), ("reserved_", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("T", ctypes.c_int32),
        ("cg_steps", ctypes.c_int32 * COFEM_MAX_T),
        ("rel_resid", ctypes.c_double * COFEM_MAX_T),
        ("used_bf16", ctypes.c_int32 * COFEM_MAX_T),
        ("clamped", ctypes.c_int64),
        ("breakdown", ctypes.c_int32),
        ("total_cg_steps", ctypes.c_int32),
        ("ms_setup", ctypes.c_double),
        ("ms_fit", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        T = self.T
        return dict(T=T, cg_steps=list(self.cg_steps[:T]), rel_resid=list(self.rel_resid[:T]),
                    used_bf16=list(self.used_bf16[:T]), clamped=int(self.clamped), breakdown=int(self.breakdown),
                    total_cg_steps=int(self.total_cg_steps), ms_setup=float(self.ms_setup),
                    ms_fit=float(self.ms_fit))


class RequestInfo(ctypes.Structure):
    _fields_ = [
        ("state", ctypes.c_int32), ("T", ctypes.c_int32), ("total_cg_steps", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("t_submit_ms", ctypes.c_double), ("t_admit_ms", ctypes.c_double), ("t_finish_ms", ctypes.c_double),
        ("bytes", ctypes.c_int64),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
        ("rejected", ctypes.c_int64), ("ticks", ctypes.c_int64), ("active", ctypes.c_int32),
        ("max_active", ctypes.c_int32), ("bytes_in_use", ctypes.c_int64), ("bytes_peak", ctypes.c_int64),
        ("budget", ctypes.c_int64), ("tick_ms", ctypes.c_double), ("dict_bytes", ctypes.c_double),
    ]


_lib = None


def load() -> ctypes.CDLL:
    """Load libcofem.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2105_10439_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "cofem_abi_version": (i32, []),
        "cofem_last_error": (ctypes.c_char_p, []),
        "cofem_create": (i32, [ctypes.POINTER(Params), vp, ctypes.POINTER(vp)]),
        "cofem_destroy": (None, [vp]),
        "cofem_set_dictionary": (i32, [vp, vp]),
        "cofem_set_dct_samples": (i32, [vp, vp]),
        "cofem_fit": (i32, [vp, vp]),
        "cofem_posterior": (i32, [vp, vp, vp, vp, ctypes.POINTER(Stats)]),
        "cofem_apply_A": (i32, [vp, vp, vp, vp, i32, i32, vp]),
        "cofem_conv_apply_A_static": (i32, [vp, i32, i64, dbl, vp, vp, vp, i32, vp, vp]),
        "cofem_variance": (i32, [vp, vp, i32, ctypes.c_uint64, vp, vp, ctypes.POINTER(Stats)]),
        "cofem_set_timing": (i32, [vp, i32]),
        "cofem_set_probe_mode": (i32, [vp, i32]),
        "cofem_get_timing": (i32, [vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(i64)]),
        "cofem_server_create": (i32, [ctypes.c_size_t, i32, i32, vp, ctypes.POINTER(vp)]),
        "cofem_server_destroy": (None, [vp]),
        "cofem_server_submit": (i32, [vp, ctypes.POINTER(Params), vp, vp, ctypes.POINTER(i64)]),
        "cofem_server_step": (i32, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "cofem_server_poll": (i32, [vp, i64, vp, vp, vp, ctypes.POINTER(RequestInfo)]),
        "cofem_server_get_stats": (i32, [vp, ctypes.POINTER(ServerStats)]),
        "cofem_server_cancel": (i32, [vp, i64]),
        "cofem_mt_create": (i32, [ctypes.POINTER(Params), i32, vp, ctypes.POINTER(vp)]),
        "cofem_mt_create_mode": (i32, [ctypes.POINTER(Params), i32, i32, vp, ctypes.POINTER(vp)]),
        "cofem_mt_batched": (i32, [vp]),
        "cofem_mt_destroy": (None, [vp]),
        "cofem_mt_set_dictionary": (i32, [vp, i32, vp]),
        "cofem_mt_set_dct_samples": (i32, [vp, i32, vp]),
        "cofem_mt_fit": (i32, [vp, ctypes.POINTER(vp)]),
        "cofem_mt_posterior": (i32, [vp, i32, vp, vp, vp, ctypes.POINTER(Stats)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if lib.cofem_abi_version() != ABI_VERSION:
        raise RuntimeError(f"{LIB_PATH} has ABI version {lib.cofem_abi_version()}, the binding expects "
                           f"{ABI_VERSION}: rebuild it with `python -m paper_2105_10439_amd.build`")
    _lib = lib
    return lib


def _check(rc: int) -> None:
    if rc != 0:
        raise CofemError(rc, load().cofem_last_error().decode())


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def make_params(N, D, beta, K, T, U, tol, theta="ones", stop="joint", op="dense", phi_dtype="fp32",
                refine_last=0, conv_taps=0, seed=0, alpha_floor=1e-30, mstep="gaussian") -> Params:
    return Params(N=int(N), D=int(D), beta=float(beta), K=int(K), T=int(T), U=int(U), tol=float(tol),
                  theta_mode=THETA[theta], stop_mode=STOP[stop], op_kind=OPS[op], phi_dtype=DTYPES[phi_dtype],
                  refine_last=int(refine_last), conv_taps=int(conv_taps), seed=int(seed) & ((1 << 64) - 1),
                  alpha_floor=float(alpha_floor), mstep_mode=MSTEP[mstep], reserved_=0)


class CoFEM:
    """One problem shape on the current device and torch stream."""

    def __init__(self, N, D, beta, K, T, U, tol, theta="ones", stop="joint", op="dense", phi_dtype="fp32",
                 refine_last=0, conv_taps=0, seed=0, alpha_floor=1e-30, mstep="gaussian", stream=None):
        import torch

        lib = load()
        self.params = make_params(N, D, beta, K, T, U, tol, theta, stop, op, phi_dtype, refine_last, conv_taps,
                                  seed, alpha_floor, mstep)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(lib.cofem_create(ctypes.byref(self.params), ctypes.c_void_p(self.stream.cuda_stream),
                                ctypes.byref(h)))
        self._h = h
        self.N, self.D = int(N), int(D)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().cofem_destroy(self._h)
            self._h = None

    __del__ = close

    def _dev(self, t, n, name):
        import torch

        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
        if t.numel() != n:
            raise ValueError(f"{name} must have {n} elements, got {t.numel()}")
        return ctypes.c_void_p(t.data_ptr())

    def set_dictionary(self, phi):
        """Dense: the N x D matrix; conv: the taps; DCT: the N kept sample indices (int32)."""
        import torch

        if self.params.op_kind == OPS["dct"]:
            if not (isinstance(phi, torch.Tensor) and phi.is_cuda and phi.dtype == torch.int32
                    and phi.is_contiguous() and phi.numel() == self.N):
                raise TypeError(f"rows must be a contiguous int32 CUDA tensor of {self.N} sample indices")
            _check(load().cofem_set_dct_samples(self._h, ctypes.c_void_p(phi.data_ptr())))
            return
        n = self.N * self.D if self.params.op_kind == 0 else self.params.conv_taps
        _check(load().cofem_set_dictionary(self._h, self._dev(phi, n, "phi")))

    def fit(self, y):
        _check(load().cofem_fit(self._h, self._dev(y, self.N, "y")))

    def posterior(self):
        import torch

        dev = torch.device("cuda", torch.cuda.current_device())
        mu = torch.empty(self.D, dtype=torch.float32, device=dev)
        s = torch.empty_like(mu)
        alpha = torch.empty_like(mu)
        st = Stats()
        _check(load().cofem_posterior(self._h, ctypes.c_void_p(mu.data_ptr()), ctypes.c_void_p(s.data_ptr()),
                                      ctypes.c_void_p(alpha.data_ptr()), ctypes.byref(st)))
        return mu, s, alpha, st.as_dict()

    def variance(self, batches, seed=0, alpha=None):
        """diag(Sigma) at alpha (default: the fit's) from K * batches probes; returns (s, mu, stats)."""
        import torch

        dev = torch.device("cuda", torch.cuda.current_device())
        s = torch.empty(self.D, dtype=torch.float32, device=dev)
        mu = torch.empty_like(s)
        st = Stats()
        a = self._dev(alpha, self.D, "alpha") if alpha is not None else None
        _check(load().cofem_variance(self._h, a, int(batches), int(seed) & ((1 << 64) - 1),
                                     ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(mu.data_ptr()), ctypes.byref(st)))
        return s, mu, st.as_dict()

    def apply_A(self, alpha, P, use_bf16=False, want_pi=False):
        """Psi = beta Phi^T Phi P + alpha * P for P of shape (ncols, D) (rows = columns of the block)."""
        import torch

        ncols = P.shape[0]
        Psi = torch.empty_like(P)
        pi = torch.empty(ncols, dtype=torch.float64, device=P.device) if want_pi else None
        _check(load().cofem_apply_A(self._h, self._dev(alpha, self.D, "alpha"),
                                    self._dev(P, ncols * self.D, "P"), ctypes.c_void_p(Psi.data_ptr()),
                                    int(ncols), int(bool(use_bf16)),
                                    ctypes.c_void_p(pi.data_ptr()) if pi is not None else None))
        return (Psi, pi) if want_pi else Psi

    def set_timing(self, enable: bool):
        _check(load().cofem_set_timing(self._h, int(bool(enable))))

    def set_probe_mode(self, mode: str):
        """Test hook: "hash" (default) or "hadamard" probes for later E-steps."""
        _check(load().cofem_set_probe_mode(self._h, PROBE_MODES[mode]))

    def get_timing(self, which: str):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(load().cofem_get_timing(self._h, 1 if which == "bf16" else 0, ctypes.byref(ms), ctypes.byref(n)))
        return float(ms.value), int(n.value)


STATIC_SCRATCH_BYTES = 64 << 20  # COFEM_STATIC_SCRATCH_BYTES of include/cofem.h


def conv_apply_A_static(h, alpha, P, beta, want_pi=False, stream=None):
    """cofem_conv_apply_A_static: Psi = beta Phi^T Phi P + alpha * P for the FIR dictionary with
    taps h, P of shape (ncols, D), with no context and no device allocation by the library
    (its scratch is a static device array).  Only enqueues on `stream` (default: torch's
    current stream); the outputs are allocated here by torch, not by the library."""
    import torch

    stream = stream if stream is not None else torch.cuda.current_stream()
    for name, t in (("h", h), ("alpha", alpha), ("P", P)):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
    ncols, D = int(P.shape[0]), int(P.shape[1])
    if alpha.numel() != D:
        raise ValueError(f"alpha must have {D} elements")
    Psi = torch.empty_like(P)
    pi = torch.empty(ncols, dtype=torch.float64, device=P.device) if want_pi else None
    _check(load().cofem_conv_apply_A_static(ctypes.c_void_p(h.data_ptr()), int(h.numel()), D, float(beta),
                                            ctypes.c_void_p(alpha.data_ptr()), ctypes.c_void_p(P.data_ptr()),
                                            ctypes.c_void_p(Psi.data_ptr()), ncols,
                                            ctypes.c_void_p(pi.data_ptr()) if pi is not None else None,
                                            ctypes.c_void_p(stream.cuda_stream)))
    return (Psi, pi) if want_pi else Psi


MT_MODES = {"auto": 0, "streams": 1, "batched": 2}


class MultiTask(CoFEM):
    """Multi-task CoFEM (cofem_mt_*): L problems of one shape sharing alpha.  mode: "batched"
    (all tasks' systems together, one launch per phase), "streams" (one context per task on
    its own stream) or "auto" (batched when the settings allow it and L > 4, else streams)."""

    def __init__(self, L, N, D, beta, K, T, U, tol, theta="ones", stop="joint", op="dense", phi_dtype="fp32",
                 refine_last=0, conv_taps=0, seed=0, alpha_floor=1e-30, stream=None, mode="auto"):
        import torch

        lib = load()
        self.params = make_params(N, D, beta, K, T, U, tol, theta, stop, op, phi_dtype, refine_last, conv_taps,
                                  seed, alpha_floor)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        if mode not in MT_MODES:
            raise ValueError(f"mode must be one of {sorted(MT_MODES)}")
        _check(lib.cofem_mt_create_mode(ctypes.byref(self.params), int(L), MT_MODES[mode],
                                        ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.L, self.N, self.D = int(L), int(N), int(D)
        self.batched = bool(lib.cofem_mt_batched(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().cofem_mt_destroy(self._h)
            self._h = None

    __del__ = close

    def set_dictionary(self, task, phi):
        """Task `task`'s dictionary: as CoFEM.set_dictionary (DCT: int32 sample indices)."""
        import torch

        if self.params.op_kind == OPS["dct"]:
            if not (isinstance(phi, torch.Tensor) and phi.is_cuda and phi.dtype == torch.int32
                    and phi.is_contiguous() and phi.numel() == self.N):
                raise TypeError(f"rows must be a contiguous int32 CUDA tensor of {self.N} sample indices")
            _check(load().cofem_mt_set_dct_samples(self._h, int(task), ctypes.c_void_p(phi.data_ptr())))
            return
        n = self.N * self.D if self.params.op_kind == 0 else self.params.conv_taps
        _check(load().cofem_mt_set_dictionary(self._h, int(task), self._dev(phi, n, "phi")))

    def fit(self, ys):
        if len(ys) != self.L:
            raise ValueError(f"need {self.L} observation vectors")
        arr = (ctypes.c_void_p * self.L)(*[self._dev(y, self.N, f"ys[{l}]") for l, y in enumerate(ys)])
        _check(load().cofem_mt_fit(self._h, arr))

    def posterior(self, task):
        import torch

        dev = torch.device("cuda", torch.cuda.current_device())
        mu = torch.empty(self.D, dtype=torch.float32, device=dev)
        s = torch.empty_like(mu)
        alpha = torch.empty_like(mu)
        st = Stats()
        _check(load().cofem_mt_posterior(self._h, int(task), ctypes.c_void_p(mu.data_ptr()),
                                         ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(alpha.data_ptr()),
                                         ctypes.byref(st)))
        return mu, s, alpha, st.as_dict()

    def apply_A(self, *a, **k):
        raise NotImplementedError("apply_A is a single-problem test hook")

    def set_timing(self, enable: bool):
        raise NotImplementedError("operator timing is per single-problem context")

    get_timing = set_timing


class Server:
    """Continuous-batching server (cofem_server_*).  Dictionaries and observations are
    host float32 arrays; they are kept referenced here until the request is admitted."""

    def __init__(self, budget_bytes: int, max_slots: int = 64, steps_per_tick: int = 4, stream=None):
        lib = load()
        h = ctypes.c_void_p()
        st = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
        _check(lib.cofem_server_create(ctypes.c_size_t(int(budget_bytes)), int(max_slots), int(steps_per_tick), st,
                                       ctypes.byref(h)))
        self._h = h
        self._held = {}   # request id -> (phi, y) kept alive until admission
        self._D = {}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().cofem_server_destroy(self._h)
            self._h = None

    __del__ = close

    def submit(self, phi, y, *, beta, K, T, U, tol, theta="ones", stop="joint", seed=0, alpha_floor=1e-30,
               mstep="gaussian") -> int:
        import numpy as np

        phi = np.ascontiguousarray(phi, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        N, D = phi.shape
        if y.shape != (N,):
            raise ValueError("y must have N elements")
        p = make_params(N, D, beta, K, T, U, tol, theta, stop, "dense", "fp32", 0, 0, seed, alpha_floor, mstep)
        rid = ctypes.c_int64()
        _check(load().cofem_server_submit(self._h, ctypes.byref(p), phi.ctypes.data_as(ctypes.c_void_p),
                                          y.ctypes.data_as(ctypes.c_void_p), ctypes.byref(rid)))
        self._held[rid.value] = (phi, y)
        self._D[rid.value] = D
        return rid.value

    def step(self):
        run = ctypes.c_int32()
        pend = ctypes.c_int32()
        _check(load().cofem_server_step(self._h, ctypes.byref(run), ctypes.byref(pend)))
        for rid in list(self._held):
            if self.info(rid)["state"] != "pending":
                del self._held[rid]
        return run.value, pend.value

    def info(self, rid: int) -> dict:
        inf = RequestInfo()
        _check(load().cofem_server_poll(self._h, int(rid), None, None, None, ctypes.byref(inf)))
        return dict(state=REQ_STATE[inf.state], T=inf.T, total_cg_steps=inf.total_cg_steps,
                    t_submit_ms=inf.t_submit_ms, t_admit_ms=inf.t_admit_ms, t_finish_ms=inf.t_finish_ms,
                    bytes=inf.bytes)

    def result(self, rid: int):
        """(mu, s, alpha, info) of a finished request (releases its record), or None if not done."""
        import numpy as np

        inf = self.info(rid)
        if inf["state"] != "done":
            return None
        D = self._D.pop(rid)
        mu = np.empty(D, np.float32)
        s = np.empty(D, np.float32)
        alpha = np.empty(D, np.float32)
        _check(load().cofem_server_poll(self._h, int(rid), mu.ctypes.data_as(ctypes.c_void_p),
                                        s.ctypes.data_as(ctypes.c_void_p), alpha.ctypes.data_as(ctypes.c_void_p),
                                        None))
        return mu, s, alpha, inf

    def cancel(self, rid: int) -> None:
        """Withdraw a pending, running or finished request (its id is unknown afterwards)."""
        _check(load().cofem_server_cancel(self._h, int(rid)))
        self._held.pop(rid, None)
        self._D.pop(rid, None)

    def stats(self) -> dict:
        st = ServerStats()
        _check(load().cofem_server_get_stats(self._h, ctypes.byref(st)))
        return {f[0]: getattr(st, f[0]) for f in ServerStats._fields_}
