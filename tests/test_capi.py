"""Host-side checks of the C ABI (no GPU needed).

* every function declared in include/cofem.h is exported by libcofem.so;
* the ctypes structs match the C layout (sizes and offsets, from gcc);
* cofem_create rejects bad parameters before touching the device.
"""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2105_10439_amd as lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cofem.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cofem_[A-Za-z_0-9]+)\s*\(", src)))


def test_header_declares_binding_exports():
    assert _declared_functions() == sorted(lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    so = lib.load()
    for name in _declared_functions():
        assert hasattr(so, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (cofem_\w+)", out))
    assert exported == set(_declared_functions())


def _c_layout(struct, fields):
    prog = "#include <stdio.h>\n#include <stddef.h>\n#include \"cofem.h\"\nint main(void){\n"
    prog += f'printf("%zu\\n", sizeof({struct}));\n'
    for f in fields:
        prog += f'printf("%zu\\n", offsetof({struct}, {f}));\n'
    prog += "return 0;}\n"
    d = os.environ.get("TMPDIR", "/tmp")
    src = os.path.join(d, f"layout_{os.getpid()}.c")
    exe = src[:-2]
    open(src, "w").write(prog)
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
    vals = [int(v) for v in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    os.remove(src)
    os.remove(exe)
    return vals[0], vals[1:]


@pytest.mark.parametrize("cls,cname", [(lib.Params, "cofem_params"), (lib.Stats, "cofem_stats"),
                                       (lib.RequestInfo, "cofem_request_info"),
                                       (lib.ServerStats, "cofem_server_stats")])
def test_struct_layout_matches_c(cls, cname):
    names = [f[0] for f in cls._fields_]
    size, offs = _c_layout(cname, names)
    assert ctypes.sizeof(cls) == size
    assert [getattr(cls, n).offset for n in names] == offs


@pytest.mark.parametrize("bad", [
    dict(N=0), dict(D=0), dict(beta=0.0), dict(beta=float("nan")), dict(K=0), dict(K=64), dict(T=0),
    dict(T=513), dict(U=0), dict(tol=-1.0), dict(theta_mode=7), dict(stop_mode=3), dict(phi_dtype=2),
    dict(refine_last=9), dict(alpha_floor=0.0), dict(op_kind=5), dict(mstep_mode=2),
    dict(op_kind=1, conv_taps=0), dict(op_kind=1, conv_taps=257), dict(op_kind=1, N=100, D=200),
    dict(op_kind=2, D=300), dict(op_kind=2, D=8, N=4), dict(op_kind=2, D=65536), dict(op_kind=2, N=300),
    dict(op_kind=2, phi_dtype=1),
])
def test_create_rejects_bad_params_without_device_work(bad):
    so = lib.load()
    p = lib.make_params(N=64, D=256, beta=1e4, K=8, T=5, U=10, tol=1e-6)
    for k, v in bad.items():
        setattr(p, k, v)
    h = ctypes.c_void_p()
    rc = so.cofem_create(ctypes.byref(p), None, ctypes.byref(h))
    assert rc == -1 and not h.value
    assert so.cofem_last_error().decode()


@pytest.mark.parametrize("L,bad", [(0, {}), (65, {}), (2, dict(mstep_mode=1)), (2, dict(K=0)), (2, dict(op_kind=2, D=300))])
def test_multitask_create_rejects_bad_arguments_without_device_work(L, bad):
    so = lib.load()
    p = lib.make_params(N=64, D=256, beta=1e4, K=8, T=5, U=10, tol=1e-6)
    for k, v in bad.items():
        setattr(p, k, v)
    h = ctypes.c_void_p()
    rc = so.cofem_mt_create(ctypes.byref(p), L, None, ctypes.byref(h))
    assert rc == -1 and not h.value
    assert so.cofem_last_error().decode()


@pytest.mark.parametrize("mode,bad", [(3, {}), (-1, {}), (2, dict(phi_dtype=1)), (2, dict(refine_last=2)),
                                      (2, dict(K=32)), (2, dict(op_kind=1, conv_taps=16, N=256))])
def test_multitask_mode_rejects_what_it_cannot_run_without_device_work(mode, bad):
    """An unknown mode, or the batched form with settings it does not take (bf16 or refined
    dictionaries, K > 31, a FIR dictionary), fails before any device work."""
    so = lib.load()
    p = lib.make_params(N=64, D=256, beta=1e4, K=8, T=5, U=10, tol=1e-6)
    for k, v in bad.items():
        setattr(p, k, v)
    h = ctypes.c_void_p()
    rc = so.cofem_mt_create_mode(ctypes.byref(p), 2, mode, None, ctypes.byref(h))
    assert rc == -1 and not h.value
    msg = so.cofem_last_error().decode()
    assert ("mode" in msg) if mode not in (0, 1, 2) else ("batched" in msg)


def test_null_arguments_are_rejected():
    so = lib.load()
    assert so.cofem_create(None, None, None) == -1
    assert so.cofem_fit(None, None) == -1
    assert so.cofem_set_dictionary(None, None) == -1
    assert so.cofem_set_dct_samples(None, None) == -1
    assert so.cofem_mt_set_dct_samples(None, 0, None) == -1
    assert so.cofem_set_probe_mode(None, 1) == -1
    assert so.cofem_posterior(None, None, None, None, None) == -1
    so.cofem_destroy(None)
    assert so.cofem_abi_version() == 7
    assert so.cofem_mt_batched(None) == 0


def test_server_rejects_bad_arguments_without_device_work():
    so = lib.load()
    h = ctypes.c_void_p()
    assert so.cofem_server_create(ctypes.c_size_t(1 << 30), 0, 4, None, ctypes.byref(h)) == -1
    assert so.cofem_server_create(ctypes.c_size_t(1 << 30), 129, 4, None, ctypes.byref(h)) == -1
    assert so.cofem_server_create(ctypes.c_size_t(1 << 30), 8, 0, None, ctypes.byref(h)) == -1
    assert so.cofem_server_create(ctypes.c_size_t(1000), 8, 4, None, ctypes.byref(h)) == -1
    assert not h.value
    assert so.cofem_server_step(None, None, None) == -1
    so.cofem_server_destroy(None)


def test_static_conv_operator_rejects_without_device_work():
    """cofem_conv_apply_A_static validates every argument, including the scratch its size
    needs against the static array, before touching the device (the pointers here are
    never dereferenced)."""
    so = lib.load()
    p = ctypes.c_void_p(0x1000)
    cases = [
        ((None, 4, 16, 400.0, p, p, p, 1, None, None), "NULL"),
        ((p, 0, 16, 400.0, p, p, p, 1, None, None), "L must"),
        ((p, 257, 16, 400.0, p, p, p, 1, None, None), "L must"),
        ((p, 4, 0, 400.0, p, p, p, 1, None, None), "D must"),
        ((p, 4, 16, 0.0, p, p, p, 1, None, None), "beta"),
        ((p, 4, 16, float("inf"), p, p, p, 1, None, None), "beta"),
        ((p, 4, 16, 400.0, p, p, p, 0, None, None), "ncols"),
        ((p, 4, 16, 400.0, p, p, p, 65, None, None), "ncols"),
        ((p, 256, 1 << 20, 400.0, p, p, p, 33, None, None), "scratch"),   # about 600 MB of scratch
        ((p, 256, 1 << 17, 400.0, p, p, p, 33, None, None), "scratch"),   # 75 MB: just over the 64 MiB
    ]
    for args, msg in cases:
        assert so.cofem_conv_apply_A_static(*args) == -1, args
        assert msg in so.cofem_last_error().decode(), (args, so.cofem_last_error())
    assert lib.STATIC_SCRATCH_BYTES == 64 << 20
