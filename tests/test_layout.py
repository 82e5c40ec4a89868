"""The tile-interleaved layout of the FIR dictionary's bf16 signal slices, checked on the
host by `tests/c/layout_check` (built by the package build step from
`tests/c/layout_check.hip`, which includes the library's device helpers): a one-to-one
map of the real columns onto Q Dp elements for every Q up to 64, and the address
arithmetic of the filter kernels' loads against it.  Bit-exact index work, no GPU."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "c", "layout_check")


def test_signal_layout_is_a_bijection_and_matches_kernel_addressing():
    if not os.path.exists(EXE):
        pytest.fail(f"{EXE} is missing: run the package build (python -m paper_2105_10439_amd.build)")
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "layout ok"
