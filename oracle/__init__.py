"""CPU FP64 oracle for covariance-free EM (CoFEM).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the test suite, the package smoke
check and the CPU-baseline leg of the benchmark use it.  It shares no code with
the GPU library (no headers, kernels, helpers or constant tables) and does not
import it.

Every function here is plain NumPy in float64 and follows the paper's
equations and algorithms step by step, in their order and notation; see the
docstrings of `oracle.cofem` for the passage each one restates.
"""
from .cofem import (  # noqa: F401
    GOLDEN_GAMMA,
    splitmix64_outputs,
    mix64,
    probe_words,
    rademacher_probes,
    hadamard_probes,
    DenseOperator,
    ConvOperator,
    DctOperator,
    dct_matrix,
    PCGResult,
    pcg,
    diag_estimate,
    diag_estimate_general,
    CoFEMResult,
    cofem,
    exact_em,
    log_evidence,
    woodbury_sigma,
    nonneg_second_moment,
    cofem_multitask,
    posterior_variance,
)
