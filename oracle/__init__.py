"""FP64 CPU oracle for the factorization-based DPP sampler.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers. Nothing here is shared with, imported
by, or imports the HIP library package.
"""
from .oracle import (ldlh, lu, zldlh, zlu, conditional_pivot, conditional_kernel, lensemble_marginal,
                     reconstruct_ldlh, reconstruct_lu, load_library, omp_threads)

__all__ = ["ldlh", "lu", "zldlh", "zlu", "conditional_pivot", "conditional_kernel", "lensemble_marginal",
           "reconstruct_ldlh", "reconstruct_lu", "load_library", "omp_threads"]
