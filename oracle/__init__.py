"""CPU FP64 oracle for the per-level implicit diffusion solve (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this package.  It shares no code with the GPU library and does not import it.
"""
from .fld_oracle import (  # noqa: F401
    Oracle, lp_limiter, minerbo_limiter, harmonic_mean, pcg_jacobi, dense_solve,
    SAME, C2F, F2C, OUTER, DIRICHLET, NEUMANN, ROBIN,
)
