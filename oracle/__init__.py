"""FP64 CPU oracle for the filtered matrix-sign iterations.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are its only users.  The HIP library never imports, links or
calls anything here, and nothing here imports the library.

* ``nsf_oracle.c`` -- scalar FP64 CSR implementation of Algorithm 3.2.1
  (filtered Newton-Schulz) and Algorithm 3.1.1 (filtered Newton), loaded
  through ctypes from ``liboracle.so`` (built by :func:`build`).
* ``closed_forms.py`` -- exact signs that pin the oracle: the sine eigenbasis
  of tridiagonal Toeplitz matrices and dense eigen/Schur definitions.
"""
from .core import (  # noqa: F401
    build,
    load,
    nsf,
    nmf,
    spgemm,
    ns_step,
    bucket,
    bucket_hi,
    bucket_lo,
    select,
    filter_values,
    nsf_budget,
    nmf_budget,
    norm_inf,
    OracleResult,
    STATUS,
)
