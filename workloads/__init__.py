"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This package builds matrices and request streams only.  It holds none of the
sign-function arithmetic (no products, norms, thresholds or iterations), so
that the oracle and the GPU path can both be fed the same inputs without
sharing any of the method's code.
"""
from .generators import (  # noqa: F401
    Csr,
    tridiag_c1,
    ode_block_matrix,
    laplacian_1d,
    laplacian_2d,
    laplacian_3d,
    convdiff_2d,
    random_sparse,
    config_matrix,
    served_stream,
    request_matrix,
    CONFIGS,
)
