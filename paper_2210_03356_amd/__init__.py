"""libsignfn: filtered Newton-Schulz / filtered Newton matrix sign on AMD MI355X.

The compute path is the HIP library ``libsignfn.so`` (C ABI in
``include/signfn.h``); this package is its ctypes binding.
"""
from .signfn import (  # noqa: F401
    DeviceCsr,
    Result,
    Server,
    SignError,
    default_opts,
    load,
    release_cached,
    sign_filter,
    sign_filter_noalloc,
    NOALLOC_MAX_ROWS,
    sign_newton,
    sign_ns,
    sign_spgemm,
    LIB_PATH,
)
