"""ctypes front end of the C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess
import threading
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nsf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "ENOCONV", -4: "EDIVERGED"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-Wall", "-shared", "-fPIC", _SRC, "-lm", "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


class _Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("stop_rule", C.c_int), ("c_fixed", C.c_double),
                ("switch_res", C.c_double), ("max_iter", C.c_int), ("filter_y", C.c_int),
                ("scale", C.c_double), ("nthreads", C.c_int), ("trace_cap", C.c_int)]


class _Res(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64),
                ("rp", C.POINTER(C.c_int64)), ("ci", C.POINTER(C.c_int32)),
                ("v", C.POINTER(C.c_double)),
                ("status", C.c_int), ("iters", C.c_int), ("stagnated", C.c_int),
                ("scale", C.c_double), ("res_fro", C.c_double), ("step_fro", C.c_double),
                ("e", C.POINTER(C.c_double)), ("d", C.POINTER(C.c_double)),
                ("tau", C.POINTER(C.c_double)), ("xfro", C.POINTER(C.c_double)),
                ("ffro", C.POINTER(C.c_double)),
                ("nnz_x", C.POINTER(C.c_int64)), ("nnz_bar", C.POINTER(C.c_int64)),
                ("nnz_r", C.POINTER(C.c_int64)), ("bstar", C.POINTER(C.c_int)),
                ("inner_total", C.c_int64)]


_P64 = np.ctypeslib.ndpointer(np.int64, flags="C")
_P32 = np.ctypeslib.ndpointer(np.int32, flags="C")
_PD = np.ctypeslib.ndpointer(np.float64, flags="C")


def load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB):
            build(force=True)
        lib = C.CDLL(_LIB)
        lib.oracle_nsf.argtypes = [C.c_int64, _P64, _P32, _PD, C.POINTER(_Opts), C.POINTER(_Res)]
        lib.oracle_nsf.restype = C.c_int
        lib.oracle_nmf.argtypes = [C.c_int64, _P64, _P32, _PD, C.POINTER(_Opts), C.POINTER(_Res)]
        lib.oracle_nmf.restype = C.c_int
        lib.oracle_free_result.argtypes = [C.POINTER(_Res)]
        lib.oracle_bucket.argtypes = [C.c_double]
        lib.oracle_bucket.restype = C.c_int
        lib.oracle_bucket_hi.argtypes = [C.c_int]
        lib.oracle_bucket_hi.restype = C.c_double
        lib.oracle_bucket_lo.argtypes = [C.c_int]
        lib.oracle_bucket_lo.restype = C.c_double
        lib.oracle_select.argtypes = [np.ctypeslib.ndpointer(np.uint64, flags="C"), C.c_double]
        lib.oracle_select.restype = C.c_int
        lib.oracle_filter_values.argtypes = [C.c_int64, _PD, C.c_double,
                                             np.ctypeslib.ndpointer(np.uint8, flags="C"),
                                             C.POINTER(C.c_double)]
        lib.oracle_filter_values.restype = C.c_int
        lib.oracle_nsf_budget.argtypes = [C.c_double] * 5
        lib.oracle_nsf_budget.restype = C.c_double
        lib.oracle_nmf_budget.argtypes = [C.c_double] * 6
        lib.oracle_nmf_budget.restype = C.c_double
        pp = [C.POINTER(C.POINTER(C.c_int64)), C.POINTER(C.POINTER(C.c_int32)),
              C.POINTER(C.POINTER(C.c_double)), C.POINTER(C.c_int64)]
        lib.oracle_spgemm.argtypes = [C.c_int64, _P64, _P32, _PD, _P64, _P32, _PD] + pp
        lib.oracle_spgemm.restype = C.c_int
        lib.oracle_ns_step.argtypes = [C.c_int64, _P64, _P32, _PD] + pp
        lib.oracle_ns_step.restype = C.c_int
        lib.oracle_free_csr.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        lib.oracle_norm_inf.argtypes = [C.c_int64, _P64, _P32, _PD]
        lib.oracle_norm_inf.restype = C.c_double
        _lib = lib
        return lib


@dataclasses.dataclass
class OracleResult:
    status: str
    indptr: np.ndarray
    indices: np.ndarray
    data: np.ndarray
    n: int
    iters: int
    stagnated: bool
    scale: float
    res_fro: float
    step_fro: float
    trace: dict

    @property
    def nnz(self):
        return int(self.indptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.data, self.indices, self.indptr), shape=(self.n, self.n))


def _arrays(A):
    return (np.ascontiguousarray(A.indptr, dtype=np.int64),
            np.ascontiguousarray(A.indices, dtype=np.int32),
            np.ascontiguousarray(A.data, dtype=np.float64))


def _opts(tol, stop_rule, c_fixed, switch_res, max_iter, filter_y, scale, nthreads):
    return _Opts(tol=tol, stop_rule=stop_rule, c_fixed=c_fixed, switch_res=switch_res,
                 max_iter=max_iter, filter_y=filter_y, scale=scale, nthreads=nthreads,
                 trace_cap=max_iter + 2)


def _collect(lib, res: _Res) -> OracleResult:
    n, nnz = res.n, res.nnz
    if res.rp:
        indptr = np.ctypeslib.as_array(res.rp, shape=(n + 1,)).copy()
        indices = np.ctypeslib.as_array(res.ci, shape=(max(nnz, 1),))[:nnz].copy()
        data = np.ctypeslib.as_array(res.v, shape=(max(nnz, 1),))[:nnz].copy()
    else:
        indptr = np.zeros(1, np.int64); indices = np.zeros(0, np.int32); data = np.zeros(0)
    k = res.iters + 1
    tr = {}
    if res.e:
        for name in ("e", "d", "tau", "xfro", "ffro"):
            tr[name] = np.ctypeslib.as_array(getattr(res, name), shape=(k,)).copy()
        for name in ("nnz_x", "nnz_bar", "nnz_r"):
            tr[name] = np.ctypeslib.as_array(getattr(res, name), shape=(k,)).copy()
        tr["bstar"] = np.ctypeslib.as_array(res.bstar, shape=(k,)).copy()
    tr["inner_total"] = int(res.inner_total)
    out = OracleResult(status=STATUS.get(res.status, str(res.status)), indptr=indptr,
                       indices=indices, data=data, n=int(n), iters=int(res.iters),
                       stagnated=bool(res.stagnated), scale=float(res.scale),
                       res_fro=float(res.res_fro), step_fro=float(res.step_fro), trace=tr)
    lib.oracle_free_result(C.byref(res))
    return out


def nsf(A, tol: float = 1e-12, stop_rule: int = 0, c_fixed: float = 1e-4,
        switch_res: float = 1e-6, max_iter: int = 100, filter_y: int = 0, scale: float = 0.0,
        nthreads: int = 0) -> OracleResult:
    """Filtered Newton-Schulz (Algorithm 3.2.1) on a CSR matrix with fields indptr/indices/data."""
    lib = load()
    rp, ci, v = _arrays(A)
    o = _opts(tol, stop_rule, c_fixed, switch_res, max_iter, filter_y, scale, nthreads)
    res = _Res()
    lib.oracle_nsf(int(A.n if hasattr(A, "n") else len(rp) - 1), rp, ci, v, C.byref(o),
                   C.byref(res))
    return _collect(lib, res)


def nmf(A, tol: float = 1e-12, c_fixed: float = 1e-4, switch_res: float = 1e-6,
        max_iter: int = 100, scale: float = 1.0, nthreads: int = 0) -> OracleResult:
    """Filtered Newton (Algorithm 3.1.1), inverse by filtered Newton-Schulz inversion."""
    lib = load()
    rp, ci, v = _arrays(A)
    o = _opts(tol, 0, c_fixed, switch_res, max_iter, 0, scale, nthreads)
    res = _Res()
    lib.oracle_nmf(int(len(rp) - 1), rp, ci, v, C.byref(o), C.byref(res))
    return _collect(lib, res)


def _take_csr(lib, n, rp, ci, v, nnz):
    indptr = np.ctypeslib.as_array(rp, shape=(n + 1,)).copy()
    m = nnz.value
    indices = np.ctypeslib.as_array(ci, shape=(max(m, 1),))[:m].copy()
    data = np.ctypeslib.as_array(v, shape=(max(m, 1),))[:m].copy()
    lib.oracle_free_csr(C.cast(rp, C.c_void_p), C.cast(ci, C.c_void_p), C.cast(v, C.c_void_p))
    return indptr, indices, data


def spgemm(A, B):
    """Plain Gustavson product A*B (exact zeros dropped, sorted columns)."""
    lib = load()
    n = len(A.indptr) - 1
    a = _arrays(A); b = _arrays(B)
    rp = C.POINTER(C.c_int64)(); ci = C.POINTER(C.c_int32)(); v = C.POINTER(C.c_double)()
    nnz = C.c_int64()
    st = lib.oracle_spgemm(n, *a, *b, C.byref(rp), C.byref(ci), C.byref(v), C.byref(nnz))
    if st != 0:
        raise MemoryError("oracle_spgemm failed")
    return _take_csr(lib, n, rp, ci, v, nnz)


def ns_step(X):
    """One unfiltered Newton-Schulz update X + 1/2 X (I - X^2)."""
    lib = load()
    n = len(X.indptr) - 1
    rp = C.POINTER(C.c_int64)(); ci = C.POINTER(C.c_int32)(); v = C.POINTER(C.c_double)()
    nnz = C.c_int64()
    st = lib.oracle_ns_step(n, *_arrays(X), C.byref(rp), C.byref(ci), C.byref(v), C.byref(nnz))
    if st != 0:
        raise MemoryError("oracle_ns_step failed")
    return _take_csr(lib, n, rp, ci, v, nnz)


def bucket(x: float) -> int:
    return int(load().oracle_bucket(float(x)))


def bucket_hi(b: int) -> float:
    return float(load().oracle_bucket_hi(int(b)))


def bucket_lo(b: int) -> float:
    return float(load().oracle_bucket_lo(int(b)))


def select(counts: np.ndarray, tau: float) -> int:
    c = np.zeros(2048, np.uint64)
    c[: len(counts)] = counts
    return int(load().oracle_select(c, float(tau)))


def filter_values(vals: np.ndarray, tau: float):
    """Returns (bstar, keep mask, dropped sum of squares) for a flat value array."""
    v = np.ascontiguousarray(vals, dtype=np.float64)
    keep = np.zeros(len(v), np.uint8)
    dsq = C.c_double()
    b = load().oracle_filter_values(len(v), v, float(tau), keep, C.byref(dsq))
    return int(b), keep.astype(bool), float(dsq.value)


def nsf_budget(e, xfro, tol, c_fixed=1e-4, switch_res=1e-6) -> float:
    return float(load().oracle_nsf_budget(e, xfro, tol, c_fixed, switch_res))


def nmf_budget(e, xfro, zfro, tol, c_fixed=1e-4, switch_res=1e-6) -> float:
    return float(load().oracle_nmf_budget(e, xfro, zfro, tol, c_fixed, switch_res))


def norm_inf(A) -> float:
    return float(load().oracle_norm_inf(len(A.indptr) - 1, *_arrays(A)))
