"""Thin ctypes binding of libsignfn (argument marshalling only).

Every computation runs inside ``libsignfn.so`` (HIP kernels for gfx950).
PyTorch provides device memory for inputs and the HIP stream; results live in
library-owned device buffers and are copied out on request.  If the shared
library is missing, :func:`load` raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsignfn.so")

SIGN_OK, SIGN_PENDING = 0, 1
STATUS = {0: "OK", 1: "PENDING", -1: "EINVAL", -2: "ENOMEM", -3: "ENOCONV", -4: "EDIVERGED",
          -5: "EDEVICE", -6: "EBUSY", -7: "ENOTFOUND"}


class SignError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class sign_csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p), ("val_f32", C.c_int)]


_ALLOC = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class sign_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("stop_rule", C.c_int), ("c_fixed", C.c_double),
                ("switch_res", C.c_double), ("max_iter", C.c_int), ("precision", C.c_int),
                ("polish_steps", C.c_int), ("refine_steps", C.c_int), ("filter_y", C.c_int),
                ("scale", C.c_double), ("staging_bytes", C.c_size_t), ("alloc", _ALLOC),
                ("free", _FREE), ("alloc_ctx", C.c_void_p)]


class sign_stats(C.Structure):
    _fields_ = [("status", C.c_int), ("iters", C.c_int), ("stagnated", C.c_int),
                ("scale", C.c_double), ("res_fro", C.c_double), ("step_fro", C.c_double),
                ("nnz", C.c_int64), ("seconds", C.c_double), ("products", C.c_int64),
                ("spgemm_ms", C.c_double), ("spgemm_bytes", C.c_double),
                ("inner_steps", C.c_int), ("comm_rel", C.c_double), ("hot_tile", C.c_int),
                ("hot_threads", C.c_int), ("hot_fp32", C.c_int), ("hot_group", C.c_int),
                ("hot_launches", C.c_int64),
                ("hot_ms", C.c_double),
                ("hot_bytes", C.c_double), ("hot_products", C.c_int64),
                ("hot_gathered", C.c_int64), ("hot_regtile", C.c_int),
                ("madds", C.c_int64), ("hot_madds", C.c_int64), ("hot_pages", C.c_int)]


class sign_iter_stats(C.Structure):
    _fields_ = [("e", C.c_double), ("d", C.c_double), ("tau", C.c_double),
                ("xfro", C.c_double), ("ffro", C.c_double), ("nnz_x", C.c_int64),
                ("nnz_r", C.c_int64), ("nnz_bar", C.c_int64), ("bstar", C.c_int),
                ("fp32", C.c_int), ("e_bound", C.c_int), ("ms", C.c_double)]


class sign_server_opts(C.Structure):
    _fields_ = [("device", C.c_int), ("hbm_budget_bytes", C.c_size_t), ("max_slots", C.c_int),
                ("max_queue", C.c_int), ("mem_limit_bytes", C.c_size_t)]


class sign_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("active", C.c_int64),
                ("queued", C.c_int64), ("p50_ms", C.c_double), ("p99_ms", C.c_double),
                ("busy_seconds", C.c_double), ("ticks", C.c_int64), ("max_active", C.c_int64),
                ("failed", C.c_int64), ("relayout_seconds", C.c_double),
                ("residual_seconds", C.c_double), ("update_seconds", C.c_double),
                ("filter_seconds", C.c_double)]


_lib = None
_hip = None


def load():
    """Load libsignfn.so (built in-tree by ``build.py``); raise if absent."""
    global _lib, _hip
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2210_03356_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER
    lib.sign_opts_default.argtypes = [P(sign_opts)]
    lib.sign_opts_default.restype = None
    for name in ("sign_ns", "sign_newton"):
        f = getattr(lib, name)
        f.argtypes = [P(sign_csr), P(sign_opts), C.c_void_p, P(C.c_void_p)]
        f.restype = C.c_int
    lib.sign_spgemm.argtypes = [P(sign_csr), P(sign_csr), C.c_void_p, P(C.c_void_p)]
    lib.sign_spgemm.restype = C.c_int
    lib.sign_filter.argtypes = [P(sign_csr), C.c_double, C.c_void_p, P(C.c_void_p), P(C.c_int)]
    lib.sign_filter.restype = C.c_int
    lib.sign_filter_noalloc.argtypes = [P(sign_csr), C.c_double, C.c_void_p, P(sign_csr),
                                        C.c_int64, P(C.c_int), P(C.c_double)]
    lib.sign_filter_noalloc.restype = C.c_int
    lib.sign_result_csr.argtypes = [C.c_void_p, P(sign_csr)]
    lib.sign_result_csr.restype = C.c_int
    lib.sign_result_stats.argtypes = [C.c_void_p, P(sign_stats)]
    lib.sign_result_stats.restype = C.c_int
    lib.sign_result_trace.argtypes = [C.c_void_p, C.c_int, P(sign_iter_stats)]
    lib.sign_result_trace.restype = C.c_int
    lib.sign_result_free.argtypes = [C.c_void_p]
    lib.sign_result_free.restype = None
    lib.sign_last_error.argtypes = []
    lib.sign_last_error.restype = C.c_char_p
    lib.sign_release_cached.argtypes = []
    lib.sign_release_cached.restype = C.c_size_t
    lib.sign_server_create.argtypes = [P(sign_server_opts), P(C.c_void_p)]
    lib.sign_server_create.restype = C.c_int
    lib.sign_serve_submit.argtypes = [C.c_void_p, P(sign_csr), P(sign_opts), P(C.c_uint64)]
    lib.sign_serve_submit.restype = C.c_int
    lib.sign_serve_poll.argtypes = [C.c_void_p, C.c_uint64, P(C.c_void_p)]
    lib.sign_serve_poll.restype = C.c_int
    lib.sign_server_stats_get.argtypes = [C.c_void_p, P(sign_server_stats)]
    lib.sign_server_stats_get.restype = C.c_int
    lib.sign_server_destroy.argtypes = [C.c_void_p]
    lib.sign_server_destroy.restype = None
    _lib = lib
    _hip = C.CDLL("libamdhip64.so")
    _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    _hip.hipMemcpy.restype = C.c_int
    return lib


def _err(status: int) -> SignError:
    return SignError(status, load().sign_last_error().decode(errors="replace"))


def default_opts(**kw) -> sign_opts:
    o = sign_opts()
    load().sign_opts_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _stream_ptr(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


class DeviceCsr:
    """CSR held in torch device tensors (row_ptr int64, col int32, val f64/f32)."""

    def __init__(self, n, row_ptr, col, val):
        import torch
        assert row_ptr.dtype == torch.int64 and col.dtype == torch.int32
        assert val.dtype in (torch.float64, torch.float32)
        self.n = int(n)
        self.row_ptr, self.col, self.val = row_ptr.contiguous(), col.contiguous(), val.contiguous()

    @classmethod
    def from_host(cls, A, device="cuda", dtype=None):
        """From any object with n/indptr/indices/data (e.g. workloads.Csr)."""
        import torch
        n = A.n if hasattr(A, "n") else A.shape[0]
        data = np.asarray(A.data)
        if dtype is not None:
            data = data.astype(dtype)
        return cls(n, torch.as_tensor(np.asarray(A.indptr, np.int64), device=device),
                   torch.as_tensor(np.asarray(A.indices, np.int32), device=device),
                   torch.as_tensor(data, device=device))

    def struct(self) -> sign_csr:
        import torch
        return sign_csr(n=self.n, nnz=int(self.col.numel()), row_ptr=self.row_ptr.data_ptr(),
                        col=self.col.data_ptr() if self.col.numel() else None,
                        val=self.val.data_ptr() if self.val.numel() else None,
                        val_f32=int(self.val.dtype == torch.float32))


class Result:
    """Owns a sign_result*; copies its CSR out on request."""

    def __init__(self, ptr: int, status: int):
        self._ptr = C.c_void_p(ptr)
        self.status = STATUS.get(status, str(status))

    def __del__(self):
        if getattr(self, "_ptr", None) and self._ptr.value and _lib is not None:
            _lib.sign_result_free(self._ptr)
            self._ptr = C.c_void_p(None)

    def view(self) -> sign_csr:
        v = sign_csr()
        st = load().sign_result_csr(self._ptr, C.byref(v))
        if st != 0:
            raise _err(st)
        return v

    def stats(self) -> dict:
        s = sign_stats()
        load().sign_result_stats(self._ptr, C.byref(s))
        return {f: getattr(s, f) for f, _ in sign_stats._fields_}

    def trace(self) -> list:
        out = []
        k = 0
        while True:
            it = sign_iter_stats()
            if load().sign_result_trace(self._ptr, k, C.byref(it)) != 0:
                break
            out.append({f: getattr(it, f) for f, _ in sign_iter_stats._fields_})
            k += 1
        return out

    def to_numpy(self):
        """(indptr int64, indices int32, data float64/float32) host copies."""
        v = self.view()
        load()
        rp = np.empty(v.n + 1, np.int64)
        ci = np.empty(v.nnz, np.int32)
        va = np.empty(v.nnz, np.float32 if v.val_f32 else np.float64)
        _copy_d2h(rp, v.row_ptr)
        if v.nnz:
            _copy_d2h(ci, v.col)
            _copy_d2h(va, v.val)
        return rp, ci, va

    def rows(self, idx):
        """Host copies of the listed rows only: {i: (columns int32, values)}."""
        v = self.view()
        load()
        rp = np.empty(v.n + 1, np.int64)
        _copy_d2h(rp, v.row_ptr)
        isz = 4
        vsz = 4 if v.val_f32 else 8
        out = {}
        for i in sorted(set(int(i) for i in idx)):
            b, e = int(rp[i]), int(rp[i + 1])
            ci = np.empty(e - b, np.int32)
            va = np.empty(e - b, np.float32 if v.val_f32 else np.float64)
            if e > b:
                _copy_d2h(ci, v.col + b * isz)
                _copy_d2h(va, v.val + b * vsz)
            out[i] = (ci, va)
        return out

    def to_scipy(self):
        import scipy.sparse as sp
        rp, ci, va = self.to_numpy()
        n = len(rp) - 1
        return sp.csr_matrix((va, ci, rp), shape=(n, n))

    def to_torch(self, device="cuda"):
        """Device copies as torch tensors (row_ptr, col, val)."""
        import torch
        v = self.view()
        rp = torch.empty(v.n + 1, dtype=torch.int64, device=device)
        ci = torch.empty(v.nnz, dtype=torch.int32, device=device)
        va = torch.empty(v.nnz, dtype=torch.float32 if v.val_f32 else torch.float64, device=device)
        torch.cuda.synchronize()
        _copy_d2d(rp.data_ptr(), v.row_ptr, 8 * (v.n + 1))
        if v.nnz:
            _copy_d2d(ci.data_ptr(), v.col, 4 * v.nnz)
            _copy_d2d(va.data_ptr(), v.val, va.element_size() * v.nnz)
        return rp, ci, va


def _copy_d2h(dst: np.ndarray, src_ptr) -> None:
    st = _hip.hipMemcpy(dst.ctypes.data, src_ptr, dst.nbytes, 2)  # hipMemcpyDeviceToHost
    if st != 0:
        raise RuntimeError(f"hipMemcpy failed ({st})")


def _copy_d2d(dst_ptr, src_ptr, nbytes: int) -> None:
    st = _hip.hipMemcpy(dst_ptr, src_ptr, nbytes, 3)  # hipMemcpyDeviceToDevice
    if st != 0:
        raise RuntimeError(f"hipMemcpy failed ({st})")


def _call(fn, *args) -> Result:
    out = C.c_void_p()
    st = fn(*args, C.byref(out))
    if out.value is None:
        raise _err(st)
    return Result(out.value, st)


def release_cached() -> int:
    """Returns the library's cached idle device memory to HIP; bytes released."""
    return int(load().sign_release_cached())


def sign_ns(A: DeviceCsr, opts: Optional[sign_opts] = None, stream=None) -> Result:
    o = opts if opts is not None else default_opts()
    a = A.struct()
    return _call(load().sign_ns, C.byref(a), C.byref(o), C.c_void_p(_stream_ptr(stream)))


def sign_newton(A: DeviceCsr, opts: Optional[sign_opts] = None, stream=None) -> Result:
    o = opts if opts is not None else default_opts()
    a = A.struct()
    return _call(load().sign_newton, C.byref(a), C.byref(o), C.c_void_p(_stream_ptr(stream)))


def sign_spgemm(A: DeviceCsr, B: DeviceCsr, stream=None) -> Result:
    a, b = A.struct(), B.struct()
    return _call(load().sign_spgemm, C.byref(a), C.byref(b), C.c_void_p(_stream_ptr(stream)))


def sign_filter(A: DeviceCsr, tau: float, stream=None):
    a = A.struct()
    b = C.c_int(-1)
    out = C.c_void_p()
    st = load().sign_filter(C.byref(a), float(tau), C.c_void_p(_stream_ptr(stream)),
                            C.byref(out), C.byref(b))
    if out.value is None:
        raise _err(st)
    return Result(out.value, st), int(b.value)


NOALLOC_MAX_ROWS = 1048576  # SIGN_NOALLOC_MAX_ROWS


def sign_filter_noalloc(A: DeviceCsr, tau: float, out_row_ptr, out_col, out_val, stream=None):
    """sign_filter into caller-owned device tensors (int64 row_ptr of n+1, int32 col and
    float64 val of equal capacity); the library allocates no device memory.  Returns
    (nnz kept, cut bucket, ||F||_F of the dropped part)."""
    import torch
    assert out_row_ptr.dtype == torch.int64 and out_row_ptr.numel() >= A.n + 1
    assert out_col.dtype == torch.int32 and out_val.dtype == torch.float64
    cap = min(out_col.numel(), out_val.numel())
    a = A.struct()
    o = sign_csr(n=0, nnz=0, row_ptr=out_row_ptr.data_ptr(),
                 col=out_col.data_ptr() if cap else None,
                 val=out_val.data_ptr() if cap else None, val_f32=0)
    b = C.c_int(-1)
    d = C.c_double(0.0)
    st = load().sign_filter_noalloc(C.byref(a), float(tau), C.c_void_p(_stream_ptr(stream)),
                                    C.byref(o), cap, C.byref(b), C.byref(d))
    if st != 0:
        raise _err(st)
    return int(o.nnz), int(b.value), float(d.value)


class Server:
    """Continuous-batching server (sign_server_*); requests are host CSR."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0, max_slots: int = 0,
                 max_queue: int = 0, mem_limit_bytes: int = 0):
        o = sign_server_opts(device=device, hbm_budget_bytes=hbm_budget_bytes,
                             max_slots=max_slots, max_queue=max_queue,
                             mem_limit_bytes=mem_limit_bytes)
        p = C.c_void_p()
        st = load().sign_server_create(C.byref(o), C.byref(p))
        if st != 0:
            raise _err(st)
        self._p = p

    def submit(self, A, opts: Optional[sign_opts] = None) -> int:
        rp = np.ascontiguousarray(A.indptr, np.int64)
        ci = np.ascontiguousarray(A.indices, np.int32)
        va = np.ascontiguousarray(A.data, np.float64)
        s = sign_csr(n=len(rp) - 1, nnz=len(ci), row_ptr=rp.ctypes.data, col=ci.ctypes.data,
                     val=va.ctypes.data, val_f32=0)
        o = opts if opts is not None else default_opts()
        t = C.c_uint64()
        st = load().sign_serve_submit(self._p, C.byref(s), C.byref(o), C.byref(t))
        if st != 0:
            raise _err(st)
        return int(t.value)

    def poll(self, ticket: int):
        out = C.c_void_p()
        st = load().sign_serve_poll(self._p, C.c_uint64(ticket), C.byref(out))
        if st == SIGN_PENDING:
            return None
        if out.value is None:
            raise _err(st)
        return Result(out.value, st)

    def stats(self) -> dict:
        s = sign_server_stats()
        st = load().sign_server_stats_get(self._p, C.byref(s))
        if st != 0:
            raise _err(st)
        return {f: getattr(s, f) for f, _ in sign_server_stats._fields_}

    def close(self):
        if self._p and self._p.value:
            load().sign_server_destroy(self._p)
            self._p = C.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
