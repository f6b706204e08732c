"""Whole-matrix checksum of a CSR result, shared by the golden-data script and
the GPU tests (test infrastructure; none of the method's arithmetic).

Row probe p_i = sum_j X_ij w(i, j) with w(i, j) = +-1 from an integer hash of
(i, j).  For two matrices X and S on any patterns, p_i(X) - p_i(S) =
sum_j (X - S)_ij w(i, j), whose square has expectation ||(X - S)_i||^2 when the
signs behave as independent fair coins, so sum_i (p_i(X) - p_i(S))^2 estimates
||X - S||_F^2 with every entry of either matrix taking part.  The hash stays
below 2^63 at every step, so numpy int64 and torch int64 give the same bits.
"""
import numpy as np

_M1 = 0x9E3779B1
_M2 = 0x85EBCA77
_M3 = 0x45D9F3B
_MASK = 0xFFFFFFFF


def weights(rows, cols, xp=np):
    """+-1 (as float64) for int64 arrays rows, cols of the same shape (values < 2^31)."""
    h = (rows * _M1) ^ (cols * _M2)
    h = h & _MASK
    h = (((h >> 16) ^ h) * _M3) & _MASK
    h = (((h >> 16) ^ h) * _M3) & _MASK
    h = (h >> 16) ^ h
    b = h & 1
    if xp is np:
        return 1.0 - 2.0 * b.astype(np.float64)
    return 1.0 - 2.0 * b.to(xp.float64)


def row_probe_numpy(indptr, indices, data):
    n = len(indptr) - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(indptr))
    w = weights(rows, indices.astype(np.int64))
    return np.bincount(rows, weights=data * w, minlength=n)


def row_probe_torch(row_ptr, col, val, chunk=1 << 26):
    """Same probe on device tensors (int64 row_ptr, int32 col, float val)."""
    import torch
    n = row_ptr.numel() - 1
    out = torch.zeros(n, dtype=torch.float64, device=row_ptr.device)
    nnz = col.numel()
    for s0 in range(0, nnz, chunk):
        s1 = min(nnz, s0 + chunk)
        pos = torch.arange(s0, s1, device=row_ptr.device, dtype=torch.int64)
        r = torch.searchsorted(row_ptr, pos, right=True) - 1
        w = weights(r, col[s0:s1].long(), xp=torch)
        out.index_add_(0, r, val[s0:s1].double() * w)
    return out
