"""sign_filter_noalloc (the allocation-free filter) against sign_filter, through
the C ABI: same kept entries, values, cut bucket and dropped norm, bit for bit,
on two calls in a row into the same caller buffers, the second on a smaller
input, so that state left in the shared scratch array by the first call cannot
leak into the second.  Also against the oracle's selection, and the error paths
that the host detects before or after the kernels (no kernel is made to fail)."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sf():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    import paper_2210_03356_amd as pkg
    pkg.load()
    oracle.build(force=False)
    return pkg


def _matrix(n, seed, mean_row):
    rng = np.random.default_rng(seed)
    A = W.random_sparse(n, mean_row=mean_row, seed=seed + 50)
    A.data = np.exp(rng.uniform(-80, 1, A.nnz)) * rng.choice([-1, 1], A.nnz)
    A.data[A.data > 1] = 0.75
    tau = float(np.exp(rng.uniform(-60, -5)))
    return A, tau


def _noalloc(sf, dA, tau, bufs):
    import torch
    rp, col, val = bufs
    nnz, b, dropped = sf.sign_filter_noalloc(dA, tau, rp, col, val)
    torch.cuda.synchronize()
    return (rp[: dA.n + 1].cpu().numpy(), col[:nnz].cpu().numpy(), val[:nnz].cpu().numpy(),
            b, dropped)


def _same_as_sign_filter(sf, A, tau, bufs, dtype=None):
    dA = sf.DeviceCsr.from_host(A, dtype=dtype)
    ref, b_ref = sf.sign_filter(dA, tau)
    rrp, rci, rva = ref.to_numpy()
    rp, ci, va, b, dropped = _noalloc(sf, dA, tau, bufs)
    assert b == b_ref
    assert np.array_equal(rp, rrp)
    assert np.array_equal(ci, rci)
    assert np.array_equal(va, rva)        # the same kernels in the same order: bit-exact
    assert dropped == ref.stats()["step_fro"]
    assert dropped <= tau
    # and the oracle's selection (the cut and the kept set are exact decisions)
    b_or, keep, _ = oracle.filter_values(A.data.astype(dtype or np.float64).astype(np.float64),
                                         tau)
    assert b == b_or
    assert int(rp[-1]) == int(keep.sum())
    return b


def test_noalloc_matches_sign_filter_twice_shrinking(sf):
    import torch
    A1, t1 = _matrix(20000, 3, 24)
    A2, t2 = _matrix(3001, 4, 9)       # second call: fewer rows, fewer entries
    cap = A1.nnz
    bufs = (torch.full((A1.n + 1,), -7, dtype=torch.int64, device="cuda"),
            torch.full((cap,), -7, dtype=torch.int32, device="cuda"),
            torch.full((cap,), float("nan"), dtype=torch.float64, device="cuda"))
    _same_as_sign_filter(sf, A1, t1, bufs)
    _same_as_sign_filter(sf, A2, t2, bufs)


def test_noalloc_fp32_input_and_edges(sf):
    import torch
    A, tau = _matrix(4097, 7, 12)
    bufs = (torch.empty(A.n + 1, dtype=torch.int64, device="cuda"),
            torch.empty(A.nnz, dtype=torch.int32, device="cuda"),
            torch.empty(A.nnz, dtype=torch.float64, device="cuda"))
    _same_as_sign_filter(sf, A, tau, bufs, dtype=np.float32)
    # zero budget keeps every nonzero; one row; an empty matrix of order 5
    _same_as_sign_filter(sf, A, 0.0, bufs)
    one = W.Csr(n=1, indptr=np.array([0, 1], np.int64), indices=np.array([0], np.int32),
                data=np.array([0.5]))
    _same_as_sign_filter(sf, one, 1e-3, bufs)
    empty = W.Csr(n=5, indptr=np.zeros(6, np.int64), indices=np.zeros(0, np.int32),
                  data=np.zeros(0))
    rp, ci, va, b, dropped = _noalloc(sf, sf.DeviceCsr.from_host(empty), 1e-3, bufs)
    assert np.array_equal(rp, np.zeros(6, np.int64)) and len(ci) == 0 and dropped == 0.0


def test_noalloc_errors(sf):
    import torch
    A, tau = _matrix(2000, 9, 10)
    dA = sf.DeviceCsr.from_host(A)
    ref, _ = sf.sign_filter(dA, tau)
    kept = ref.stats()["nnz"]
    small = (torch.empty(A.n + 1, dtype=torch.int64, device="cuda"),
             torch.empty(kept - 1, dtype=torch.int32, device="cuda"),
             torch.empty(kept - 1, dtype=torch.float64, device="cuda"))
    with pytest.raises(sf.SignError, match="ENOMEM"):
        sf.sign_filter_noalloc(dA, tau, *small)
    # the scratch array is intact afterwards
    bufs = (torch.empty(A.n + 1, dtype=torch.int64, device="cuda"),
            torch.empty(A.nnz, dtype=torch.int32, device="cuda"),
            torch.empty(A.nnz, dtype=torch.float64, device="cuda"))
    _same_as_sign_filter(sf, A, tau, bufs)
    # more rows than the scratch array is sized for: rejected before any GPU work
    big = sf.DeviceCsr(sf.NOALLOC_MAX_ROWS + 1,
                       torch.zeros(sf.NOALLOC_MAX_ROWS + 2, dtype=torch.int64, device="cuda"),
                       torch.zeros(0, dtype=torch.int32, device="cuda"),
                       torch.zeros(0, dtype=torch.float64, device="cuda"))
    bbufs = (torch.empty(sf.NOALLOC_MAX_ROWS + 2, dtype=torch.int64, device="cuda"),
             torch.empty(1, dtype=torch.int32, device="cuda"),
             torch.empty(1, dtype=torch.float64, device="cuda"))
    with pytest.raises(sf.SignError, match="row limit"):
        sf.sign_filter_noalloc(big, 1e-3, *bbufs)
    # a malformed input (columns not ascending) is reported, not computed on
    bad = W.Csr(n=3, indptr=np.array([0, 2, 2, 2], np.int64),
                indices=np.array([2, 1], np.int32), data=np.array([1.0, 2.0]))
    with pytest.raises(sf.SignError, match="ascending"):
        sf.sign_filter_noalloc(sf.DeviceCsr.from_host(bad), 1e-3, *bufs)
