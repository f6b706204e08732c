"""Parity at the full workload sizes, in the launch configuration bench.py times.

The FP64 oracle cannot solve these sizes in a test, so the HIP results are
checked on sampled rows the oracle side can compute one by one: row i of the
dense sign of the principal patch on the ball of graph radius r around i
(exponential decay of the sign of a gapped matrix makes the patch row equal to
row i of sign(A) to about q^r), plus properties that hold at any size: X^2 = I
and XA = AX on sampled rows, and trace(X) = (# eigenvalues right) - (# left),
which the staggered gap term fixes as the sum of (-1)^(x+y(+z)).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as cf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sf():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    import paper_2210_03356_amd as pkg
    pkg.load()
    return pkg


def _rows(A):
    """Sampled rows: the centre, a centre-row neighbour, both ends, an edge
    middle and a random row."""
    n = A.n
    N = int(A.meta["shape"][0]) if "shape" in A.meta else int(round(math.sqrt(n)))
    rng = np.random.default_rng(11)
    return sorted({n // 2, n // 2 + N // 2, 0, n - 1, N // 2, int(rng.integers(0, n))})


def _row_error(got, idx, ref):
    """||got_i - ref_i|| / ||ref_i|| with got entries outside the patch counted in full."""
    cols, vals = got
    vals = vals.astype(np.float64)
    pos = np.searchsorted(idx, cols)
    inside = (pos < len(idx)) & (idx[np.minimum(pos, len(idx) - 1)] == cols)
    g = np.zeros(len(idx))
    g[pos[inside]] = vals[inside]
    out = float(np.sum(vals[~inside] ** 2))
    return math.sqrt(float(np.sum((g - ref) ** 2)) + out) / float(np.linalg.norm(ref))


def _properties(res, A, rows):
    """max over rows of ||(X^2 - I)_i|| and ||(XA - AX)_i|| / (||X_i|| ||A||_inf)."""
    xr = res.rows(rows)
    need = set()
    for i in rows:
        need.update(int(k) for k in xr[i][0])
        need.update(int(j) for j in A.indices[A.indptr[i]:A.indptr[i + 1]])
    xk = res.rows(sorted(need))
    anorm = float(np.max(np.add.reduceat(np.abs(A.data), A.indptr[:-1])))
    sq, comm = 0.0, 0.0
    for i in rows:
        ci, va = xr[i]
        va = va.astype(np.float64)
        x2 = np.zeros(A.n)
        xa = np.zeros(A.n)
        for k, v in zip(ci, va):
            kc, kv = xk[int(k)]
            x2[kc] += v * kv.astype(np.float64)
            b, e = A.indptr[int(k)], A.indptr[int(k) + 1]
            xa[A.indices[b:e]] += v * A.data[b:e]
        x2[i] -= 1.0
        for j, a in zip(A.indices[A.indptr[i]:A.indptr[i + 1]],
                        A.data[A.indptr[i]:A.indptr[i + 1]]):
            jc, jv = xk[int(j)]
            xa[jc] -= a * jv.astype(np.float64)
        sq = max(sq, float(np.linalg.norm(x2)))
        comm = max(comm, float(np.linalg.norm(xa)) / (float(np.linalg.norm(va)) * anorm))
    return sq, comm


def _trace(res):
    import torch
    import paper_2210_03356_amd as pkg
    pkg.release_cached()
    rp, ci, va = res.to_torch()
    n = rp.numel() - 1
    r = torch.repeat_interleave(torch.arange(n, device=rp.device), rp[1:] - rp[:-1])
    return float(va[ci.long() == r].double().sum())


def _check_sampled(res, A, ref_row, rel_tol):
    rows = _rows(A)
    got = res.rows(rows)
    worst = 0.0
    for i in rows:
        idx, ref = ref_row(i)
        worst = max(worst, _row_error(got[i], idx, ref))
    assert worst <= rel_tol, worst
    sq, comm = _properties(res, A, rows)
    assert sq <= 1e-8, sq
    # a relative error q of X shows as a relative commutator of about 2q|lambda|/||A||,
    # so the commutator is held to the accuracy bound itself (1e-10 in FP64)
    assert comm <= rel_tol, comm
    t = _trace(res)
    assert abs(t - A.meta["inertia"]) <= 1e-6 * A.n, (t, A.meta["inertia"])
    return worst


def _c3_scaling(A):
    """d with D^-1 A D symmetric for upwind convection-diffusion (x fastest):
    the west coupling is (1+b) times the east one, so d_x = (1+b)^(x/2)."""
    N = int(A.meta["shape"][0])
    return np.sqrt(1.0 + A.meta["b"]) ** (np.arange(A.n) % N)


def test_c2_full_fp64(sf):
    """2D 256 x 256, FP64, tol 1e-12: sampled rows within 1e-10 of the sign."""
    A = W.config_matrix("c2")
    res = sf.sign_ns(sf.DeviceCsr.from_host(A), sf.default_opts(tol=1e-12))
    assert res.status == "OK"
    _check_sampled(res, A, lambda i: cf.local_sign_row(A, i, 34), 1e-10)


def test_c2_full_mixed(sf):
    """The same workload with FP32 bulk products and FP64 polish: within 1e-8."""
    A = W.config_matrix("c2")
    res = sf.sign_ns(sf.DeviceCsr.from_host(A), sf.default_opts(tol=1e-12, precision=1))
    assert res.status == "OK"
    _check_sampled(res, A, lambda i: cf.local_sign_row(A, i, 34), 1e-8)


def test_c2_full_newton(sf):
    """Filtered Newton (inverse by filtered Newton-Schulz) at full size."""
    A = W.config_matrix("c2")
    res = sf.sign_newton(sf.DeviceCsr.from_host(A), sf.default_opts(tol=1e-12))
    assert res.status == "OK"
    _check_sampled(res, A, lambda i: cf.local_sign_row(A, i, 34), 1e-10)


@pytest.mark.parametrize("precision,rel_tol", [(1, 1e-8), (0, 1e-10)])
def test_c3_full(sf, precision, rel_tol):
    """2D 512 x 512 upwind convection-diffusion (nonsymmetric), filter_y on,
    mixed precision as configured and plain FP64."""
    A = W.config_matrix("c3")
    d = _c3_scaling(A)
    res = sf.sign_ns(sf.DeviceCsr.from_host(A),
                     sf.default_opts(tol=1e-12, filter_y=1, precision=precision))
    assert res.status == "OK"
    _check_sampled(res, A, lambda i: cf.local_sign_row_similar(A, i, 34, d), rel_tol)


@pytest.mark.parametrize("precision,rel_tol", [(1, 1e-8), (0, 1e-10)])
def test_c4_scaled_against_dense_sign(sf, precision, rel_tol):
    """3D 7-point on 16^3 (the largest 3D grid whose dense sign a test can form):
    the whole result against the dense eigendecomposition sign."""
    A = W.config_matrix("c4", N=16)
    res = sf.sign_ns(sf.DeviceCsr.from_host(A),
                     sf.default_opts(tol=1e-10, filter_y=1, precision=precision))
    assert res.status == "OK"
    S = cf.dense_sign_sym(A.to_scipy().toarray())
    X = res.to_scipy().toarray()
    assert np.linalg.norm(X - S) / np.linalg.norm(S) <= rel_tol
    assert abs(np.trace(X) - A.meta["inertia"]) <= 1e-6


def test_c1_full_against_closed_form(sf):
    """1D tridiag(-1, 0, -1), n = 1024, stop rule on the step: the whole result
    against the sine-basis closed form."""
    A = W.config_matrix("c1")
    res = sf.sign_ns(sf.DeviceCsr.from_host(A), sf.default_opts(tol=1e-12, stop_rule=1))
    assert res.status == "OK"
    X = res.to_scipy().toarray()
    S = cf.sign_tridiag_c1(A.n)
    assert np.linalg.norm(X - S) / math.sqrt(A.n) <= 1e-10
    assert np.linalg.norm(X @ X - np.eye(A.n)) <= 1e-8
