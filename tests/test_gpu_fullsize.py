"""Parity at the full workload sizes, in the launch configuration bench.py times.

C2 (256 x 256) and C3 (512 x 512) are compared with the FP64 oracle's own solves
of the same matrices, stored by tests/golden/make_fullsize_golden.py (runs of
several minutes, too long for a test): the whole matrix through per-row hash
probes, which estimate ||X - S||_F, and entry by entry on complete stored rows.
Independently of the oracle, C3 rows are also checked against the dense sign of
the principal patch on a ball of graph radius 34 around them (the exponential
decay of the sign of a gapped matrix makes the patch row equal to the row of
sign(A) to about q^34), several hundred rows from shared patches, plus
properties that hold at any size: X^2 = I and XA = AX on sampled rows, and
trace(X) = (# eigenvalues right) - (# left), which the staggered gap term fixes
as the sum of (-1)^(x+y(+z)).
"""
import math
import os
import sys

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


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
if GOLDEN not in sys.path:
    sys.path.insert(0, GOLDEN)


def _golden(cfg):
    import make_fullsize_golden as mk
    g = dict(np.load(os.path.join(GOLDEN, f"{cfg}_fp64_oracle.npz")))
    A = W.config_matrix(cfg)
    assert str(g["fingerprint"]) == mk.fingerprint(A), f"{cfg} generator changed since the golden run"
    return A, g


@pytest.fixture(scope="module")
def c2_golden():
    """The FP64 oracle's solve of the full C2 matrix (tests/golden/
    make_fullsize_golden.py): summary, per-row probes and complete sample rows."""
    return _golden("c2")


@pytest.fixture(scope="module")
def c3_golden():
    """The same for C3 (the oracle's full solve, run on a host with the memory it
    needs)."""
    return _golden("c3")


def _check_against_oracle(res, g, rel_tol):
    """Whole matrix: sum_i (probe_i(X) - probe_i(S))^2 estimates ||X - S||_F^2 with
    every entry of X and S taking part (tests/golden/probe.py); entry by entry on
    the oracle's stored rows (union of the patterns); Frobenius norm and trace."""
    import torch
    import probe
    import paper_2210_03356_amd as pkg
    pkg.release_cached()
    rp, ci, va = res.to_torch()
    p = probe.row_probe_torch(rp, ci, va).cpu().numpy()
    xfro = float(torch.linalg.vector_norm(va.double()))
    del rp, ci, va
    torch.cuda.empty_cache()
    fro = float(g["fro"])
    est = math.sqrt(float(np.sum((p - g["probe"]) ** 2))) / fro
    assert est <= rel_tol, est
    assert abs(xfro - fro) <= rel_tol * fro, (xfro, fro)
    rows = g["rows"]
    got = res.rows(rows)
    off, worst, smax = 0, 0.0, 0.0
    for i, L in zip(rows, g["row_len"]):
        sc, sv = g["row_cols"][off:off + L], g["row_vals"][off:off + L]
        off += L
        gc_, gv = got[int(i)]
        u = np.union1d(sc, gc_)
        a = np.zeros(len(u))
        b = np.zeros(len(u))
        a[np.searchsorted(u, gc_)] = gv.astype(np.float64)
        b[np.searchsorted(u, sc)] = sv
        worst = max(worst, float(np.abs(a - b).max()) if len(u) else 0.0)
        smax = max(smax, float(np.abs(sv).max()) if L else 0.0)
    assert worst <= rel_tol * smax, (worst, smax)
    assert len(rows) >= 64
    return est, worst / smax


def test_c2_full_fp64(sf, c2_golden):
    """2D 256 x 256, FP64, tol 1e-12: the whole matrix against the FP64 oracle's
    (rel. Frobenius <= 1e-10, entry-wise <= 1e-10 max|S| on its stored rows), plus
    the sampled-row properties."""
    A, g = c2_golden
    res = sf.sign_ns(sf.DeviceCsr.from_host(A), sf.default_opts(tol=1e-12))
    assert res.status == "OK"
    _check_against_oracle(res, g, 1e-10)
    _check_sampled(res, A, lambda i: cf.local_sign_row(A, i, 34), 1e-10)


def test_c2_full_mixed(sf, c2_golden):
    """The same workload with FP32 bulk products and FP64 polish: within 1e-8 of
    the FP64 oracle, whole matrix and entry-wise."""
    A, g = c2_golden
    res = sf.sign_ns(sf.DeviceCsr.from_host(A), sf.default_opts(tol=1e-12, precision=1))
    assert res.status == "OK"
    _check_against_oracle(res, g, 1e-8)


def test_c2_full_newton(sf, c2_golden):
    """Filtered Newton (inverse by filtered Newton-Schulz) at full size: the sign is
    unique, so the FP64 NSF oracle's result is its reference too."""
    A, g = c2_golden
    res = sf.sign_newton(sf.DeviceCsr.from_host(A), sf.default_opts(tol=1e-12))
    assert res.status == "OK"
    _check_against_oracle(res, g, 1e-10)


# Patch centres (x, y) on the 512 x 512 grid: the centre, both sides of the
# half-row boundary where a new 64-group XCD chunk starts, the four edges, a
# corner and two interior points; each patch yields the rows within 4 hops.
C3_CENTRES = [(256, 256), (256, 100), (255, 401), (0, 0), (511, 300), (3, 511), (137, 421),
              (128, 16), (384, 200)]


@pytest.fixture(scope="module")
def c3_reference_rows():
    A = W.config_matrix("c3")
    d = _c3_scaling(A)
    N = int(A.meta["shape"][0])
    ref = {}
    for x, y in C3_CENTRES:
        ref.update(cf.local_sign_rows_similar(A, y * N + x, 34, 4, d))
    assert len(ref) >= 256
    return A, ref


@pytest.mark.parametrize("precision,rel_tol", [(1, 1e-8), (0, 1e-10)])
def test_c3_full_against_oracle(sf, c3_golden, precision, rel_tol):
    """C3 (the bench's workload) FP64 and mixed against the FP64 oracle's own full
    solve: the whole matrix through the row probes and entry by entry on the stored
    rows; the FP64 result has the oracle's number of entries."""
    A, g = c3_golden
    res = sf.sign_ns(sf.DeviceCsr.from_host(A),
                     sf.default_opts(tol=1e-12, filter_y=1, precision=precision))
    assert res.status == "OK"
    _check_against_oracle(res, g, rel_tol)
    if precision == 0:
        assert abs(res.stats()["nnz"] - int(g["nnz"])) <= 1e-3 * int(g["nnz"])


@pytest.mark.parametrize("precision,rel_tol", [(1, 1e-8), (0, 1e-10)])
def test_c3_full(sf, c3_reference_rows, precision, rel_tol):
    """2D 512 x 512 upwind convection-diffusion (nonsymmetric), filter_y on,
    mixed precision as configured and plain FP64: every reference row (patch
    signs, at least 256 rows spread over XCD chunks, row groups and the grid's
    edges) within rel_tol, and the sampled-row properties."""
    A, ref = c3_reference_rows
    res = sf.sign_ns(sf.DeviceCsr.from_host(A),
                     sf.default_opts(tol=1e-12, filter_y=1, precision=precision))
    assert res.status == "OK"
    rows = sorted(ref)
    got = res.rows(rows)
    worst = max(_row_error(got[i], *ref[i]) for i in rows)
    assert worst <= rel_tol, worst
    d = _c3_scaling(A)
    _check_sampled(res, A, lambda i: cf.local_sign_row_similar(A, i, 34, d), rel_tol)


@pytest.mark.parametrize("nB", [500, 1000, 3000, 5000])
def test_ode_matrix_paper_sizes(sf, nB):
    """Section 4.2 at the sizes of Table 4.2.1: the whole result against the eq. 1.26
    closed form, and the filtered-vs-unfiltered difference AE within 10x of the
    paper's printed value."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table_4_2_1.txt"))
            if l.strip() and not l.startswith("#")]
    paper_ae = {int(r[0]): float(r[2]) for r in rows}[nB]
    A = W.ode_block_matrix(nB)
    dA = sf.DeviceCsr.from_host(A)
    f = sf.sign_ns(dA, sf.default_opts(tol=1e-12))
    u = sf.sign_ns(dA, sf.default_opts(tol=1e-12, c_fixed=0.0, switch_res=0.0))
    assert f.status == "OK" and u.status == "OK"
    X = f.to_scipy()
    S = cf.sign_ode_block(nB)
    D = X.toarray() - S
    assert np.linalg.norm(D) / np.linalg.norm(S) <= 1e-10
    ae = float(np.sqrt(((X - u.to_scipy()).power(2)).sum()))
    assert ae <= 10 * paper_ae, (ae, paper_ae)


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
