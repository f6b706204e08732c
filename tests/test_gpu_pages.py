"""Page windows of the row-group product against the FP64 oracle.

A group of rows whose column range spans more than one dense LDS window marks
the 2^shift-column pages its B rows, D rows and diagonal occupy, ranks them, and
sweeps windows over the occupied pages only.  These tests force page windows
(SIGNFN_PAGES=on) on products and whole solves whose ranges are wide enough for
them, check from the product's progress line that they ran, and compare with the
oracle: products entry by entry, solves in relative Frobenius norm.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads as W
from test_gpu_parity import _check_product, _dev, _wide_rows_matrix

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


def _pages_env(monkeypatch, group=None, shift=None):
    monkeypatch.setenv("SIGNFN_PAGES", "on")
    monkeypatch.setenv("SIGNFN_PROGRESS", "1")
    if group is None:
        monkeypatch.delenv("SIGNFN_ROW_GROUP", raising=False)
    else:
        monkeypatch.setenv("SIGNFN_ROW_GROUP", str(group))
    if shift is None:
        monkeypatch.delenv("SIGNFN_PAGE_SHIFT", raising=False)
    else:
        monkeypatch.setenv("SIGNFN_PAGE_SHIFT", str(shift))


@pytest.mark.parametrize("group,shift", [(2, 4), (4, 4), (8, 4), (16, 4), (8, 5), (4, 6), (8, 8)])
def test_page_window_products(sf, monkeypatch, capfd, group, shift):
    """Products of rows that hold every grid point within a diamond (each grid row
    a short run of columns in a range of ~9,000) and of random rows times them
    (ranges spanning the matrix): the product is the oracle's for every group size
    and page size."""
    _pages_env(monkeypatch, group, shift)
    A = _wide_rows_matrix()
    R = W.random_sparse(A.n, mean_row=6, seed=9, powerlaw=False)
    for left in (A, R):
        st = _check_product(sf, left, A).stats()
        assert st["madds"] == st["products"]
    err = capfd.readouterr().err
    assert "(page windows)" in err, err[-2000:]


def _grid_stencil(nx=203, ny=61, seed=23):
    """The 5-point stencil pattern of the same nx x ny grid (x fastest), random
    values: rows of at most five entries, the short B rows of X*A."""
    rng = np.random.default_rng(seed)
    n = nx * ny
    rows = []
    for y in range(ny):
        for x in range(nx):
            c = [y * nx + x]
            if x > 0: c.append(y * nx + x - 1)
            if x < nx - 1: c.append(y * nx + x + 1)
            if y > 0: c.append((y - 1) * nx + x)
            if y < ny - 1: c.append((y + 1) * nx + x)
            rows.append(np.sort(np.array(c, np.int32)))
    indptr = np.zeros(n + 1, np.int64)
    indptr[1:] = np.cumsum([len(c) for c in rows])
    indices = np.concatenate(rows)
    data = rng.uniform(0.1, 1.0, len(indices)) * rng.choice([-1.0, 1.0], len(indices))
    return W.Csr(n=n, indptr=indptr, indices=indices, data=data)


@pytest.mark.parametrize("group", [None, 2, 4, 8, 16])
def test_page_windows_short_b_rows(sf, monkeypatch, capfd, group):
    """Long rows times short ones (X*A with A the stencil: each lane walks its own
    slot's B row of at most five entries) in page windows: the product is the
    oracle's entry by entry, for every group size."""
    _pages_env(monkeypatch, group)
    A = _wide_rows_matrix()
    B = _grid_stencil()
    st = _check_product(sf, A, B).stats()
    assert st["madds"] == st["products"]
    err = capfd.readouterr().err
    assert "(page windows)" in err, err[-2000:]


def _band_and_far_matrix(n=135000, half=8, seed=5):
    """Rows holding a band i-half .. i+half and two columns far away: a product's
    row groups then span nearly all n columns, more than the LDS page table holds
    at 16-column pages (131,072 columns), so those groups use dense windows inside
    the page-window kernel while the narrower ones use pages."""
    rng = np.random.default_rng(seed)
    rows = []
    far = rng.integers(0, n, size=(n, 2))
    for i in range(n):
        c = np.arange(max(0, i - half), min(n, i + half + 1))
        rows.append(np.unique(np.concatenate([c, far[i]])).astype(np.int32))
    indptr = np.zeros(n + 1, np.int64)
    indptr[1:] = np.cumsum([len(c) for c in rows])
    indices = np.concatenate(rows)
    data = rng.uniform(0.1, 1.0, len(indices)) * rng.choice([-1.0, 1.0], len(indices))
    return W.Csr(n=n, indptr=indptr, indices=indices, data=data)


def test_page_windows_wider_than_the_table(sf, monkeypatch, capfd):
    """Groups whose column range holds more pages than the LDS table fall back to
    dense windows in the same kernel; the product is still the oracle's."""
    _pages_env(monkeypatch, 4)
    A = _band_and_far_matrix()
    # column range of product row i: from the first to the last column of the B
    # rows it gathers; on a sample of rows some exceed the table's 131,072 columns
    # (dense windows) and some do not (pages)
    first = A.indices[A.indptr[:-1]]
    last = A.indices[A.indptr[1:] - 1]
    wide = [last[k].max() - first[k].min() + 1 > 131072
            for k in (A.indices[A.indptr[i]:A.indptr[i + 1]] for i in range(0, A.n, 331))]
    assert 0 < sum(wide) < len(wide)
    _check_product(sf, A, A)
    err = capfd.readouterr().err
    assert "(page windows)" in err, err[-2000:]


@pytest.fixture(scope="module")
def pages_cases():
    """A symmetric 2D case (products from lower triangles, fused update, diagonal)
    and a nonsymmetric one with filtered residuals; both grow rows spanning more
    than one dense window."""
    lap = W.laplacian_2d(96, jitter=0.05, seed=2, m=8.0)
    cd = W.convdiff_2d(96, beta=0.5, sigma=4.0, m=8.0)
    return {
        "lap2d_96": (lap, dict(tol=1e-12), oracle.nsf(lap, tol=1e-12).to_scipy()),
        "convdiff_96_filter_y": (cd, dict(tol=1e-12, filter_y=1),
                                 oracle.nsf(cd, tol=1e-12, filter_y=1).to_scipy()),
    }


@pytest.mark.parametrize("group", [None, 4, 8])
@pytest.mark.parametrize("name", ["lap2d_96", "convdiff_96_filter_y"])
def test_page_windows_solve(sf, monkeypatch, capfd, pages_cases, name, group):
    """Whole solves with page windows, FP64 and mixed precision, match the oracle
    (1e-10 and 1e-8 in relative Frobenius norm)."""
    _pages_env(monkeypatch, group)
    A, kw, S = pages_cases[name]
    r = sf.sign_ns(_dev(sf, A), sf.default_opts(**kw))
    assert r.status == "OK"
    assert sp.linalg.norm(r.to_scipy() - S) <= 1e-10 * sp.linalg.norm(S)
    m = sf.sign_ns(_dev(sf, A), sf.default_opts(precision=1, **kw))
    assert m.status == "OK"
    assert sp.linalg.norm(m.to_scipy() - S) <= 1e-8 * sp.linalg.norm(S)
    err = capfd.readouterr().err
    assert "(page windows)" in err, err[-2000:]


@pytest.mark.parametrize("group", [4, 8])
def test_page_windows_in_many_batches(sf, monkeypatch, pages_cases, group):
    """A 1 MB staging budget splits every product into row batches (cursors and
    merged lists per batch, page lists of the whole B): the solve equals the
    one-batch solve and the oracle's."""
    _pages_env(monkeypatch, group)
    A, kw, S = pages_cases["convdiff_96_filter_y"]
    one = sf.sign_ns(_dev(sf, A), sf.default_opts(**kw))
    many = sf.sign_ns(_dev(sf, A), sf.default_opts(staging_bytes=1 << 20, **kw))
    assert one.status == "OK" and many.status == "OK"
    X1, X2 = one.to_scipy(), many.to_scipy()
    assert sp.linalg.norm(X2 - X1) <= 1e-13 * sp.linalg.norm(X1)
    assert sp.linalg.norm(X2 - S) <= 1e-10 * sp.linalg.norm(S)
