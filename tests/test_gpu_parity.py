"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
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
    oracle.build(force=False)
    return pkg


def _dev(sf, A, dtype=None):
    return sf.DeviceCsr.from_host(A, dtype=dtype)


def _abs(A):
    return W.Csr(n=A.n, indptr=A.indptr, indices=A.indices, data=np.abs(A.data))


def _check_product(sf, A, B, rtol=4e-15, exact_pattern=True):
    r = sf.sign_spgemm(_dev(sf, A), _dev(sf, B))
    assert r.status == "OK"
    rp, ci, va = r.to_numpy()
    orp, oci, ova = oracle.spgemm(A, B)
    brp, bci, bound = oracle.spgemm(_abs(A), _abs(B))
    kmax = max(1, int(np.diff(A.indptr).max()))
    for i in range(A.n):   # sorted, unique columns in every row
        assert np.all(np.diff(ci[rp[i]:rp[i + 1]]) > 0)
    assert np.all(va != 0.0)
    if exact_pattern:
        # random values: no exact cancellation, so the patterns are identical
        assert np.array_equal(rp, orp)
        assert np.array_equal(ci, oci)
        assert np.all(np.abs(va - ova) <= rtol * kmax * bound + 1e-300)
    else:
        # heavy cancellation: an entry may round to exactly zero (and be
        # dropped) on one side only; compare on the union pattern
        n = A.n
        G = sp.csr_matrix((va, ci, rp), shape=(n, n))
        O = sp.csr_matrix((ova, oci, orp), shape=(n, n))
        Bd = sp.csr_matrix((bound, bci, brp), shape=(n, n))
        D = (G - O).tocsr()
        D.sort_indices()
        lim = Bd.multiply(D != 0).tocsr()   # bound restricted to D's pattern
        lim.sort_indices()
        assert np.array_equal(D.indptr, lim.indptr) and np.array_equal(D.indices, lim.indices)
        assert np.all(np.abs(D.data) <= rtol * kmax * lim.data + 1e-300)
        # entries present on one side only are within the bound of zero
    return r


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_spgemm_random_powerlaw(sf, seed):
    A = W.random_sparse(900, mean_row=7, seed=seed)
    B = W.random_sparse(900, mean_row=11, seed=seed + 100)
    _check_product(sf, A, B)


def test_spgemm_multiwindow_rows(sf):
    # columns spread over 30000: each output row sweeps several LDS windows
    A = W.random_sparse(30000, mean_row=5, seed=4, powerlaw=False)
    B = W.random_sparse(30000, mean_row=9, seed=5, powerlaw=False)
    r = _check_product(sf, A, B)
    assert r.stats()["products"] > 0


def test_spgemm_dense_rows_and_empty_rows(sf):
    rng = np.random.default_rng(3)
    n = 5000
    # a few dense rows (class 3, several windows), many empty rows, a ragged tail
    rows, cols = [], []
    for i in range(n):
        if i % 7 == 0:
            continue
        k = 2500 if i % 997 == 0 else int(rng.integers(1, 20))
        c = rng.choice(n, size=k, replace=False)
        rows.append(np.full(k, i)); cols.append(c)
    r = np.concatenate(rows); c = np.concatenate(cols)
    M = sp.csr_matrix((rng.uniform(0.1, 1, len(r)) * rng.choice([-1, 1], len(r)), (r, c)),
                      shape=(n, n))
    M.sort_indices()
    A = W.Csr(n=n, indptr=M.indptr.astype(np.int64), indices=M.indices.astype(np.int32),
              data=M.data)
    _check_product(sf, A, A)


@pytest.mark.parametrize("n", [2047, 2048, 2049, 8192, 8193])
def test_spgemm_scan_boundaries(sf, n):
    # row counts at the edges of one scan chunk (2048 entries) and of the
    # one-workgroup scan (8192 entries): the product's capacities and row starts
    # come from these scans
    A = W.random_sparse(n, mean_row=4, seed=n)
    B = W.random_sparse(n, mean_row=5, seed=n + 1)
    _check_product(sf, A, B)


@pytest.mark.parametrize("blen", [255, 256, 257, 512, 768])
def test_spgemm_chunk_sized_b_rows(sf, blen):
    # B rows of whole and almost whole 256-entry chunks (one gather step of the
    # product kernel): a chunk that exactly fills the row or the window is followed
    # by an empty or partial refill; A mixes short and long rows, so both the
    # single-row and the row-group kernels read them
    n = 4096
    rng = np.random.default_rng(blen)
    starts = rng.integers(0, n - blen, size=n)
    B = sp.csr_matrix((rng.uniform(0.5, 1.5, n * blen),
                       (np.repeat(np.arange(n), blen),
                        (starts[:, None] + np.arange(blen)[None, :]).ravel())), shape=(n, n))
    B.sort_indices()
    rows, cols = [], []
    for i in range(n):
        k = 60 if i % 5 == 0 else int(rng.integers(1, 6))
        c = np.unique(np.clip(i + rng.integers(-300, 300, size=k), 0, n - 1))
        rows.append(np.full(len(c), i)); cols.append(c)
    r = np.concatenate(rows); c = np.concatenate(cols)
    A = sp.csr_matrix((rng.uniform(0.5, 1.5, len(r)), (r, c)), shape=(n, n))
    A.sort_indices()
    to_csr = lambda M: W.Csr(n=n, indptr=M.indptr.astype(np.int64),
                             indices=M.indices.astype(np.int32), data=M.data)
    _check_product(sf, to_csr(A), to_csr(B))


def test_spgemm_tiny_and_identity(sf):
    one = W.Csr(n=1, indptr=np.array([0, 1], np.int64), indices=np.array([0], np.int32),
                data=np.array([-3.0]))
    r = sf.sign_spgemm(_dev(sf, one), _dev(sf, one))
    rp, ci, va = r.to_numpy()
    assert rp.tolist() == [0, 1] and ci.tolist() == [0] and va.tolist() == [9.0]
    empty = W.Csr(n=5, indptr=np.zeros(6, np.int64), indices=np.zeros(0, np.int32),
                  data=np.zeros(0))
    r = sf.sign_spgemm(_dev(sf, empty), _dev(sf, W.tridiag_c1(5)))
    assert r.to_numpy()[0].tolist() == [0] * 6


def test_spgemm_grid_square(sf):
    # square of a dense-ish iterate of the 2D family (rows of a few thousand)
    A = W.laplacian_2d(40, jitter=0.05, seed=2, m=8.0)
    X = oracle.nsf(A, tol=1e-12)
    Xc = W.Csr(n=A.n, indptr=X.indptr, indices=X.indices, data=X.data)
    _check_product(sf, Xc, Xc, exact_pattern=False)


def test_spgemm_fp32(sf):
    A = W.random_sparse(2000, mean_row=8, seed=7)
    B = W.random_sparse(2000, mean_row=8, seed=8)
    Af = W.Csr(n=A.n, indptr=A.indptr, indices=A.indices, data=A.data.astype(np.float32)
               .astype(np.float64))
    Bf = W.Csr(n=B.n, indptr=B.indptr, indices=B.indices, data=B.data.astype(np.float32)
               .astype(np.float64))
    r = sf.sign_spgemm(_dev(sf, A, np.float32), _dev(sf, B, np.float32))
    rp, ci, va = r.to_numpy()
    assert va.dtype == np.float32
    orp, oci, ova = oracle.spgemm(Af, Bf)
    _, _, bound = oracle.spgemm(_abs(Af), _abs(Bf))
    assert np.array_equal(rp, orp) and np.array_equal(ci, oci)
    assert np.all(np.abs(va - ova) <= 2 ** -23 * 40 * bound)


@pytest.mark.parametrize("seed,n", [(0, 3000), (1, 3000), (2, 3000), (3, 3000),
                                    (4, 8192), (5, 8193), (6, 1)])
def test_filter_matches_oracle_selection(sf, seed, n):
    rng = np.random.default_rng(seed)
    A = W.random_sparse(n, mean_row=20, seed=seed + 50)
    A.data = np.exp(rng.uniform(-80, 1, A.nnz)) * rng.choice([-1, 1], A.nnz)
    A.data[A.data > 1] = 0.75
    tau = float(np.exp(rng.uniform(-60, -5)))
    r, bstar = sf.sign_filter(_dev(sf, A), tau)
    b_ref, keep, dsq = oracle.filter_values(A.data, tau)
    assert bstar == b_ref
    rp, ci, va = r.to_numpy()
    rows = np.repeat(np.arange(A.n), np.diff(A.indptr))
    ref = sp.csr_matrix((A.data[keep], (rows[keep], A.indices[keep])), shape=(A.n, A.n))
    assert np.array_equal(rp, ref.indptr) and np.array_equal(ci, ref.indices)
    assert np.array_equal(va, ref.data)           # dropping is exact
    assert r.stats()["step_fro"] <= tau
    assert abs(r.stats()["step_fro"] ** 2 - dsq) <= 1e-12 * dsq + 1e-300


def _rel(X, S):
    return np.linalg.norm(X - S) / np.linalg.norm(S)


CASES = {
    "c1_64": (lambda: W.tridiag_c1(64), dict(tol=1e-12, stop_rule=1)),
    "c1_1024": (lambda: W.tridiag_c1(1024), dict(tol=1e-12, stop_rule=1)),
    "lap2d_17": (lambda: W.laplacian_2d(17, jitter=0.05, seed=2, m=8.0), dict(tol=1e-12)),
    "lap2d_48": (lambda: W.laplacian_2d(48, jitter=0.05, seed=2, m=8.0), dict(tol=1e-12)),
    "convdiff_30": (lambda: W.convdiff_2d(30, beta=0.5, sigma=4.0, m=8.0), dict(tol=1e-12)),
    "lap3d_9": (lambda: W.laplacian_3d(9, perturb=0.5, seed=4, m=12.0), dict(tol=1e-10)),
    "lap1d_3001": (lambda: W.laplacian_1d(3001, sigma=2.0, jitter=0.05, seed=9, m=4.0),
                   dict(tol=1e-12)),
    "ode_300": (lambda: W.ode_block_matrix(300), dict(tol=1e-12)),
    "lap2d_32_filter_y": (lambda: W.laplacian_2d(32, jitter=0.05, seed=2, m=8.0),
                          dict(tol=1e-12, filter_y=1)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_nsf_matches_oracle(sf, name):
    make, kw = CASES[name]
    A = make()
    r = sf.sign_ns(_dev(sf, A), sf.default_opts(**kw))
    assert r.status == "OK"
    X = r.to_scipy()
    ref = oracle.nsf(A, **kw)
    assert ref.status == "OK"
    S = ref.to_scipy()
    rel = sp.linalg.norm(X - S) / sp.linalg.norm(S)
    assert rel <= 1e-10, rel
    st = r.stats()
    assert st["res_fro"] <= max(kw["tol"], 1e-11) * 10 or kw.get("stop_rule") == 1
    # same iteration count as the oracle, or one apart when a stop test sits on the edge
    assert abs(st["iters"] - ref.iters) <= 1
    if name.startswith("c1"):
        n = A.n
        Sx = cf.sign_tridiag_c1(n)
        assert np.linalg.norm(X.toarray() - Sx) / math.sqrt(n) <= 1e-10
    if name.startswith("ode"):
        assert _rel(X.toarray(), cf.sign_ode_block(300)) <= 1e-10


def test_nsf_fp32_input_values(sf):
    A = W.laplacian_2d(20, jitter=0.05, seed=2, m=8.0)
    A32 = W.Csr(n=A.n, indptr=A.indptr, indices=A.indices,
                data=A.data.astype(np.float32).astype(np.float64))
    r = sf.sign_ns(_dev(sf, A, np.float32), sf.default_opts(tol=1e-12))
    ref = oracle.nsf(A32, tol=1e-12)
    X, S = r.to_scipy(), ref.to_scipy()
    assert sp.linalg.norm(X - S) / sp.linalg.norm(S) <= 1e-10


def test_status_paths(sf):
    A = W.laplacian_2d(8, jitter=0.05, seed=2, m=8.0)
    r = sf.sign_ns(_dev(sf, A), sf.default_opts(max_iter=1))
    assert r.status == "ENOCONV" and r.stats()["iters"] == 1
    ref = oracle.nsf(A, max_iter=1)
    assert _rel(r.to_scipy().toarray(), ref.to_scipy().toarray()) < 1e-13
    r = sf.sign_ns(_dev(sf, A), sf.default_opts(scale=1.0))
    assert r.status == "EDIVERGED"
    one = W.Csr(n=1, indptr=np.array([0, 1], np.int64), indices=np.array([0], np.int32),
                data=np.array([-3.0]))
    r = sf.sign_ns(_dev(sf, one), sf.default_opts())
    assert r.status == "OK" and r.to_numpy()[2].tolist() == [-1.0]
    bad = W.tridiag_c1(6)
    bad.indices = bad.indices.copy()
    assert list(bad.indices[1:3]) == [0, 2]
    bad.indices[1], bad.indices[2] = 2, 0   # row 1 not ascending
    with pytest.raises(sf.SignError, match="ascending"):
        sf.sign_ns(_dev(sf, bad), sf.default_opts())
    nan = W.tridiag_c1(6)
    nan.data = nan.data.copy()
    nan.data[2] = np.nan
    with pytest.raises(sf.SignError, match="non-finite"):
        sf.sign_ns(_dev(sf, nan), sf.default_opts())


def test_trace_records_budget_and_filter(sf):
    A = W.laplacian_2d(30, jitter=0.05, seed=2, m=8.0)
    r = sf.sign_ns(_dev(sf, A), sf.default_opts(tol=1e-12))
    tr = r.trace()
    assert len(tr) == r.stats()["iters"] + 1
    for t in tr[:-1]:
        assert t["ffro"] <= t["tau"]
        assert t["nnz_x"] > 0 and t["nnz_bar"] >= t["nnz_x"]
    ref = oracle.nsf(A, tol=1e-12)
    e_gpu = np.array([t["e"] for t in tr])
    e_ref = ref.trace["e"][: len(tr)]
    # residual histories agree until the rounding floor
    big = e_ref > 1e-10
    assert np.allclose(e_gpu[big], e_ref[big], rtol=1e-9)
    # the GPU's own budgets: c4*tol before the switch, eq. 1.18 of the same step's
    # e_k and ||X^_k||_F after it (Section 3.2, Section 4)
    tau = np.array([t["tau"] for t in tr[:-1]])
    e = e_gpu[:-1]
    x = np.array([t["xfro"] for t in tr[:-1]])
    after = e < 1e-6
    assert after.any() and (~after).any()
    assert np.all(tau[~after] == 1e-16)
    np.testing.assert_allclose(tau[after], 0.75 * e[after] ** 2 / (3 * x[after] + x[after] ** 3),
                               rtol=1e-14)



@pytest.mark.parametrize("name", ["lap2d_48", "convdiff_30", "lap3d_9", "lap2d_32_filter_y"])
def test_certified_last_residual(sf, name):
    """The last residual certified from a thinned copy of the iterate is a true
    bound: the residual of the returned matrix, formed here with scipy in FP64, lies
    below it, and the bound itself is at most tol."""
    make, kw = CASES[name]
    A = make()
    r = sf.sign_ns(_dev(sf, A), sf.default_opts(**kw))
    assert r.status == "OK"
    tr = r.trace()
    assert not any(t["e_bound"] for t in tr[:-1])
    last = tr[-1]
    if name in ("lap2d_48", "convdiff_30"):
        assert last["e_bound"] == 1
    X = r.to_scipy()
    e_full = sp.linalg.norm(sp.identity(A.n, format="csr") - X @ X)
    assert e_full <= last["e"] <= kw["tol"], (e_full, last["e"])
    assert r.stats()["res_fro"] == last["e"]


@pytest.mark.parametrize("group", ["2", "4", "8", "auto"])
@pytest.mark.parametrize("name", ["lap2d_48", "convdiff_30"])
def test_products_in_many_batches(sf, monkeypatch, name, group):
    """A staging budget of 1 MB splits every product into many row batches, whose
    cursors and merged group lists cover only the batch's A entries: the solve
    gives what the one-batch solve gives (forced row groups, pairs, and the
    per-product rule)."""
    if group == "auto":
        monkeypatch.delenv("SIGNFN_ROW_GROUP", raising=False)
    else:
        monkeypatch.setenv("SIGNFN_ROW_GROUP", group)
    make, kw = CASES[name]
    A = make()
    one = sf.sign_ns(_dev(sf, A), sf.default_opts(**kw))
    many = sf.sign_ns(_dev(sf, A), sf.default_opts(staging_bytes=1 << 20, **kw))
    assert one.status == "OK" and many.status == "OK"
    assert many.stats()["iters"] == one.stats()["iters"]
    X1, X2 = one.to_scipy(), many.to_scipy()
    assert sp.linalg.norm(X2 - X1) <= 1e-13 * sp.linalg.norm(X1)
    # the same arithmetic row by row: every product is the oracle's within rounding
    ref = oracle.nsf(A, **kw).to_scipy()
    assert sp.linalg.norm(X2 - ref) <= 1e-10 * sp.linalg.norm(ref)

def _uneven_fill_matrix(n_low=20000, n_high=6000, d=500, seed=31):
    """Rows whose squares fill their reserved output poorly (entries i-d, i, i+d:
    9 products fold into 5 columns) followed by rows that fill it almost fully
    (8 random columns), so a product sized from its first batch's fill ratio
    outgrows its output in a later batch."""
    rng = np.random.default_rng(seed)
    n = n_low + n_high
    rows = []
    for i in range(n):
        if i < n_low:
            c = [j for j in (i - d, i, i + d) if 0 <= j < n]
        else:
            c = sorted(set(rng.integers(0, n, 8).tolist()))
        rows.append(np.array(c, np.int32))
    indptr = np.zeros(n + 1, np.int64)
    indptr[1:] = np.cumsum([len(c) for c in rows])
    data = rng.uniform(0.5, 1.0, int(indptr[-1]))
    return W.Csr(n=n, indptr=indptr, indices=np.concatenate(rows), data=data)


def test_product_output_regrown_across_batches(sf, monkeypatch, capfd):
    """Products split into batches size their output from the first batch's fill
    ratio; a later batch that outgrows it triggers one regrow from the fill ratio
    of all rows done so far, keeping the entries stored: the product equals the
    oracle's, and the regrow branch ran."""
    monkeypatch.setenv("SIGNFN_STAGING_BYTES", str(1 << 20))
    monkeypatch.setenv("SIGNFN_PROGRESS", "1")
    A = _uneven_fill_matrix()
    _check_product(sf, A, A)
    err = capfd.readouterr().err
    assert "regrown from the fill ratio" in err, err[-2000:]


NMF_CASES = {
    "lap2d_10": (lambda: W.laplacian_2d(10, jitter=0.05, seed=2, m=8.0), {}),
    "lap2d_24": (lambda: W.laplacian_2d(24, jitter=0.05, seed=2, m=8.0), {}),
    "convdiff_12": (lambda: W.convdiff_2d(12, beta=0.5, sigma=4.0, m=8.0), {}),
    "ode_100": (lambda: W.ode_block_matrix(100), {}),
}


@pytest.mark.parametrize("name", list(NMF_CASES))
def test_newton_matches_oracle(sf, name):
    make, kw = NMF_CASES[name]
    A = make()
    r = sf.sign_newton(_dev(sf, A), sf.default_opts(tol=1e-12, **kw))
    assert r.status == "OK"
    ref = oracle.nmf(A, tol=1e-12)
    assert ref.status == "OK"
    X, S = r.to_scipy(), ref.to_scipy()
    assert sp.linalg.norm(X - S) / sp.linalg.norm(S) <= 1e-10
    st = r.stats()
    assert st["inner_steps"] > 0
    assert abs(st["iters"] - ref.iters) <= 1
    if name.startswith("ode"):
        assert _rel(X.toarray(), cf.sign_ode_block(100)) <= 1e-10


def test_newton_agrees_with_ns_on_gpu(sf):
    A = W.laplacian_2d(30, jitter=0.05, seed=2, m=8.0)
    a = sf.sign_ns(_dev(sf, A), sf.default_opts(tol=1e-12)).to_scipy()
    b = sf.sign_newton(_dev(sf, A), sf.default_opts(tol=1e-12)).to_scipy()
    assert sp.linalg.norm(a - b) / sp.linalg.norm(a) <= 1e-10


MIXED_CASES = {
    "convdiff_40": (lambda: W.convdiff_2d(40, beta=0.5, sigma=4.0, m=8.0),
                    dict(tol=1e-12, filter_y=1)),
    "lap3d_10": (lambda: W.laplacian_3d(10, perturb=0.5, seed=4, m=12.0),
                 dict(tol=1e-10, filter_y=1)),
    "lap2d_48": (lambda: W.laplacian_2d(48, jitter=0.05, seed=2, m=8.0), dict(tol=1e-12)),
}


@pytest.mark.parametrize("name", list(MIXED_CASES))
def test_mixed_precision_matches_fp64_oracle(sf, name):
    """FP32 bulk + FP64 polish and commutator refinement reaches 1e-8 of the FP64 oracle."""
    make, kw = MIXED_CASES[name]
    A = make()
    r = sf.sign_ns(_dev(sf, A), sf.default_opts(precision=1, **kw))
    assert r.status == "OK"
    ref = oracle.nsf(A, tol=1e-12, filter_y=kw.get("filter_y", 0))
    X, S = r.to_scipy(), ref.to_scipy()
    rel = sp.linalg.norm(X - S) / sp.linalg.norm(S)
    assert rel <= 1e-8, rel
    tr = r.trace()
    assert any(t["fp32"] for t in tr) and not tr[-1]["fp32"]
    st = r.stats()
    assert st["res_fro"] <= 10 * kw["tol"]
    assert st["comm_rel"] > 0.0
    # the refinement is what removes the error part that Newton-Schulz keeps
    r0 = sf.sign_ns(_dev(sf, A), sf.default_opts(precision=1, refine_steps=0, **kw))
    rel0 = sp.linalg.norm(r0.to_scipy() - S) / sp.linalg.norm(S)
    assert rel <= rel0


def _wide_rows_matrix(nx=203, ny=61, radius=11, seed=21):
    """Rows of a 2D grid (x fastest) holding every point within Manhattan distance
    `radius`: interior rows span 2*radius*nx + 1 > 4096 columns (the wide class),
    rows near the top and bottom edges span fewer, so aligned row groups mix wide
    and narrower rows; n = nx*ny is odd."""
    rng = np.random.default_rng(seed)
    n = nx * ny
    rows = []
    for y in range(ny):
        for x in range(nx):
            parts = []
            for dy in range(-radius, radius + 1):
                yy = y + dy
                if 0 <= yy < ny:
                    r = radius - abs(dy)
                    parts.append(yy * nx + np.arange(max(0, x - r), min(nx - 1, x + r) + 1))
            rows.append(np.concatenate(parts))
    indptr = np.zeros(n + 1, np.int64)
    indptr[1:] = np.cumsum([len(c) for c in rows])
    indices = np.concatenate(rows).astype(np.int32)
    data = rng.uniform(0.1, 1.0, len(indices)) * rng.choice([-1.0, 1.0], len(indices))
    return W.Csr(n=n, indptr=indptr, indices=indices, data=data)


GROUPS = [1, 2, 4, 8, 16]


@pytest.mark.parametrize("group", GROUPS)
def test_row_groups_match_oracle(sf, monkeypatch, group):
    """Wide rows computed in groups (one gather of a B row feeding the
    accumulators of up to 16 consecutive output rows) give the oracle's product,
    including groups that mix wide and narrower rows and a ragged last group."""
    monkeypatch.setenv("SIGNFN_ROW_GROUP", str(group))
    A = _wide_rows_matrix()
    R = W.random_sparse(A.n, mean_row=6, seed=9, powerlaw=False)
    # (A, R): B rows short (lane-per-slot accumulation); (R, A): a handful of
    # slots per row, spread over the waves one or a few each
    for left, right in ((A, A), (A, R), (R, A)):
        r = _check_product(sf, left, right)
        st = r.stats()
        assert st["products"] > 0
        # the kernels' own count of performed multiply-adds: every product the
        # plan counts, once
        assert st["madds"] == st["products"]


@pytest.fixture(scope="module")
def lap96_oracle():
    """2D case whose iterates have wide rows (spans above 4096 columns)."""
    A = W.laplacian_2d(96, jitter=0.05, seed=2, m=8.0)
    return A, oracle.nsf(A, tol=1e-12)


@pytest.mark.parametrize("group", GROUPS)
def test_row_groups_nsf(sf, monkeypatch, lap96_oracle, group):
    """The whole iteration with each row-group setting matches the oracle."""
    monkeypatch.setenv("SIGNFN_ROW_GROUP", str(group))
    A, X = lap96_oracle
    r = sf.sign_ns(_dev(sf, A), sf.default_opts(tol=1e-12))
    st = r.stats()
    assert st["hot_group"] in (1, group)
    S = X.to_scipy()
    assert sp.linalg.norm(r.to_scipy() - S) / sp.linalg.norm(S) <= 1e-10


@pytest.mark.parametrize("name", ["c1_1024", "lap2d_48", "lap3d_9"])
def test_symmetric_products_match_general(sf, monkeypatch, name):
    """For a symmetric input the products are formed from their lower triangle
    and mirrored: the result is exactly symmetric and agrees with the general
    path and the oracle."""
    make, kw = CASES[name]
    A = make()
    monkeypatch.setenv("SIGNFN_SYMMETRIC", "1")
    rs = sf.sign_ns(_dev(sf, A), sf.default_opts(**kw))
    Xs = rs.to_scipy()
    assert (Xs - Xs.T).nnz == 0                      # exactly symmetric
    monkeypatch.setenv("SIGNFN_SYMMETRIC", "0")
    rg = sf.sign_ns(_dev(sf, A), sf.default_opts(**kw))
    Xg = rg.to_scipy()
    # rows of a lower-triangle product stop at the diagonal: fewer multiply-adds
    # performed than the plan counts; the general products perform them all
    assert rs.stats()["madds"] < rs.stats()["products"]
    assert rg.stats()["madds"] == rg.stats()["products"]
    S = oracle.nsf(A, **kw).to_scipy()
    assert sp.linalg.norm(Xs - Xg) <= 1e-10 * sp.linalg.norm(S)
    assert sp.linalg.norm(Xs - S) <= 1e-10 * sp.linalg.norm(S)
    # mixed precision takes the same route in its FP32 phase
    monkeypatch.setenv("SIGNFN_SYMMETRIC", "1")
    Xm = sf.sign_ns(_dev(sf, A), sf.default_opts(precision=1, **kw)).to_scipy()
    assert sp.linalg.norm(Xm - S) <= 1e-8 * sp.linalg.norm(S)


TWO_PASS_CASES = {
    "lap2d_32_filter_y": (lambda: W.laplacian_2d(32, jitter=0.05, seed=2, m=8.0),
                          dict(tol=1e-12, filter_y=1)),
    "convdiff_30_filter_y": (lambda: W.convdiff_2d(30, beta=0.5, sigma=4.0, m=8.0),
                             dict(tol=1e-12, filter_y=1)),
    "lap3d_9_filter_y": (lambda: W.laplacian_3d(9, perturb=0.5, seed=4, m=12.0),
                         dict(tol=1e-10, filter_y=1)),
}


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", list(TWO_PASS_CASES))
def test_two_pass_residual(sf, monkeypatch, capfd, name, precision):
    """Steps formed in two passes, as under memory pressure -- for the residual and
    for the update, a first pass forms the norm and the filter's histogram and
    stores nothing, a second stores only the entries from one bucket below the cut
    -- give the one-pass solve's residual history and result, and the oracle's
    (1e-10 in FP64, 1e-8 mixed)."""
    make, kw = TWO_PASS_CASES[name]
    A = make()
    monkeypatch.delenv("SIGNFN_RESIDUAL_TWO_PASS", raising=False)
    one = sf.sign_ns(_dev(sf, A), sf.default_opts(precision=precision, **kw))
    monkeypatch.setenv("SIGNFN_RESIDUAL_TWO_PASS", "1")
    monkeypatch.setenv("SIGNFN_PROGRESS", "1")
    two = sf.sign_ns(_dev(sf, A), sf.default_opts(precision=precision, **kw))
    err = capfd.readouterr().err
    assert "residual in two passes" in err, err[-2000:]
    assert one.status == "OK" and two.status == "OK"
    X1, X2 = one.to_scipy(), two.to_scipy()
    if precision == 0:
        t1, t2 = one.trace(), two.trace()
        assert len(t1) == len(t2)
        # the first residual is the same matrix in both: the first pass gives its
        # exact entry count and norm
        assert t1[0]["nnz_r"] == t2[0]["nnz_r"]
        assert abs(t1[0]["e"] - t2[0]["e"]) <= 1e-12 * t1[0]["e"]
        # later iterates differ by what the extra bucket kept, far below the
        # iteration's own residuals
        for a, b in zip(t1[1:], t2[1:]):
            if not a["e_bound"]:
                assert abs(a["nnz_r"] - b["nnz_r"]) <= 1e-2 * a["nnz_r"]
            assert abs(a["e"] - b["e"]) <= 1e-3 * a["e"] + 1e-14
        assert sp.linalg.norm(X2 - X1) <= 1e-11 * sp.linalg.norm(X1)
    # (the mixed mode's FP32 steps round their LDS sums apart from run to run, so
    # two mixed runs agree only to the mode's accuracy)
    tol = 1e-10 if precision == 0 else 1e-8
    S = oracle.nsf(A, **kw).to_scipy()
    assert sp.linalg.norm(X2 - S) <= tol * sp.linalg.norm(S)


class _CappedHooks:
    """Device allocation hooks for sign_opts (hipMalloc/hipFree) that refuse any
    allocation taking the bytes in use past `cap`: a device smaller than it is."""

    def __init__(self, sf, cap):
        import ctypes as C
        from paper_2210_03356_amd import signfn as S
        hip = C.CDLL("libamdhip64.so")
        self.cap, self.used, self.peak, self.refused, self._size = cap, 0, 0, 0, {}

        def alloc(nbytes, stream, ctx):
            if self.used + nbytes > self.cap:
                self.refused += 1
                return None
            p = C.c_void_p()
            if hip.hipMalloc(C.byref(p), C.c_size_t(nbytes)) != 0:
                return None
            self.used += nbytes
            self.peak = max(self.peak, self.used)
            self._size[p.value] = nbytes
            return p.value

        def free(ptr, stream, ctx):
            if ptr:
                hip.hipFree(C.c_void_p(ptr))
                self.used -= self._size.pop(ptr)

        self.alloc, self.free = S._ALLOC(alloc), S._FREE(free)


@pytest.mark.parametrize("cap_mb", [300, 380, 440])
def test_two_pass_after_running_out_of_memory(sf, monkeypatch, capfd, cap_mb):
    """Under a device-memory cap (the caller's allocator refuses beyond it) the
    one-pass steps of a filtered-residual solve run out (its peak is ~480 MB) in the
    residual's product, its filter or the update, depending on the cap; that step
    is redone and the rest run in two passes (peak ~265 MB) -- or, near the top,
    only the certification of the last residual from a thinned copy runs out and
    the residual is formed in full -- and the result is the oracle's.  Below the
    two-pass peak the call fails with ENOMEM, a host-side error."""
    A = W.convdiff_2d(64, beta=0.5, sigma=4.0, m=8.0)
    kw = dict(tol=1e-12, filter_y=1)
    monkeypatch.delenv("SIGNFN_RESIDUAL_TWO_PASS", raising=False)
    monkeypatch.setenv("SIGNFN_PROGRESS", "1")
    h = _CappedHooks(sf, cap_mb << 20)
    r = sf.sign_ns(_dev(sf, A), sf.default_opts(staging_bytes=1 << 20, alloc=h.alloc,
                                                free=h.free, **kw))
    err = capfd.readouterr().err
    assert r.status == "OK"
    assert h.refused > 0 and h.peak <= h.cap
    # (at the larger cap only the last residual's certification runs out: it is
    # formed in full instead)
    assert "out of device memory" in err, err[-2000:]
    if cap_mb < 440:
        assert "two passes" in err, err[-2000:]
    S = oracle.nsf(A, **kw).to_scipy()
    X = r.to_scipy()
    del r
    assert sp.linalg.norm(X - S) <= 1e-10 * sp.linalg.norm(S)
    if cap_mb != 380:
        return
    small = _CappedHooks(sf, 150 << 20)
    with pytest.raises(sf.SignError, match="ENOMEM"):
        sf.sign_ns(_dev(sf, A), sf.default_opts(staging_bytes=1 << 20, alloc=small.alloc,
                                                free=small.free, **kw))
    assert small.used == 0  # every block handed back
