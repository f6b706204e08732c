"""The register-accumulator product kernel (k_spgemm_regtile), forced for every
product it supports through SIGNFN_REGTILE, against the FP64 oracle: single
products (wide rows, grid squares with multi-window rows, FP32 values, ragged
groups), whole solves (symmetric and nonsymmetric, filtered residuals, mixed
precision, products split into many row batches)."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads as W
from test_gpu_parity import CASES, _check_product, _dev, _wide_rows_matrix

pytestmark = pytest.mark.gpu

CONFIGS = ["8x4", "8x8", "16x2", "16x4"]


@pytest.fixture(scope="module")
def sf():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    import paper_2210_03356_amd as pkg
    pkg.load()
    oracle.build(force=False)
    return pkg


@pytest.mark.parametrize("cfg", CONFIGS)
def test_regtile_products_match_oracle(sf, monkeypatch, cfg):
    monkeypatch.setenv("SIGNFN_REGTILE", cfg)
    A = _wide_rows_matrix()
    r = _check_product(sf, A, A)
    assert r.stats()["hot_regtile"] == 1
    # rows of a wide grid: column clusters (one per grid row) far apart, so the
    # windows jump over the gaps; compared on the union pattern
    G = W.laplacian_2d(700, jitter=0.05, seed=2, m=8.0)
    X = sp.csr_matrix((G.data, G.indices, G.indptr), shape=(G.n, G.n))
    X3 = (X @ X @ X).tocsr()
    X3.sort_indices()
    B = W.Csr(n=G.n, indptr=X3.indptr.astype(np.int64), indices=X3.indices.astype(np.int32),
              data=X3.data)
    r = _check_product(sf, B, B, exact_pattern=False)
    assert r.stats()["hot_regtile"] == 1


@pytest.mark.parametrize("cfg", ["8x4", "16x4"])
def test_regtile_fp32_products(sf, monkeypatch, cfg):
    monkeypatch.setenv("SIGNFN_REGTILE", cfg)
    A = _wide_rows_matrix()
    A32 = W.Csr(n=A.n, indptr=A.indptr, indices=A.indices,
                data=A.data.astype(np.float32).astype(np.float64))
    r = sf.sign_spgemm(_dev(sf, A32, dtype=np.float32), _dev(sf, A32, dtype=np.float32))
    assert r.status == "OK" and r.stats()["hot_regtile"] == 1
    rp, ci, va = r.to_numpy()
    orp, oci, ova = oracle.spgemm(A32, A32)
    assert np.array_equal(rp, orp) and np.array_equal(ci, oci)
    kmax = int(np.diff(A.indptr).max())
    absA = W.Csr(n=A.n, indptr=A.indptr, indices=A.indices, data=np.abs(A32.data))
    _, _, bound = oracle.spgemm(absA, absA)
    # FP64 sums of exact FP32 x FP32 products, rounded once to FP32
    assert np.all(np.abs(va - ova) <= 2 ** -24 * np.abs(ova) + 1e-15 * kmax * bound)


@pytest.mark.parametrize("cfg", CONFIGS)
def test_regtile_nsf_lap96(sf, monkeypatch, cfg):
    monkeypatch.setenv("SIGNFN_REGTILE", cfg)
    A = W.laplacian_2d(96, jitter=0.05, seed=2, m=8.0)
    S = oracle.nsf(A, tol=1e-12).to_scipy()
    r = sf.sign_ns(_dev(sf, A), sf.default_opts(tol=1e-12))
    assert r.status == "OK" and r.stats()["hot_regtile"] == 1
    X = r.to_scipy()
    assert sp.linalg.norm(X - S) / sp.linalg.norm(S) <= 1e-10
    assert (X - X.T).nnz == 0          # symmetric products, mirrored


@pytest.mark.parametrize("name", ["convdiff_30", "lap2d_32_filter_y", "lap3d_9", "lap2d_48"])
def test_regtile_nsf_cases(sf, monkeypatch, name):
    monkeypatch.setenv("SIGNFN_REGTILE", "16x4")
    make, kw = CASES[name]
    A = make()
    S = oracle.nsf(A, **kw).to_scipy()
    r = sf.sign_ns(_dev(sf, A), sf.default_opts(**kw))
    assert r.status == "OK"
    X = r.to_scipy()
    assert sp.linalg.norm(X - S) / sp.linalg.norm(S) <= 1e-10
    # and many row batches
    m = sf.sign_ns(_dev(sf, A), sf.default_opts(staging_bytes=1 << 20, **kw))
    assert m.status == "OK"
    assert sp.linalg.norm(m.to_scipy() - S) / sp.linalg.norm(S) <= 1e-10


@pytest.mark.parametrize("cfg", ["8x4", "16x4"])
def test_regtile_mixed_precision(sf, monkeypatch, cfg):
    monkeypatch.setenv("SIGNFN_REGTILE", cfg)
    A = W.convdiff_2d(64, beta=0.5, sigma=4.0, m=8.0)
    S = oracle.nsf(A, tol=1e-12, filter_y=1).to_scipy()
    r = sf.sign_ns(_dev(sf, A), sf.default_opts(tol=1e-12, filter_y=1, precision=1))
    assert r.status == "OK"
    X = r.to_scipy()
    assert sp.linalg.norm(X - S) / sp.linalg.norm(S) <= 1e-8


def test_regtile_auto_rule(sf, monkeypatch):
    """With the per-product rule the solve still matches the oracle."""
    monkeypatch.setenv("SIGNFN_REGTILE", "auto")
    A = W.laplacian_2d(96, jitter=0.05, seed=2, m=8.0)
    S = oracle.nsf(A, tol=1e-12).to_scipy()
    r = sf.sign_ns(_dev(sf, A), sf.default_opts(tol=1e-12))
    assert r.status == "OK"
    assert sp.linalg.norm(r.to_scipy() - S) / sp.linalg.norm(S) <= 1e-10
