"""Host-side checks of the input generators and the benchmark's entry contract."""
import math
import os
import subprocess
import sys

import numpy as np

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _check_csr(A):
    assert A.indptr.dtype == np.int64 and A.indices.dtype == np.int32
    assert A.indptr[0] == 0 and A.indptr[-1] == A.nnz == len(A.indices) == len(A.data)
    assert np.all(np.diff(A.indptr) >= 0)
    for i in range(0, A.n, max(1, A.n // 97)):
        row = A.indices[A.indptr[i]:A.indptr[i + 1]]
        assert np.all(np.diff(row) > 0)
    assert np.all(A.data != 0.0)


def test_config_shapes():
    c1 = W.config_matrix("c1")
    assert c1.n == 1024 and c1.nnz == 2046
    c2 = W.config_matrix("c2")
    assert c2.n == 65536 and c2.nnz == 5 * 65536 - 4 * 256
    _check_csr(c2)
    assert c2.meta["inertia"] == 0
    c3 = W.config_matrix("c3", N=64)
    assert c3.n == 4096 and not c3.meta["symmetric"]
    c4 = W.config_matrix("c4", N=8)
    assert c4.n == 512 and c4.nnz == 7 * 512 - 6 * 64
    _check_csr(c4)


def test_gapped_diagonal_recipe():
    """Diagonal of the 2D config: 4 - (4 + u) + 8 chi, u ~ U[-0.05, 0.05] (seed 2)."""
    N = 16
    A = W.laplacian_2d(N, sigma=4.0, jitter=0.05, seed=2, m=8.0).to_dense()
    u = np.random.default_rng(2).uniform(-0.05, 0.05, size=N * N)
    x, y = np.meshgrid(np.arange(N), np.arange(N))
    chi = np.where((x + y).ravel() % 2 == 0, 1.0, -1.0)
    assert np.allclose(np.diag(A), -u + 8.0 * chi, rtol=0, atol=1e-15)
    off = A - np.diag(np.diag(A))
    assert set(np.unique(off)) <= {0.0, -1.0}
    # upwind convection: west neighbour -(1 + beta h), east -1
    C = W.convdiff_2d(5, beta=0.5, sigma=4.0, m=0.0).to_dense()
    b = 0.5 / 6
    assert abs(C[1, 0] + (1 + b)) < 1e-15 and C[0, 1] == -1.0


def test_literal_configs_have_no_gap():
    """m = 0 keeps the literal (gapless) matrices: eigenvalues reach near zero."""
    A = W.config_matrix("c2", N=24, literal=True).to_dense()
    ev = np.linalg.eigvalsh(A)
    assert np.min(np.abs(ev)) < 0.02
    G = W.config_matrix("c2", N=24).to_dense()
    assert np.min(np.abs(np.linalg.eigvalsh(G))) > 7.9


def test_served_stream_recipe():
    reqs = W.served_stream(count=400, rate=50.0, seed=5)
    t = np.array([r["arrival"] for r in reqs])
    assert np.all(np.diff(t) > 0)
    assert abs(np.mean(np.diff(t)) - 0.02) < 0.004          # Poisson, 50 per second
    ns = np.array([r["n"] for r in reqs])
    assert ns.min() >= 900 and ns.max() <= 66000
    assert {r["tol"] for r in reqs} == {1e-6, 1e-10}
    assert {r["family"] for r in reqs} == {"lap1d", "lap2d", "convdiff2d"}
    for r in reqs[:12]:
        A = W.request_matrix(r)
        _check_csr(A)
        if r["family"] != "lap1d":
            assert math.isqrt(A.n) ** 2 == A.n


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "8"],
                       capture_output=True, text=True)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
