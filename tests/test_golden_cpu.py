"""The stored full-size oracle data and the whole-matrix probe, on the CPU.

* the row probe of tests/golden/probe.py gives the same bits in numpy and in
  torch, and sum_i (p_i(X) - p_i(S))^2 estimates ||X - S||_F^2 (checked on
  random perturbations spread over all rows and on one concentrated in a row);
* the stored C2 oracle solve belongs to the current generator (fingerprint) and
  has the properties the sign of that matrix must have: ||S||_F = sqrt(n) (a
  symmetric involution), trace = the inertia fixed by the staggered gap term,
  the iteration's residual below tol.
"""
import math
import os
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
sys.path.insert(0, GOLDEN)
import probe  # noqa: E402


def test_probe_numpy_and_torch_agree():
    import torch
    rng = np.random.default_rng(0)
    X = sp.random(3000, 3000, density=0.01, random_state=1, format="csr")
    X.data = rng.standard_normal(X.nnz)
    p1 = probe.row_probe_numpy(X.indptr.astype(np.int64), X.indices, X.data)
    p2 = probe.row_probe_torch(torch.as_tensor(X.indptr.astype(np.int64)),
                               torch.as_tensor(X.indices.astype(np.int32)),
                               torch.as_tensor(X.data), chunk=7777).numpy()
    assert np.allclose(p1, p2, rtol=0, atol=1e-12)
    rows = np.repeat(np.arange(3000, dtype=np.int64), np.diff(X.indptr))
    w1 = probe.weights(rows, X.indices.astype(np.int64))
    w2 = probe.weights(torch.as_tensor(rows), torch.as_tensor(X.indices.astype(np.int64)),
                       xp=torch).numpy()
    assert np.array_equal(w1, w2)
    assert abs(w1.mean()) < 0.05          # balanced signs


def test_probe_estimates_frobenius_difference():
    rng = np.random.default_rng(1)
    n = 20000
    S = sp.random(n, n, density=5e-4, random_state=2, format="csr")
    S.data = rng.standard_normal(S.nnz)
    # spread perturbation: new entries and changed values in every row
    D = sp.random(n, n, density=2e-4, random_state=3, format="csr")
    D.data = 1e-9 * rng.standard_normal(D.nnz)
    X = (S + D).tocsr()
    X.sort_indices()
    ps = probe.row_probe_numpy(S.indptr.astype(np.int64), S.indices, S.data)
    px = probe.row_probe_numpy(X.indptr.astype(np.int64), X.indices, X.data)
    est = math.sqrt(float(np.sum((px - ps) ** 2)))
    true = sp.linalg.norm(D)
    assert 0.9 * true <= est <= 1.1 * true
    # one bad entry is seen in full
    X2 = S.copy().tolil()
    X2[17, 5] = X2[17, 5] + 3e-6
    X2 = X2.tocsr()
    px2 = probe.row_probe_numpy(X2.indptr.astype(np.int64), X2.indices, X2.data)
    est2 = math.sqrt(float(np.sum((px2 - ps) ** 2)))
    assert abs(est2 - 3e-6) <= 1e-12


def test_stored_c2_oracle_solve():
    import make_fullsize_golden as mk
    g = np.load(os.path.join(GOLDEN, "c2_fp64_oracle.npz"))
    A = W.config_matrix("c2")
    assert str(g["fingerprint"]) == mk.fingerprint(A)
    assert int(g["iters"]) >= 5 and float(g["res_fro"]) <= 1e-12
    assert abs(float(g["fro"]) - math.sqrt(A.n)) <= 1e-9 * math.sqrt(A.n)
    assert abs(float(g["trace"]) - A.meta["inertia"]) <= 1e-8
    assert len(g["probe"]) == A.n and len(g["rows"]) >= 64
    off = 0
    for i, L in zip(g["rows"], g["row_len"]):
        c = g["row_cols"][off:off + L]
        off += L
        assert np.all(np.diff(c) > 0) and L > 0
    assert off == len(g["row_vals"])


def test_admission_table_covers_the_oracle_fill():
    """The server's admission table (kFill in csrc/serve.hip) covers the peak
    resident entries per row that the oracle's solves of the served families
    reach (tests/golden/serving_fill.txt), within a 1.5x margin."""
    import re
    src = open(os.path.join(os.path.dirname(GOLDEN), "..", "paper_2210_03356_amd", "csrc",
                            "serve.hip")).read()
    body = src[src.index("constexpr FillEntry kFill[] = {"):]
    body = body[:body.index("};")]
    table = [(float(a), int(b), float(c), float(d)) for a, b, c, d in
             re.findall(r"\{([\d.]+), (\d+), ([\d.e+-]+), (\d+)\}", body)]
    assert len(table) >= 6
    rows = [l.split() for l in open(os.path.join(GOLDEN, "serving_fill.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) >= 9
    for fam, n, avg, tol, peak in rows:
        n, avg, tol, peak = int(n), float(avg), float(tol), float(peak)
        per_row = next(p for a, nm, t, p in table
                       if avg <= a and (nm == 0 or n <= nm) and tol >= t)
        assert peak <= per_row <= 1.5 * peak, (fam, n, tol, peak, per_row)


def test_stored_c3_oracle_solve():
    import make_fullsize_golden as mk
    g = np.load(os.path.join(GOLDEN, "c3_fp64_oracle.npz"))
    A = W.config_matrix("c3")
    assert str(g["fingerprint"]) == mk.fingerprint(A)
    assert int(g["iters"]) >= 5 and float(g["res_fro"]) <= 1e-12
    # nonsymmetric: no norm identity, but the trace is the inertia of the gap term
    assert abs(float(g["trace"]) - A.meta["inertia"]) <= 1e-8
    assert len(g["probe"]) == A.n and len(g["rows"]) >= 64
