"""Pins of the FP64 oracle against things other than itself.

Each check ties a part of the oracle to a closed form, a library routine
applied to the plain definition, an exact identity of the paper, or brute
force, so that a plausible slip in the oracle (a dropped term, a sign, an
index, a transposed operand, an off-by-one bucket) fails at least one test.
"""
import math
import struct

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import closed_forms as cf


def _rel(X, S):
    return np.linalg.norm(X - S) / np.linalg.norm(S)


def _dense(r):
    return r.to_scipy().toarray()


# ---------------------------------------------------------------------------
# closed forms themselves, against library eigen/Schur routines
# ---------------------------------------------------------------------------
def test_sine_closed_form_matches_eigh():
    n = 256
    A = W.tridiag_c1(n).to_dense()
    S = cf.sign_tridiag_c1(n)
    assert _rel(S, cf.dense_sign_sym(A)) < 1e-13
    # Frobenius norm of an orthogonal involution of order n is sqrt(n)
    assert abs(np.linalg.norm(S) - math.sqrt(n)) < 1e-12


def test_ode_closed_form_matches_schur():
    nB = 48
    A = W.ode_block_matrix(nB).to_dense()
    S = cf.sign_ode_block(nB)
    assert _rel(S, cf.dense_sign_schur(A)) < 1e-12
    half, mhalf = cf.ode_sqrt_blocks(nB)
    B = A[:nB, nB:]
    assert np.abs(half @ half - B).max() < 1e-14
    assert np.abs(half @ mhalf - np.eye(nB)).max() < 1e-14


def test_schur_sign_matches_eigh_on_symmetric():
    A = W.laplacian_2d(6, jitter=0.05, seed=3, m=8.0).to_dense()
    assert _rel(cf.dense_sign_schur(A), cf.dense_sign_sym(A)) < 1e-13


# ---------------------------------------------------------------------------
# end-to-end NSF against exact signs
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [64, 1024])
def test_nsf_c1_matches_sine_closed_form(oracle_lib, n):
    A = W.tridiag_c1(n)
    r = oracle_lib.nsf(A, tol=1e-12, stop_rule=1)
    assert r.status == "OK"
    X = _dense(r)
    S = cf.sign_tridiag_c1(n)
    assert np.linalg.norm(X - S) / math.sqrt(n) < 1e-12
    # chiral structure: sign(tridiag(-1,0,-1)) has no entry with i+k even,
    # and the iteration never creates one
    rows = np.repeat(np.arange(n), np.diff(r.indptr))
    assert np.all((rows + r.indices) % 2 == 1)
    if n == 1024:
        assert r.nnz == n * n // 2


def test_nsf_ode_matrix_matches_eq_1_26(oracle_lib):
    nB = 500
    A = W.ode_block_matrix(nB)
    r = oracle_lib.nsf(A, tol=1e-12)
    assert r.status == "OK"
    # ||A||_inf = 1 here, so the scaled start is the paper's X_1 = A
    assert r.scale == 1.0
    S = cf.sign_ode_block(nB)
    assert _rel(_dense(r), S) < 1e-12


def test_nsf_vs_ns_difference_matches_table_4_2_1(oracle_lib):
    """AE = ||X_NS - X_NSF|| stays at the order the paper prints (Table 4.2.1)."""
    rows = [l.split() for l in open(__file__.replace("test_oracle_pins.py",
                                                     "golden/table_4_2_1.txt"))
            if l.strip() and not l.startswith("#")]
    paper = {int(r[0]): float(r[2]) for r in rows}
    nB = 500
    A = W.ode_block_matrix(nB)
    f = oracle_lib.nsf(A, tol=1e-12)
    u = oracle_lib.nsf(A, tol=1e-12, c_fixed=0.0, switch_res=0.0)   # tau = 0: plain NS
    assert u.trace["ffro"][: u.iters].max() == 0.0
    ae = np.linalg.norm(_dense(f) - _dense(u))
    assert ae <= 10 * paper[nB], (ae, paper[nB])


@pytest.mark.parametrize("make", [
    lambda: W.laplacian_1d(160, sigma=2.0, jitter=0.05, seed=1, m=4.0),
    lambda: W.laplacian_2d(12, jitter=0.05, seed=2, m=8.0),
    lambda: W.convdiff_2d(12, beta=0.5, sigma=4.0, m=8.0),
    lambda: W.convdiff_2d(10, beta=0.5, sigma=4.0, m=8.0, scale_by_h=False),
    lambda: W.laplacian_3d(5, perturb=0.5, seed=4, m=12.0),
], ids=["lap1d", "lap2d", "convdiff", "convdiff_unscaled_beta", "lap3d"])
def test_nsf_matches_dense_definition(oracle_lib, make):
    A = make()
    r = oracle_lib.nsf(A, tol=1e-12)
    assert r.status == "OK"
    S = cf.dense_sign(A.to_dense())
    assert _rel(_dense(r), S) < 1e-11
    # trace(S) = n+ - n- equals the staggering sum for the gapped families
    assert round(np.trace(S)) == A.meta["inertia"]
    assert abs(_dense(r).trace() - A.meta["inertia"]) < 1e-9


def test_nsf_invariants_at_moderate_size(oracle_lib):
    A = W.laplacian_2d(40, jitter=0.05, seed=2, m=8.0)
    r = oracle_lib.nsf(A, tol=1e-12)
    assert r.status == "OK"
    S = r.to_scipy()
    As = A.to_scipy()
    n = A.n
    I = sp.identity(n, format="csr")
    assert sp.linalg.norm(S @ S - I) < 1e-10
    comm = sp.linalg.norm(S @ As - As @ S) / (sp.linalg.norm(S) * sp.linalg.norm(As))
    assert comm < 1e-13
    assert sp.linalg.norm(S - S.T) < 1e-12
    assert abs(S.diagonal().sum() - A.meta["inertia"]) < 1e-8
    assert abs(sp.linalg.norm(S) - math.sqrt(n)) < 1e-8


# ---------------------------------------------------------------------------
# Lemma 2.1.1 (eq. 1.3): one unfiltered NS step maps R to 3/4 R^2 + 1/4 R^3
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("sym", [True, False])
def test_ns_step_residual_recurrence(oracle_lib, sym):
    if sym:
        A = W.laplacian_2d(9, jitter=0.05, seed=7, m=8.0)
    else:
        A = W.convdiff_2d(9, beta=0.5, sigma=4.0, m=8.0, scale_by_h=False)
    X0 = A.to_scipy() / oracle_lib.norm_inf(A)
    X0 = sp.csr_matrix(X0)
    Xc = W.Csr(n=A.n, indptr=X0.indptr.astype(np.int64), indices=X0.indices.astype(np.int32),
               data=X0.data)
    rp, ci, v = oracle_lib.ns_step(Xc)
    X1 = sp.csr_matrix((v, ci, rp), shape=(A.n, A.n)).toarray()
    D0 = X0.toarray()
    I = np.eye(A.n)
    R0 = I - D0 @ D0
    R1 = I - X1 @ X1
    pred = 0.75 * R0 @ R0 + 0.25 * R0 @ R0 @ R0
    assert np.linalg.norm(R1 - pred) <= 1e-14 * max(1.0, np.linalg.norm(R0))
    # the step itself against the dense formula 1/2 X (3I - X^2)
    assert np.abs(X1 - 0.5 * D0 @ (3 * I - D0 @ D0)).max() < 1e-15


# ---------------------------------------------------------------------------
# products
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [0, 1])
def test_spgemm_matches_dense_product(oracle_lib, seed):
    A = W.random_sparse(300, mean_row=6, seed=seed)
    B = W.random_sparse(300, mean_row=9, seed=seed + 10)
    rp, ci, v = oracle_lib.spgemm(A, B)
    C = sp.csr_matrix((v, ci, rp), shape=(300, 300))
    ref = A.to_dense() @ B.to_dense()
    assert np.abs(C.toarray() - ref).max() <= 1e-14 * max(1.0, np.abs(ref).max())
    # sorted, unique columns; no stored zeros
    for i in range(300):
        row = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0)
    assert np.all(v != 0.0)
    # pattern = nonzeros of the exact product (values are random, no cancellation)
    assert C.nnz == np.count_nonzero(ref)


def test_spgemm_non_commuting_operands(oracle_lib):
    """A*B and B*A differ for these operands; catches a swapped operand order."""
    A = W.convdiff_2d(6, beta=0.5, sigma=4.0, m=1.0, scale_by_h=False)
    B = W.random_sparse(36, mean_row=5, seed=3)
    rp, ci, v = oracle_lib.spgemm(A, B)
    C = sp.csr_matrix((v, ci, rp), shape=(36, 36)).toarray()
    assert np.abs(C - A.to_dense() @ B.to_dense()).max() < 1e-14
    assert np.abs(C - B.to_dense() @ A.to_dense()).max() > 1e-3


# ---------------------------------------------------------------------------
# element threshold from a norm budget
# ---------------------------------------------------------------------------
def _bucket_bits(x: float) -> int:
    """Bucket from the IEEE-754 bit pattern (independent of frexp)."""
    bits = struct.unpack("<Q", struct.pack("<d", abs(x)))[0]
    if abs(x) >= 1.0:
        return 2033
    ebits = (bits >> 52) & 0x7FF
    E = ebits - 1023
    if x == 0.0 or ebits == 0 or E < -127:
        return 0
    j = (bits >> 48) & 0xF
    return 1 + 16 * (E + 127) + j


def test_bucket_matches_bit_pattern(oracle_lib):
    rng = np.random.default_rng(0)
    xs = np.concatenate([
        rng.uniform(-1, 1, 2000),
        np.exp(rng.uniform(-300, 0, 4000)) * rng.choice([-1, 1], 4000),
        [0.0, 1.0, -1.0, 2.0, 0.5, 2.0 ** -127, 2.0 ** -128, 2.0 ** -127 * 1.99, 1 - 2 ** -53,
         5e-324, 1e-310],
    ])
    for x in xs:
        assert oracle_lib.bucket(float(x)) == _bucket_bits(float(x)), x


def test_bucket_edges(oracle_lib):
    for b in range(1, 2033):
        lo, hi = oracle_lib.bucket_lo(b), oracle_lib.bucket_hi(b)
        assert lo < hi
        assert oracle_lib.bucket(lo) == b
        assert oracle_lib.bucket(np.nextafter(hi, 0)) == b
        assert oracle_lib.bucket(hi) == b + 1 if b + 1 < 2033 else True
        assert hi / lo <= 17.0 / 16.0 + 1e-15
    assert oracle_lib.bucket(2.0 ** -127) == 1
    assert oracle_lib.bucket(np.nextafter(2.0 ** -127, 0)) == 0
    # scaling by 2 moves a value by exactly 16 buckets
    for x in [3e-5, 0.3, 1.7e-20]:
        assert oracle_lib.bucket(2 * x) == oracle_lib.bucket(x) + 16


def _brute_cut(vals, tau):
    counts = np.zeros(2048, np.int64)
    for x in vals:
        counts[_bucket_bits(x)] += 1
    hi = [2.0 ** -127] + [(1 + ((b - 1) % 16 + 1) / 16) * 2.0 ** ((b - 1) // 16 - 127)
                          for b in range(1, 2033)]
    best = 0
    for c in range(0, 2034):
        bound = sum(counts[b] * hi[b] ** 2 for b in range(c) if counts[b])
        if bound <= tau * tau:
            best = c
    return best


@pytest.mark.parametrize("seed", range(6))
def test_select_matches_brute_force(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(1, 60))
    vals = np.exp(rng.uniform(-60, 1, m)) * rng.choice([-1, 1], m)
    vals[vals > 1] = 0.9
    tau = float(np.exp(rng.uniform(-60, 0)))
    b, keep, dsq = oracle_lib.filter_values(vals, tau)
    assert b == _brute_cut(vals, tau)
    # rigorous budget: the dropped entries have Frobenius norm <= tau
    assert math.sqrt(dsq) <= tau
    assert dsq == pytest.approx(float(np.sum(vals[~keep] ** 2)), rel=1e-15, abs=0)
    # ties go to keep: an entry exactly at the lower edge of the cut bucket stays
    if 0 < b < 2033:
        lo = oracle_lib.bucket_lo(b)
        b2, keep2, _ = oracle_lib.filter_values(np.append(vals, lo), tau)
        if b2 == b:
            assert keep2[-1]


def test_select_zero_budget_drops_nothing(oracle_lib):
    vals = np.array([1e-300, 1e-30, 0.5, 2.0 ** -130])
    b, keep, dsq = oracle_lib.filter_values(vals, 0.0)
    assert keep.all() and dsq == 0.0


def test_select_never_drops_entries_at_or_above_one(oracle_lib):
    vals = np.array([1.0, 3.0, 1e-3])
    b, keep, _ = oracle_lib.filter_values(vals, 1e6)
    assert b == 2033
    assert keep.tolist() == [True, True, False]


# ---------------------------------------------------------------------------
# filtering theory: Theorem 3.2.1 and the budget bookkeeping
# ---------------------------------------------------------------------------
def test_filter_budget_respected_every_step(oracle_lib):
    A = W.laplacian_2d(30, jitter=0.05, seed=2, m=8.0)
    r = oracle_lib.nsf(A, tol=1e-12)
    k = r.iters
    assert np.all(r.trace["ffro"][:k] <= r.trace["tau"][:k])
    # before the switch the budget is the fixed c4*tol, after it eq. 1.18
    e = r.trace["e"][:k]
    assert np.all(r.trace["tau"][:k][e >= 1e-6] == 1e-4 * 1e-12)
    after = e < 1e-6
    assert np.any(after)
    assert np.all(r.trace["tau"][:k][after] < 1e-16)


# Budgets worked out by hand from eq. 1.18, ||F|| <= (3/4) e^2 / (3x + x^3), and
# eq. 1.13, ||F|| <= e^2 / (x + z), at points where the arithmetic is short:
#   e = 4e-7, x = 1:  (3/4)(1.6e-13) / (3 + 1)      = 3e-14
#   e = 6e-7, x = 3:  (3/4)(3.6e-13) / (9 + 27)     = 7.5e-15
#   e = 2e-7, x = 2:  (3/4)(4e-14)   / (6 + 8)      = 3e-14 / 14
#   e = 1e-7, x = 30: (3/4)(1e-14)   / (90 + 27000) = 7.5e-15 / 27090
#   e = 1e-7, x = 2, z = 3: 1e-14 / 5 = 2e-15
#   e = 3e-7, x = 1, z = 8: 9e-14 / 9 = 1e-14
# Each slip fails at least one row: without the 3/4 row 1 gives 4e-14; x^2 for
# x^3 gives 7.5e-15 * 2 in row 2; e for e^2 is off by 1e7; 3x -> x gives 6e-14 in
# row 1; x*z for x+z gives 1e-14/6 and 9e-14/8.
EQ_1_18_POINTS = [(4e-7, 1.0, 3e-14), (6e-7, 3.0, 7.5e-15), (2e-7, 2.0, 3e-14 / 14),
                  (1e-7, 30.0, 7.5e-15 / 27090)]
EQ_1_13_POINTS = [(1e-7, 2.0, 3.0, 2e-15), (3e-7, 1.0, 8.0, 1e-14)]


@pytest.mark.parametrize("e,x,want", EQ_1_18_POINTS)
def test_nsf_budget_hand_values_eq_1_18(oracle_lib, e, x, want):
    assert oracle_lib.nsf_budget(e, x, 1e-12) == pytest.approx(want, rel=1e-14)


@pytest.mark.parametrize("e,x,z,want", EQ_1_13_POINTS)
def test_nmf_budget_hand_values_eq_1_13(oracle_lib, e, x, z, want):
    assert oracle_lib.nmf_budget(e, x, z, 1e-12) == pytest.approx(want, rel=1e-14)


def test_budgets_switch_at_the_residual_threshold(oracle_lib):
    """Section 4: the fixed budget c*tol applies while e >= 1e-6, the adaptive one
    below; the switch value and the constant are parameters."""
    below = math.nextafter(1e-6, 0.0)
    # just below the switch: (3/4)(1e-12)/36 for eq. 1.18 and 1e-12/6 for eq. 1.13
    # (the latter is larger than the fixed budget: the formula, not a cap, applies)
    for f, want in ((lambda e: oracle_lib.nsf_budget(e, 3.0, 1e-12), 0.75e-12 / 36),
                    (lambda e: oracle_lib.nmf_budget(e, 3.0, 3.0, 1e-12), 1e-12 / 6)):
        assert f(1e-6) == 1e-16
        assert f(0.5) == 1e-16
        assert f(below) == pytest.approx(want, rel=1e-14)
    assert oracle_lib.nsf_budget(1e-3, 3.0, 1e-10, c_fixed=1e-2) == pytest.approx(1e-12,
                                                                                 rel=1e-15)
    # a switch moved up to 1e-2 puts e = 6e-7 ... 1e-3 on the adaptive side
    assert oracle_lib.nsf_budget(1e-3, 1.0, 1e-12, switch_res=1e-2) == pytest.approx(
        0.75e-6 / 4, rel=1e-14)


def test_nsf_trace_budget_is_eq_1_18_of_the_same_step(oracle_lib):
    """Every budget after the switch is eq. 1.18 of that step's e_k and ||X^_k||_F
    (the index reading of the budget), every budget before it is c4*tol."""
    A = W.laplacian_2d(30, jitter=0.05, seed=2, m=8.0)
    r = oracle_lib.nsf(A, tol=1e-12)
    k = r.iters
    e, x, tau = r.trace["e"][:k], r.trace["xfro"][:k], r.trace["tau"][:k]
    after = e < 1e-6
    assert after.sum() >= 1 and (~after).sum() >= 3
    assert np.all(tau[~after] == 1e-16)
    np.testing.assert_allclose(tau[after], 0.75 * e[after] ** 2 / (3 * x[after] + x[after] ** 3),
                               rtol=1e-14)
    # ||X^_k||_F of a converging symmetric iterate approaches sqrt(n)
    assert abs(x[-1] - math.sqrt(A.n)) < 1e-6 * math.sqrt(A.n)


def test_nmf_trace_budget_is_eq_1_13(oracle_lib):
    """After the switch the NMF budget is e^2/(||X^||_F + ||X^^-1||_F); near
    convergence X^^-1 ~ X^ (X^2 ~ I), so it is e^2/(2||X^||_F) to O(e), far from
    e^2/(||X^|| ||X^^-1||) ~ e^2/n or (3/4)e^2/(3x + x^3)."""
    A = W.laplacian_2d(12, jitter=0.05, seed=2, m=8.0)
    r = oracle_lib.nmf(A, tol=1e-12, scale=0.0)
    k = r.iters
    e, x, tau = r.trace["e"][:k], r.trace["xfro"][:k], r.trace["tau"][:k]
    after = e < 1e-6
    assert after.sum() >= 1
    assert np.all(tau[~after] == 1e-16)
    np.testing.assert_allclose(tau[after] * 2 * x[after] / e[after] ** 2, 1.0, atol=1e-5)


def test_theorem_3_2_1_nsf_vs_ns(oracle_lib):
    """Once the residual is small, ||R^_k - R_k|| <= 3 ||R_k|| (eq. 1.18 budget)."""
    A = W.laplacian_2d(20, jitter=0.05, seed=2, m=8.0)
    f = oracle_lib.nsf(A, tol=1e-12)
    u = oracle_lib.nsf(A, tol=1e-12, c_fixed=0.0, switch_res=0.0)
    k = min(f.iters, u.iters)
    # residual norms of both runs agree to within the filter budget scale
    for i in range(k + 1):
        dR = abs(f.trace["e"][i] - u.trace["e"][i])
        if u.trace["e"][i] < 1e-2:
            assert dR <= 3 * u.trace["e"][i] + 1e-13
    Xf, Xu = _dense(f), _dense(u)
    assert np.linalg.norm(Xf - Xu) < 1e-12


# ---------------------------------------------------------------------------
# status handling
# ---------------------------------------------------------------------------
def test_guard_max_iter_returns_last_iterate(oracle_lib):
    A = W.laplacian_2d(8, jitter=0.05, seed=2, m=8.0)
    r = oracle_lib.nsf(A, tol=1e-12, max_iter=1)
    assert r.status == "ENOCONV"
    assert r.iters == 1 and r.nnz > 0


def test_guard_divergence(oracle_lib):
    A = W.laplacian_2d(8, jitter=0.05, seed=2, m=8.0)
    r = oracle_lib.nsf(A, tol=1e-12, scale=1.0)     # unscaled: ||I - A^2|| >> 1
    assert r.status == "EDIVERGED"


def test_invalid_input(oracle_lib):
    A = W.tridiag_c1(8)
    bad = W.Csr(n=8, indptr=A.indptr.copy(), indices=A.indices.copy(), data=A.data.copy())
    bad.indices[0], bad.indices[1] = bad.indices[1], bad.indices[0]
    bad.indices[2] = bad.indices[3]
    assert oracle_lib.nsf(bad).status == "EINVAL"
    assert oracle_lib.nsf(A, tol=0.0).status == "EINVAL"


# ---------------------------------------------------------------------------
# filtered Newton (Algorithm 3.1.1)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("make,exact", [
    (lambda: W.laplacian_2d(10, jitter=0.05, seed=2, m=8.0), None),
    (lambda: W.convdiff_2d(10, beta=0.5, sigma=4.0, m=8.0), None),
    (lambda: W.ode_block_matrix(100), lambda: cf.sign_ode_block(100)),
], ids=["lap2d", "convdiff", "ode"])
def test_nmf_matches_exact_sign(oracle_lib, make, exact):
    A = make()
    r = oracle_lib.nmf(A, tol=1e-12)
    assert r.status == "OK"
    S = exact() if exact else cf.dense_sign(A.to_dense())
    assert _rel(_dense(r), S) < 1e-11
    assert r.trace["inner_total"] > 0


def test_nmf_agrees_with_nsf(oracle_lib):
    A = W.laplacian_2d(24, jitter=0.05, seed=2, m=8.0)
    a = oracle_lib.nsf(A, tol=1e-12)
    b = oracle_lib.nmf(A, tol=1e-12)
    assert _rel(_dense(b), _dense(a)) < 1e-11


@pytest.mark.parametrize("make", [
    lambda: W.tridiag_c1(128),
    lambda: W.convdiff_2d(9, beta=0.5, sigma=4.0, m=8.0, scale_by_h=False),
], ids=["c1", "convdiff"])
def test_nsf_loop_obeys_eq_1_8(oracle_lib, make):
    """Unfiltered steps of the NSF loop obey ||R_{k+1}|| <= 3/4||R_k||^2 + 1/4||R_k||^3
    (eq. 1.8; the Frobenius norm is submultiplicative), which pins the update
    coefficients of the loop itself (a wrong 1/2 still converges, but linearly)."""
    A = make()
    r = oracle_lib.nsf(A, tol=1e-13, c_fixed=0.0, switch_res=0.0)
    e = r.trace["e"][: r.iters + 1]
    n = A.n
    for k in range(len(e) - 1):
        assert e[k + 1] <= 0.75 * e[k] ** 2 + 0.25 * e[k] ** 3 + 1e-14 * math.sqrt(n) * 10, (k, e)


def test_local_sign_row_similar_matches_schur():
    """The diagonal-similarity route to a patch sign (symmetric eigensolver) gives
    the Schur-method row on a nonsymmetric convection-diffusion patch."""
    A = W.convdiff_2d(14, beta=0.5, sigma=4.0, m=8.0)
    N = 14
    d = np.sqrt(1.0 + A.meta["b"]) ** (np.arange(A.n) % N)
    for i in (0, 5 * N + 6, A.n - 1):
        idx1, r1 = cf.local_sign_row(A, i, 6)
        idx2, r2 = cf.local_sign_row_similar(A, i, 6, d)
        assert np.array_equal(idx1, idx2)
        assert np.abs(r1 - r2).max() <= 1e-13
    with pytest.raises(ValueError):
        cf.local_sign_row_similar(A, 7, 4, np.ones(A.n))


def test_local_sign_rows_from_one_patch():
    """Rows taken from one shared patch: on a grid the patch covers entirely they
    are the rows of the whole matrix's Schur sign (this pins the row-to-patch
    index mapping); on a larger grid every row returned equals the single-row
    patch of the same radius to the truncation level (the two patches differ, so
    the rows agree to that level, not to rounding)."""
    N = 12
    A = W.convdiff_2d(N, beta=0.5, sigma=4.0, m=8.0)
    d = np.sqrt(1.0 + A.meta["b"]) ** (np.arange(A.n) % N)
    S = cf.dense_sign_schur(A.to_dense())
    rows = cf.local_sign_rows_similar(A, 5 * N + 6, 30, 3, d)
    assert len(rows) == 2 * 3 * 3 + 2 * 3 + 1      # the Manhattan ball of radius 3
    for i, (idx, v) in rows.items():
        assert len(idx) == A.n
        assert np.abs(v - S[i]).max() <= 1e-13
    N = 40
    A = W.convdiff_2d(N, beta=0.5, sigma=4.0, m=8.0)
    d = np.sqrt(1.0 + A.meta["b"]) ** (np.arange(A.n) % N)
    rows = cf.local_sign_rows_similar(A, 20 * N + 17, 14, 2, d)
    for i in (20 * N + 17, 20 * N + 19, 21 * N + 16, 18 * N + 17):
        idx1, r1 = cf.local_sign_row_similar(A, i, 14, d)
        idx2, r2 = rows[i]
        full = np.zeros(A.n)
        full[idx2] = r2
        part = np.zeros(A.n)
        part[idx1] = r1
        # each is within the radius-14 truncation (~1e-11 here) of the sign
        assert np.abs(full - part).max() <= 1e-10 * np.abs(part).max()


# ---------------------------------------------------------------------------
# the certified last residual: with Xt = X - D thinned by a filter cut,
# ||I - X^2||_F <= ||I - Xt^2||_F + 2 ||Xt||_2 ||D||_F + ||D||_F^2,
# ||Xt||_2 <= sqrt(||X||_1 ||X||_inf), and sqrt(1 + ||I - Xt^2||_F) when Xt is
# symmetric -- checked on oracle iterates against dense norms
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("make,sym", [
    (lambda: W.laplacian_2d(20, jitter=0.05, seed=2, m=8.0), True),
    (lambda: W.convdiff_2d(14, beta=0.5, sigma=4.0, m=8.0), False),
])
def test_thinned_residual_bound(oracle_lib, make, sym):
    from oracle import core
    A = make()
    for iters in (3, 4, 100):
        r = core.nsf(A, tol=1e-12, max_iter=iters)
        X = _dense(r)
        if sym:
            X = 0.5 * (X + X.T)  # exactly symmetric, as the GPU's symmetric iterates
        I = np.eye(A.n)
        e = np.linalg.norm(I - X @ X)
        one_inf = math.sqrt(np.abs(X).sum(0).max() * np.abs(X).sum(1).max())
        for tau in (1e-3, 1e-8, 1e-13):
            _, keep, dsq = core.filter_values(X.ravel(), tau)
            Xt = np.where(keep.reshape(X.shape), X, 0.0)
            delta = math.sqrt(dsq)
            assert delta <= tau
            assert abs(np.linalg.norm(X - Xt) - delta) <= 1e-12 * max(delta, 1e-300) + 1e-300
            et = np.linalg.norm(I - Xt @ Xt)
            s2 = np.linalg.norm(Xt, 2)
            assert s2 <= one_inf * (1 + 1e-12)
            if sym:
                assert np.array_equal(Xt, Xt.T)
                assert s2 <= math.sqrt(1.0 + et) * (1 + 1e-12)
                s = math.sqrt(1.0 + et)
            else:
                s = one_inf
            assert e <= (et + 2.0 * s * delta + delta * delta) * (1 + 1e-9) + 1e-14


# ---------------------------------------------------------------------------
# the inverse starts of the filtered Newton iteration: for X' = (X + X^-1)/2,
# I - X' X^-1 = (I - X^-2)/2 and I - X' (2 X^-1) = -X^-2, and the inverse
# Newton-Schulz residual squares every step (checked on dense matrices)
# ---------------------------------------------------------------------------
def test_newton_inverse_start_identities():
    rng = np.random.default_rng(3)
    n = 40
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.concatenate([rng.uniform(1.5, 9.0, n // 2), -rng.uniform(1.5, 9.0, n - n // 2)])
    X = (Q * lam) @ Q.T
    Xi = np.linalg.inv(X)
    Xn = 0.5 * (X + Xi)
    I = np.eye(n)
    assert np.allclose(I - Xn @ Xi, 0.5 * (I - Xi @ Xi), atol=1e-12)
    assert np.allclose(I - Xn @ (2.0 * Xi), -(Xi @ Xi), atol=1e-12)
    # per eigenvalue, 2 X^-1 is the better start exactly when |x| > sqrt(3)
    e1 = np.abs(0.5 * (1 - 1 / lam ** 2))
    e2 = np.abs(1 / lam ** 2)
    assert np.array_equal(e2 < e1, np.abs(lam) > math.sqrt(3))
    # T_{j+1} = T_j^2 for Z_{j+1} = Z_j + Z_j T_j, T_j = I - X Z_j (any X, Z)
    A = rng.standard_normal((n, n))
    Z = 0.01 * rng.standard_normal((n, n))
    T = I - A @ Z
    Z1 = Z + Z @ T
    assert np.allclose(I - A @ Z1, T @ T, atol=1e-10)
