"""Exact matrix signs used to pin the oracle (test infrastructure only).

* Symmetric tridiagonal Toeplitz matrices tridiag(c, d, c) are diagonalised by
  the sine basis v_j(i) = sqrt(2/(n+1)) sin(i j theta), theta = pi/(n+1), with
  eigenvalues d + 2c cos(j theta).  Any function f of such a matrix is
      f(T)_ik = F(i-k) - F(i+k),   F(m) = 1/(n+1) sum_j f(lambda_j) cos(m j theta)
  (1-based i, k), which is evaluated here with exact argument reduction of
  m*j modulo 2(n+1) and compensated summation.
* The Section 4.2 matrix A = [[0, B], [I, 0]] has sign(A) = [[0, B^(1/2)],
  [B^(-1/2), 0]] (eq. 1.26); B = tridiag(1/16, 7/8, 1/16) is of the above kind.
* Dense definitions (Section 1): sign(A) = V sign(Lambda) V^T for symmetric A,
  and the Schur form sign(A) = Q sign(T) Q^* for general A, with the Schur
  form ordered so that the left-half-plane eigenvalues come first; then
  sign(T) = [[-I, Y], [0, I]] with T11 Y - Y T22 = -2 T12.
* A matrix diagonally similar to a symmetric one, M = D S D^-1 with S
  symmetric and D = diag(d) > 0, has sign(M) = D sign(S) D^-1, since a
  matrix function commutes with similarity.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla


def _toeplitz_function_table(n: int, lam: np.ndarray, f) -> np.ndarray:
    """F(m) for m = 0 .. 2n+1, F(m) = 1/(n+1) sum_j f(lam_j) cos(pi m j/(n+1))."""
    j = np.arange(1, n + 1, dtype=np.int64)
    fv = np.asarray(f(lam), dtype=np.float64)
    period = 2 * (n + 1)
    F = np.empty(2 * n + 2)
    for m in range(2 * n + 2):
        r = (m * j) % period                         # exact argument reduction
        terms = fv * np.cos(np.pi * r.astype(np.float64) / (n + 1))
        F[m] = math.fsum(terms) / (n + 1)
    return F


def tridiag_toeplitz_function(n: int, d: float, c: float, f) -> np.ndarray:
    """Dense f(T) for T = tridiag(c, d, c) of order n (symmetric)."""
    theta = np.pi / (n + 1)
    lam = d + 2.0 * c * np.cos(np.arange(1, n + 1) * theta)
    F = _toeplitz_function_table(n, lam, f)
    i = np.arange(1, n + 1)
    diff = np.abs(i[:, None] - i[None, :])
    summ = i[:, None] + i[None, :]
    return F[diff] - F[summ]


def sign_tridiag_c1(n: int) -> np.ndarray:
    """sign(tridiag(-1, 0, -1)), the first benchmark matrix, in closed form."""
    return tridiag_toeplitz_function(n, 0.0, -1.0, np.sign)


def ode_sqrt_blocks(nB: int, lam: float = 1.0 / 16.0):
    """(B^(1/2), B^(-1/2)) for B = tridiag(lam, 1-2lam, lam)."""
    half = tridiag_toeplitz_function(nB, 1.0 - 2.0 * lam, lam, np.sqrt)
    mhalf = tridiag_toeplitz_function(nB, 1.0 - 2.0 * lam, lam, lambda x: 1.0 / np.sqrt(x))
    return half, mhalf


def sign_ode_block(nB: int, lam: float = 1.0 / 16.0) -> np.ndarray:
    """sign([[0, B], [I, 0]]) = [[0, B^(1/2)], [B^(-1/2), 0]] (eq. 1.26)."""
    half, mhalf = ode_sqrt_blocks(nB, lam)
    S = np.zeros((2 * nB, 2 * nB))
    S[:nB, nB:] = half
    S[nB:, :nB] = mhalf
    return S


def dense_sign_sym(M: np.ndarray) -> np.ndarray:
    w, V = np.linalg.eigh(M)
    if np.any(w == 0.0):
        raise ValueError("zero eigenvalue: sign undefined")
    return (V * np.sign(w)) @ V.T


def dense_sign_schur(M: np.ndarray) -> np.ndarray:
    """Schur method of Section 1 for a real or complex square matrix."""
    T, Q, k = sla.schur(M.astype(np.complex128), output="complex", sort="lhp")
    n = M.shape[0]
    ev = np.diag(T)
    if np.any(ev.real == 0.0):
        raise ValueError("eigenvalue on the imaginary axis: sign undefined")
    T11, T12, T22 = T[:k, :k], T[:k, k:], T[k:, k:]
    sT = np.zeros((n, n), dtype=np.complex128)
    sT[:k, :k] = -np.eye(k)
    sT[k:, k:] = np.eye(n - k)
    if 0 < k < n:
        sT[:k, k:] = sla.solve_sylvester(T11, -T22, -2.0 * T12)
    S = Q @ sT @ Q.conj().T
    if np.isrealobj(M):
        return S.real
    return S


def dense_sign(M: np.ndarray) -> np.ndarray:
    if np.allclose(M, M.T, rtol=0, atol=0):
        return dense_sign_sym(M)
    return dense_sign_schur(M)


def ball(A, i: int, radius: int) -> np.ndarray:
    """Sorted indices within graph distance `radius` of i in the pattern of A (CSR)."""
    seen = {i}
    frontier = [i]
    for _ in range(radius):
        nxt = []
        for r in frontier:
            for c in A.indices[A.indptr[r]:A.indptr[r + 1]]:
                c = int(c)
                if c not in seen:
                    seen.add(c)
                    nxt.append(c)
        frontier = nxt
    return np.array(sorted(seen), dtype=np.int64)


def local_sign_row(A, i: int, radius: int):
    """Row i of sign(A_B), A_B the principal submatrix of A on the ball B of
    the given radius around i (dense definition on the patch).

    For a matrix whose sign is exponentially localised (a spectral gap), the
    entries of this row differ from those of sign(A) by a quantity that decays
    like q^radius, q < 1 the decay rate of sign(A); it is how single rows of a
    sign too large for a dense method are checked.  Returns (columns, values).
    """
    idx = ball(A, i, radius)
    sub = A.to_scipy()[idx][:, idx].toarray()
    S = dense_sign(sub)
    loc = int(np.searchsorted(idx, i))
    return idx, S[loc]


def local_sign_row_similar(A, i: int, radius: int, d: np.ndarray):
    """local_sign_row for a matrix with D^-1 A D symmetric, D = diag(d): the patch
    sign is D_B sign(D_B^-1 A_B D_B) D_B^-1 with a symmetric eigendecomposition
    (principal submatrices keep the similarity).  Raises if D^-1 A_B D_B is not
    symmetric to rounding."""
    idx = ball(A, i, radius)
    sub = A.to_scipy()[idx][:, idx].toarray()
    dB = np.asarray(d, dtype=np.float64)[idx]
    S = sub * (dB[None, :] / dB[:, None])
    if not np.allclose(S, S.T, rtol=0, atol=1e-13 * np.abs(S).max()):
        raise ValueError("patch is not symmetric under the given scaling")
    sS = dense_sign_sym(0.5 * (S + S.T))
    loc = int(np.searchsorted(idx, i))
    return idx, sS[loc] * (dB[loc] / dB)


def local_sign_rows_similar(A, center: int, radius: int, reach: int, d: np.ndarray):
    """local_sign_row_similar for every row within graph distance `reach` of
    `center`, from one patch: the ball of radius radius + reach around the
    centre contains the radius-`radius` ball of each such row, so each row is
    at least `radius` hops from the patch boundary (same truncation bound).
    Returns {row: (columns, values)}."""
    idx = ball(A, center, radius + reach)
    near = ball(A, center, reach)
    sub = A.to_scipy()[idx][:, idx].toarray()
    dB = np.asarray(d, dtype=np.float64)[idx]
    S = sub * (dB[None, :] / dB[:, None])
    if not np.allclose(S, S.T, rtol=0, atol=1e-13 * np.abs(S).max()):
        raise ValueError("patch is not symmetric under the given scaling")
    sS = dense_sign_sym(0.5 * (S + S.T))
    out = {}
    for i in near:
        loc = int(np.searchsorted(idx, i))
        out[int(i)] = (idx, sS[loc] * (dB[loc] / dB))
    return out
