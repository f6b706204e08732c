"""Seeded matrix and request-stream generators.

Every matrix is returned as a :class:`Csr` (int64 row pointers, int32 column
indices sorted within each row, float64 values, no stored zeros), the storage
convention of the method (Section 4 keeps matrices in a sparse format that
never stores zeros).

Families
--------
* ``tridiag_c1``: tridiag(-1, 2, -1) - 2I, i.e. tridiag(-1, 0, -1).
* ``ode_block_matrix``: the Section 4.2 matrix [[0, B], [I, 0]] with
  B = tridiag(1/16, 7/8, 1/16) (eqs. 1.25-1.26).
* ``laplacian_1d/2d/3d``: lattice Laplacians shifted by sigma, with a seeded
  diagonal jitter and an optional staggered on-site term m*(-1)^(x+y+z).
* ``convdiff_2d``: upwind convection-diffusion (convection in x) shifted by
  sigma, with the same optional staggered term.

The staggered term opens a spectral gap of half-width m around sigma (the
lattices are bipartite, so the hopping part anticommutes with the staggering
sign).  With m = 0 the shifted lattices have eigenvalues arbitrarily close to
zero and their sign is a dense matrix; the gapped reading keeps sign(A)
exponentially localised, like the matrices the paper targets.

Grid ordering is lexicographic with x fastest, 0-based.  Random numbers come
from ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class Csr:
    n: int
    indptr: np.ndarray   # int64, n+1
    indices: np.ndarray  # int32, nnz, sorted within each row
    data: np.ndarray     # float64, nnz, no zeros
    meta: Dict = dataclasses.field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.data, self.indices, self.indptr), shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        return self.to_scipy().toarray()


def _from_scipy(m, meta=None) -> Csr:
    m = sp.csr_matrix(m, dtype=np.float64)
    m.eliminate_zeros()
    m.sum_duplicates()
    m.sort_indices()
    return Csr(n=m.shape[0],
               indptr=np.ascontiguousarray(m.indptr, dtype=np.int64),
               indices=np.ascontiguousarray(m.indices, dtype=np.int32),
               data=np.ascontiguousarray(m.data, dtype=np.float64),
               meta=dict(meta or {}))


def _path(N: int) -> sp.csr_matrix:
    """Adjacency of a path of N sites (1 on the first off-diagonals)."""
    e = np.ones(N - 1)
    return sp.diags([e, e], [-1, 1], shape=(N, N), format="csr")


def _stagger(shape) -> np.ndarray:
    """(-1)^(x+y+z) on a lexicographic grid with x fastest."""
    idx = np.indices(shape[::-1]).reshape(len(shape), -1)  # z/y/x ordering, x fastest
    return np.where(idx.sum(axis=0) % 2 == 0, 1.0, -1.0)


def tridiag_c1(n: int = 1024) -> Csr:
    """tridiag(-1, 2, -1) - 2I = tridiag(-1, 0, -1); the zero diagonal is not stored."""
    A = -_path(n)
    return _from_scipy(A, {"family": "tridiag_c1", "symmetric": True,
                           "inertia": 0 if n % 2 == 0 else None})


def ode_block_matrix(nB: int, lam: float = 1.0 / 16.0) -> Csr:
    """A = [[0, B], [I, 0]] with B = tridiag(lam, 1-2lam, lam) (Section 4.2, eqs. 1.25-1.26).

    sign(A) = [[0, B^(1/2)], [B^(-1/2), 0]]; A is 2*nB x 2*nB.
    """
    e = np.ones(nB)
    B = sp.diags([lam * e[:-1], (1 - 2 * lam) * e, lam * e[:-1]], [-1, 0, 1], format="csr")
    I = sp.identity(nB, format="csr")
    A = sp.bmat([[None, B], [I, None]], format="csr")
    return _from_scipy(A, {"family": "ode_block", "nB": nB, "lam": lam, "symmetric": False,
                           "inertia": 0})


def laplacian_1d(n: int, sigma: float = 2.0, jitter: float = 0.0, seed: Optional[int] = None,
                 m: float = 0.0) -> Csr:
    """tridiag(-1, 2, -1) - (sigma + u_i) on the diagonal + m*(-1)^x, u ~ U[-jitter, jitter]."""
    u = _jitter(n, jitter, seed)
    chi = _stagger((n,))
    diag = 2.0 - sigma - u + m * chi
    A = sp.diags(diag, 0, format="csr") - _path(n)
    return _from_scipy(A, {"family": "lap1d", "shape": (n,), "sigma": sigma, "jitter": jitter,
                           "seed": seed, "m": m, "symmetric": True,
                           "inertia": int(chi.sum()) if (m > 0 and m > jitter + abs(2.0 - sigma)) else None})


def laplacian_2d(N: int, sigma: float = 4.0, jitter: float = 0.0, seed: Optional[int] = None,
                 m: float = 0.0) -> Csr:
    """5-point Laplacian on an N x N grid, diagonal 4 - (sigma + u_i) + m*chi_i."""
    n = N * N
    I = sp.identity(N, format="csr")
    H = sp.kron(I, _path(N)) + sp.kron(_path(N), I)
    u = _jitter(n, jitter, seed)
    chi = _stagger((N, N))
    diag = 4.0 - sigma - u + m * chi
    A = sp.diags(diag, 0, format="csr") - H
    gapped = m > 0 and m > jitter + abs(4.0 - sigma)
    return _from_scipy(A, {"family": "lap2d", "shape": (N, N), "sigma": sigma, "jitter": jitter,
                           "seed": seed, "m": m, "symmetric": True,
                           "inertia": int(chi.sum()) if gapped else None})


def laplacian_3d(N: int, sigma: float = 6.0, perturb: float = 0.0, seed: Optional[int] = None,
                 m: float = 0.0) -> Csr:
    """7-point Laplacian on an N^3 grid, diagonal 6 - sigma + u_i + m*chi_i, u ~ U[-perturb, perturb]."""
    n = N ** 3
    I = sp.identity(N, format="csr")
    P = _path(N)
    H = (sp.kron(sp.kron(I, I), P) + sp.kron(sp.kron(I, P), I) + sp.kron(sp.kron(P, I), I))
    u = _jitter(n, perturb, seed)
    chi = _stagger((N, N, N))
    diag = 6.0 - sigma + u + m * chi
    A = sp.diags(diag, 0, format="csr") - H
    gapped = m > 0 and m > perturb + abs(6.0 - sigma)
    return _from_scipy(A, {"family": "lap3d", "shape": (N, N, N), "sigma": sigma,
                           "jitter": perturb, "seed": seed, "m": m, "symmetric": True,
                           "inertia": int(chi.sum()) if gapped else None})


def convdiff_2d(N: int, beta: float = 0.5, sigma: float = 4.0, m: float = 0.0,
                scale_by_h: bool = True, jitter: float = 0.0, seed: Optional[int] = None) -> Csr:
    """Upwind convection-diffusion on an N x N grid, convection beta in +x, shifted by sigma.

    Stencil (times h^2): centre 4 + b - sigma - u_i + m*chi_i, west -(1 + b), east -1,
    north -1, south -1, with b = beta*h, h = 1/(N+1) (or b = beta when
    ``scale_by_h`` is False).
    """
    n = N * N
    b = beta / (N + 1) if scale_by_h else beta
    I = sp.identity(N, format="csr")
    e = np.ones(N - 1)
    west = sp.diags([e], [-1], shape=(N, N), format="csr")   # x-1 neighbour
    east = sp.diags([e], [1], shape=(N, N), format="csr")    # x+1 neighbour
    Hx = (1.0 + b) * sp.kron(I, west) + sp.kron(I, east)
    Hy = sp.kron(_path(N), I)
    u = _jitter(n, jitter, seed)
    chi = _stagger((N, N))
    diag = 4.0 + b - sigma - u + m * chi
    A = sp.diags(diag, 0, format="csr") - Hx - Hy
    gapped = m > 0 and m > jitter + abs(4.0 + b - sigma) + b
    return _from_scipy(A, {"family": "convdiff2d", "shape": (N, N), "beta": beta, "b": b,
                           "sigma": sigma, "m": m, "jitter": jitter, "seed": seed,
                           "symmetric": False, "inertia": int(chi.sum()) if gapped else None})


def random_sparse(n: int, mean_row: float = 8.0, seed: int = 0, powerlaw: bool = True,
                  max_row: Optional[int] = None, ncols: Optional[int] = None) -> Csr:
    """Random pattern with (optionally) power-law row lengths and U[-1,1] values.

    Used for product-level tests; carries no structure of the method.
    """
    rng = np.random.default_rng(seed)
    ncols = n if ncols is None else ncols
    if powerlaw:
        lens = np.floor(mean_row * 0.5 * (rng.pareto(1.5, size=n) + 1.0)).astype(np.int64)
    else:
        lens = rng.poisson(mean_row, size=n).astype(np.int64)
    cap = ncols if max_row is None else min(max_row, ncols)
    lens = np.clip(lens, 0, cap)
    rows, cols = [], []
    for i in range(n):
        c = rng.choice(ncols, size=int(lens[i]), replace=False) if lens[i] else np.empty(0, np.int64)
        rows.append(np.full(len(c), i))
        cols.append(c)
    r = np.concatenate(rows) if rows else np.empty(0, np.int64)
    c = np.concatenate(cols) if cols else np.empty(0, np.int64)
    v = rng.uniform(-1.0, 1.0, size=len(r))
    v[v == 0.0] = 0.5
    A = sp.csr_matrix((v, (r, c)), shape=(n, ncols))
    out = _from_scipy(A, {"family": "random", "seed": seed})
    return out


def _jitter(n: int, amp: float, seed: Optional[int]) -> np.ndarray:
    if amp == 0.0:
        return np.zeros(n)
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, size=n)


# ---------------------------------------------------------------------------
# Benchmark configurations (full size) and their run options.
# The staggered term m is the gapped reading of the shifted lattices; m = 0
# gives the literal (gapless) matrices.
# ---------------------------------------------------------------------------
CONFIGS: Dict[str, Dict] = {
    "c1": dict(desc="1D tridiag(-1,2,-1)-2I, n=1024", tol=1e-12, stop_rule=1, precision=0,
               filter_y=0),
    "c2": dict(desc="2D 5-point 256^2 minus (4+U[-.05,.05]) + 8*stagger, n=65536", tol=1e-12,
               stop_rule=0, precision=0, filter_y=0, N=256, m=8.0, seed=2),
    "c3": dict(desc="2D upwind conv-diff 512^2, beta*h, sigma=4, + 8*stagger, n=262144",
               tol=1e-12, stop_rule=0, precision=1, filter_y=1, N=512, m=8.0),
    "c4": dict(desc="3D 7-point 64^3 minus 6I + U[-.5,.5] + 12*stagger, n=262144", tol=1e-10,
               stop_rule=0, precision=1, filter_y=1, N=64, m=12.0, seed=4),
}


def config_matrix(name: str, N: Optional[int] = None, literal: bool = False) -> Csr:
    """Matrix of a named configuration; ``N`` overrides the grid size (scaled-down parity cases)."""
    cfg = CONFIGS[name]
    if name == "c1":
        return tridiag_c1(N if N is not None else 1024)
    m = 0.0 if literal else cfg["m"]
    if name == "c2":
        return laplacian_2d(N or cfg["N"], sigma=4.0, jitter=0.05, seed=cfg["seed"], m=m)
    if name == "c3":
        return convdiff_2d(N or cfg["N"], beta=0.5, sigma=4.0, m=m, scale_by_h=True)
    if name == "c4":
        return laplacian_3d(N or cfg["N"], sigma=6.0, perturb=0.5, seed=cfg["seed"], m=m)
    raise KeyError(name)


# ---------------------------------------------------------------------------
# Served request stream.
# ---------------------------------------------------------------------------
def served_stream(count: int = 2000, rate: float = 50.0, seed: int = 5, n_min: int = 1024,
                  n_max: int = 65536, tols=(1e-6, 1e-10)) -> List[Dict]:
    """Poisson arrivals of sign requests over three gapped families.

    Each request: arrival time (s), family, n, tol, jitter seed.  2D families use
    N = round(sqrt(n)) and n = N^2.  Build the matrix with :func:`request_matrix`.
    """
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    fams = rng.integers(0, 3, size=count)
    logn = rng.uniform(math.log(n_min), math.log(n_max), size=count)
    tol_idx = rng.integers(0, len(tols), size=count)
    out = []
    for i in range(count):
        fam = ("lap1d", "lap2d", "convdiff2d")[int(fams[i])]
        n = int(round(math.exp(logn[i])))
        if fam != "lap1d":
            N = max(2, int(round(math.sqrt(n))))
            n = N * N
        out.append(dict(id=i, arrival=float(t[i]), family=fam, n=n, tol=float(tols[tol_idx[i]]),
                        seed=5000 + i))
    return out


def request_matrix(req: Dict) -> Csr:
    fam, n, s = req["family"], req["n"], req["seed"]
    if fam == "lap1d":
        return laplacian_1d(n, sigma=2.0, jitter=0.05, seed=s, m=4.0)
    N = int(round(math.sqrt(n)))
    if fam == "lap2d":
        return laplacian_2d(N, sigma=4.0, jitter=0.05, seed=s, m=8.0)
    return convdiff_2d(N, beta=0.5, sigma=4.0, m=8.0, scale_by_h=True, jitter=0.05, seed=s)
