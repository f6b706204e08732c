"""Writes tests/golden/<config>_fp64_oracle.npz from the FP64 CPU oracle alone
(filtered Newton-Schulz, Algorithm 3.2.1) on a full-size workload matrix.

Stored: the oracle's summary (status, iterations, nnz, e of the result,
||S||_F, trace), a fingerprint of the input CSR, the row probe of
tests/golden/probe.py for every row (a whole-matrix checksum), and a set of
complete rows (columns and values) for entry-wise comparison.

    python tests/golden/make_fullsize_golden.py c2 [output directory]
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import oracle  # noqa: E402
import probe  # noqa: E402
import workloads as W  # noqa: E402

RUNS = {
    # config: (options of the oracle run, grid side)
    "c2": (dict(tol=1e-12), 256),
    "c3": (dict(tol=1e-12, filter_y=1), 512),
}


def fingerprint(A) -> str:
    h = hashlib.sha256()
    for a in (np.ascontiguousarray(A.indptr, np.int64), np.ascontiguousarray(A.indices, np.int32),
              np.ascontiguousarray(A.data, np.float64)):
        h.update(a.tobytes())
    return h.hexdigest()[:32]


def sample_rows(n: int, N: int):
    """Rows of every kind a product launch treats differently: the grid's corners
    and edges, the centre, both sides of the boundaries of row groups (2, 4, 8 and
    16 rows), of the 64-group chunks dealt to one XCD, and a seeded random set."""
    s = {0, 1, N - 1, N, n // 2, n // 2 + N // 2, n - N, n - 1}
    for g in (8 * 64, 4 * 64, 16 * 64):
        for c in (1, 3, 7):
            s.update({c * g - 1, c * g})
    for b in (2, 4, 8, 16):
        s.update({n // 3 // b * b - 1, n // 3 // b * b})
    rng = np.random.default_rng(12345)
    s.update(int(i) for i in rng.integers(0, n, 40))
    return np.array(sorted(i for i in s if 0 <= i < n), dtype=np.int64)


def main(cfg: str, outdir: str = HERE):
    kw, N = RUNS[cfg]
    os.environ["ORACLE_PROGRESS"] = "1"   # one line per iteration on stderr
    A = W.config_matrix(cfg)
    t = time.perf_counter()
    r = oracle.nsf(A, **kw)
    dt = time.perf_counter() - t
    print(f"{cfg}: oracle {r.status} iters={r.iters} nnz={r.nnz} e={r.res_fro:.3e} "
          f"{dt:.1f} s", flush=True)
    assert r.status == "OK"
    p = probe.row_probe_numpy(r.indptr, r.indices, r.data)
    rows = sample_rows(A.n, N)
    lens = (r.indptr[rows + 1] - r.indptr[rows]).astype(np.int64)
    rcols = np.concatenate([r.indices[r.indptr[i]:r.indptr[i + 1]] for i in rows])
    rvals = np.concatenate([r.data[r.indptr[i]:r.indptr[i + 1]] for i in rows])
    diag = 0.0
    for i in range(A.n):
        b, e = r.indptr[i], r.indptr[i + 1]
        k = np.searchsorted(r.indices[b:e], i)
        if k < e - b and r.indices[b + k] == i:
            diag += r.data[b + k]
    out = os.path.join(outdir, f"{cfg}_fp64_oracle.npz")
    np.savez_compressed(out, fingerprint=fingerprint(A), options=repr(sorted(kw.items())),
                        iters=r.iters, nnz=r.nnz, res_fro=r.res_fro,
                        fro=float(np.sqrt(np.sum(r.data ** 2))), trace=diag,
                        probe=p, rows=rows, row_len=lens, row_cols=rcols, row_vals=rvals,
                        oracle_seconds=dt, oracle_threads=os.cpu_count())
    print("wrote", out, os.path.getsize(out), "bytes", flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "c2",
         sys.argv[2] if len(sys.argv) > 2 else HERE)
