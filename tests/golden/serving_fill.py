"""Resident entries per row of the served families, from the FP64 oracle alone:
for each family (1D tridiagonal, 2D 5-point, 2D convection-diffusion; the
generators of the served stream) and tolerance, the peak over the iterations of
nnz(X^_k) + nnz(R^_k) + nnz(Xbar_{k+1}) per row -- the iterate, its residual
and the update's candidates that a request holds on the device at once.  The
server's admission table (csrc/serve.hip, kFill) is these numbers x 1.25,
rounded up; tests/test_golden_cpu.py checks that it covers this file.

    python tests/golden/serving_fill.py   # writes tests/golden/serving_fill.txt
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import oracle  # noqa: E402
import workloads as W  # noqa: E402

# the 1D fill saturates far below the served sizes; the 2D fill grows with the
# grid up to the decay radius, so 2D is measured at the largest size of each of
# the server's two size classes (n <= 128^2, n <= 256^2), and convection-diffusion
# beside it at 128^2
FAMILIES = {
    "1d": lambda: W.laplacian_1d(8192, sigma=2.0, jitter=0.05, seed=5001, m=4.0),
    "2d": lambda: W.laplacian_2d(128, sigma=4.0, jitter=0.05, seed=5002, m=8.0),
    "cd": lambda: W.convdiff_2d(128, beta=0.5, sigma=4.0, m=8.0, jitter=0.05, seed=5003),
    "2d256": lambda: W.laplacian_2d(256, sigma=4.0, jitter=0.05, seed=5002, m=8.0),
}
TOLS = (1e-6, 1e-10, 1e-12)


def main():
    lines = ["# family n avg_row_of_A tol peak_resident_entries_per_row (X^ + R^ + Xbar)"]
    for name, make in FAMILIES.items():
        A = make()
        for tol in TOLS:
            r = oracle.nsf(A, tol=tol)
            tr = r.trace
            k = r.iters
            peak = max((tr["nnz_x"][i] + tr["nnz_r"][i] + tr["nnz_bar"][i]) / A.n
                       for i in range(k))
            peak = max(peak, (tr["nnz_x"][k] + tr["nnz_r"][k]) / A.n)
            lines.append(f"{name} {A.n} {A.nnz / A.n:.2f} {tol:g} {peak:.0f}")
            print(lines[-1], flush=True)
    open(os.path.join(HERE, "serving_fill.txt"), "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
