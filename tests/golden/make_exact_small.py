"""Writes exact_small.txt: small tridiagonal matrices with their eigenvalues
from exact rational characteristic polynomials, rooted at 300 and again at
400 digits (the two must round to the same doubles: clustered roots of a
polynomial are ill-conditioned in its coefficients, and 100 digits were not
enough for the constant-diagonal case).

Only the oracle (exact_charpoly_roots) and the seeded input generator are
called. The fixture pins the oracle (bisection against exact roots) and is the
fixed reference of the GPU path's tiny cases. The matrices are the degenerate
and classic shapes of the problem: n = 1 and 2, Wilkinson's W+_21 and W-_21
(top eigenvalues of W+_21 coincide to about 14 digits), the 1-2-1 Toeplitz
matrix, a zero coupling in the middle, a graded diagonal, a constant diagonal
with tiny couplings (heavy deflation in every merge) and the paper's random
families (Section 5.1) at n = 24.

Run from the repository root:  python tests/golden/make_exact_small.py
"""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import tdgen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "exact_small.txt")


def cases():
    yield "n1", np.array([0.375]), np.zeros(0)
    yield "n2", np.array([1.0, -2.0]), np.array([0.5])
    i = np.arange(21, dtype=np.float64)
    yield "wilkinson_plus_21", np.abs(i - 10.0), np.ones(20)
    yield "wilkinson_minus_21", i - 10.0, np.ones(20)
    yield "toeplitz_121_n16", np.full(16, 2.0), np.full(15, -1.0)
    d, e = tdgen.tridiag("uniform", 20, cfg=tdgen.CFG_TEST, inst=11)
    e[9] = 0.0
    yield "uniform_zero_coupling_n20", d, e
    yield "graded_n12", 4.0 ** -np.arange(12, dtype=np.float64), 0.5 * 4.0 ** -np.arange(1, 12, dtype=np.float64)
    yield "constant_tiny_coupling_n16", np.ones(16), np.full(15, 1e-9)
    for fam in ["paper_uniform", "paper_normal", "paper_clustered"]:
        d, e = tdgen.tridiag(fam, 24, cfg=tdgen.CFG_TEST, inst=5)
        yield f"{fam}_n24", d, e


def main():
    lines = ["# name n / d (n values) / e (n-1 values) / exact eigenvalues ascending (n values)",
             "# written by tests/golden/make_exact_small.py (oracle.exact_charpoly_roots, 300 and 400 digits)"]
    for name, d, e in cases():
        if len(d) > 1:
            lam = [float(x) for x in oracle.exact_charpoly_roots(d, e, dps=300)]
            chk = [float(x) for x in oracle.exact_charpoly_roots(d, e, dps=400)]
            assert lam == chk, f"{name}: roots not converged in the working precision"
        else:
            lam = [float(d[0])]
        lines.append(f"{name} {len(d)}")
        lines.append(" ".join(repr(float(x)) for x in d))
        lines.append(" ".join(repr(float(x)) for x in e))
        lines.append(" ".join(repr(x) for x in lam))
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
