"""Accuracy measures of Example 1 (Section 4.1): e_a, e_s by power iteration and n_i.

The paper estimates the two operator norms with the power method to a relative tolerance
of 1e-2.  A and F are symmetric here (F up to its own approximation error), so the
iteration runs on the operator itself: |lambda_max| of a symmetric operator is its
2-norm.  n_i counts the iterations of the right-preconditioned GMRES of the library or
the oracle (the paper counts CG iterations) to a relative residual of 1e-12.
"""
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "example1_rss_accuracy.json")


def paper_row(tol: float, n: int) -> dict:
    with open(GOLDEN) as f:
        rows = json.load(f)["rss_s"]
    for r in rows:
        if r["tol"] == tol and r["n"] == n:
            return r
    raise KeyError((tol, n))


def power_norm(op, x0, rtol: float = 1e-2, maxit: int = 50, norm=np.linalg.norm):
    """Largest |eigenvalue| of op by power iteration from x0, to relative change rtol."""
    v = x0 / norm(x0)
    lam = 0.0
    for _ in range(maxit):
        w = op(v)
        lam_new = float(norm(w))
        if lam_new == 0.0:
            return 0.0
        v = w / lam_new
        if abs(lam_new - lam) <= rtol * lam_new:
            return lam_new
        lam = lam_new
    return lam
