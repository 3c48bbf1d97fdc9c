"""Shared helpers of the GPU parity tests: tolerances and element-wise comparisons.

Agreement bound between the HIP path and the oracle, both FP64 (`FP64_AGREE`): the two
compute the same factor with different operation orders (double-double Gram matrix and
pivoted Cholesky against Householder QR for the ID; Gauss-Jordan against LU for X_RR;
MFMA tiles against numpy products), so every result differs by rounding only.  The
interpolation matrix T = R11^{-1} R12 carries the largest amplification: cond(R11) is up
to |R_00| / |R_kk| ~ 1 / tol, so an entry of T can move by ~u / tol relative to max |T|.
At tol >= 1e-6 that is <= 2.2e-10 in the worst case, but the measured agreement of T, of
every other record block and of F^{-1} b, F b is far tighter (see the per-case prints);
the bounds below sit above the measured values by the margins stated with them.
"""
import contextlib
import os
import sys

import numpy as np

EPS = np.finfo(np.float64).eps


def vec_bound(tol: float) -> float:
    """Element-wise bound on |x_gpu - x_oracle| / max|x_oracle| for F^{-1} b and F b (FP64
    factors of a well-conditioned matrix, cond(A) ~ 1.13 for the second-kind systems).  F
    and F^{-1} do not depend on the rounding of T at first order (a change of T changes the
    dropped far-field block only by tol times that change), so the bound does not grow as
    1 / tol: measured <= 3.4e-15 (norm-relative) at tol 1e-3, 1e-6 and 1e-9, and 1e-12
    leaves a factor ~300.  Ill-conditioned systems (the first-kind equation) pass their own
    bound."""
    return 1e-12


def record_bound(tol: float) -> float:
    """Element-wise bound on record blocks (T, X_RR, X_JR, G) relative to the block's
    largest entry: u cond(R11), and greedy pivoted QR keeps cond(R11) within a modest
    factor of |R_00| / |R_kk| <= 1 / tol: measured up to 13 u / tol over the strong steps
    of the parity cases (tol 1e-3 to 1e-9) and 130 u / tol for a weak step of RS-WS at
    tol 1e-9 (larger ranks, so R11 closer to its worst case), so 1000 u / tol, never below
    1e-12."""
    return max(1e-12, 1000.0 * EPS / tol)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_maxdiff(a, b) -> float:
    """max |a - b| / max |b| (0 for empty or all-zero references)."""
    a = np.asarray(a)
    b = np.asarray(b)
    if b.size == 0:
        return 0.0
    m = float(np.abs(b).max())
    d = float(np.abs(a - b).max())
    return d / m if m > 0 else d


def compare_skeletons(F, skeletons: dict):
    """Every box of every level: the GPU's (S, R) equal the oracle's exactly."""
    mism = []
    for (t, box), (S, R) in skeletons.items():
        Sg, Rg = F.box_sets(t, box)
        if not (np.array_equal(Sg, S) and np.array_equal(Rg, R)):
            mism.append((t, box, len(S), len(Sg)))
    assert not mism, f"skeleton mismatches (depth, box, |S| oracle, |S| gpu): {mism[:10]}"
    return len(skeletons)


def compare_record(F, depth: int, box: int, ref: dict, tol: float, weak: bool = False):
    """T, X_RR, X_JR (= E X_RR of the oracle) and G element-wise, J exactly; the rows of J
    are matched by global index.  Returns the largest relative difference."""
    g = F.box_record(depth, box, weak=weak)
    assert np.array_equal(g["J"], ref["J"]), (depth, box, "J list")
    worst = 0.0
    for key in ("T", "XRR", "XJR", "G"):
        a, b = g[key], ref[key]
        assert a.shape == b.shape, (depth, box, key, a.shape, b.shape)
        e = rel_maxdiff(a, b)
        worst = max(worst, e)
        assert e <= record_bound(tol), (depth, box, key, e)
    return worst


@contextlib.contextmanager
def plan_override(spec: str):
    """Launch-plan values for the factorizations created inside the block (the library reads
    RSS_TUNE at every rss_factor_create), so a test can run a kernel variant that the tuned
    table does not pick for its box counts."""
    old = os.environ.get("RSS_TUNE")
    if spec:
        os.environ["RSS_TUNE"] = spec
    try:
        yield
    finally:
        if old is None:
            os.environ.pop("RSS_TUNE", None)
        else:
            os.environ["RSS_TUNE"] = old
