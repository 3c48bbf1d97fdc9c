"""Shared helpers of the GPU parity tests (tolerances and the case runner)."""
import sys

import numpy as np

EPS = np.finfo(np.float64).eps


def factor_tol(tol: float) -> float:
    """Relative tolerance for F^{-1} b, F x and log|det F| between two correct FP64 RS-S
    implementations: T = R11^{-1} R12 carries u * cond(R11) <= u * 100 / tol relative
    rounding error (cond(R11) ~ |R_00| / |R_kk| >= 1 / tol), and F depends on T through
    the near-field blocks at first order."""
    return 1e-12 + 100.0 * EPS / max(tol, 1e-12)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()
