"""Seeded synthetic inputs shared by the GPU path's tests/bench and the oracle.

This module holds no arithmetic of the factorization itself: it only produces
point sets, right-hand sides and the problem constants of the discretized
integral equation (Section 1, the regular-grid Nystrom system; Section 4.1,
Example 1 on the unit square).

Workloads (2D Laplace, second kind): N = n*n cell centres of a uniform grid on
[0,1]^2, DOF g = i + n*j at ((i+1/2)h, (j+1/2)h) with h = 1/n, A_ii = 1 and
A_ij = h^2 * (-1/(2*pi)) * log|x_i - x_j|.
"""
from __future__ import annotations

import numpy as np


def grid_points(n: int) -> np.ndarray:
    """Cell centres of the uniform n x n grid on the unit square, row order g = i + n*j."""
    h = 1.0 / n
    c = (np.arange(n, dtype=np.float64) + 0.5) * h
    x = np.empty((n * n, 2), dtype=np.float64)
    x[:, 0] = np.tile(c, n)
    x[:, 1] = np.repeat(c, n)
    return x


def random_points(npts: int, seed: int) -> np.ndarray:
    """Uniform random points in the open unit square (seeded)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(npts, 2)).astype(np.float64)


def jittered_grid_points(n: int, jitter: float, seed: int) -> np.ndarray:
    """Grid cell centres moved by U(-jitter*h, jitter*h) in each coordinate (seeded)."""
    h = 1.0 / n
    rng = np.random.default_rng(seed)
    x = grid_points(n)
    x += rng.uniform(-jitter * h, jitter * h, size=x.shape)
    return x


def rhs(npts: int, seed: int = 0, nrhs: int = 1) -> np.ndarray:
    """Right-hand side b ~ N(0,1), FP64; shape (N,) for one RHS, else (N, nrhs) column-major data."""
    rng = np.random.default_rng(seed)
    if nrhs == 1:
        return rng.standard_normal(npts)
    return np.asfortranarray(rng.standard_normal((nrhs, npts)).T)


def laplace2d_weight(n: int) -> float:
    """Quadrature weight h^2 of the n x n grid (the 1/N of the regular-grid Nystrom system)."""
    return 1.0 / float(n * n)


# Named problem configurations: the small parity case, the medium refinement case
# and the headline case (2D Laplace, leaf <= 64 points, 16 proxy points on a circle
# of radius 1.25 box sides = 2.5 box half-widths).
CONFIGS = {
    "laplace2d_n64": dict(n=64, tol=1e-6),
    "laplace2d_n512": dict(n=512, tol=1e-6),
    "laplace2d_n1024": dict(n=1024, tol=1e-6),
}


def problem(n: int, tol: float = 1e-6, leaf_size: int = 64, n_proxy: int = 16,
            proxy_radius: float = 1.25) -> dict:
    """Parameter dictionary for the 2D Laplace grid problem of side n."""
    return dict(dim=2, diag=1.0, weight=laplace2d_weight(n), tol=tol, leaf_size=leaf_size,
                n_proxy=n_proxy, proxy_radius=proxy_radius, root_lo=(0.0, 0.0), root_side=1.0)


def laplace2d_cell_self_term(n: int) -> float:
    """Integral of K(z) = -(1/(2 pi)) log|z| over one grid cell [-h/2, h/2]^2, h = 1/n.

    This is the diagonal entry of the first-kind system of Example 1 (Section 4.1), where
    the paper approximates the same integral by adaptive quadrature.  Closed form: by the
    eight-fold symmetry of the square, in polar coordinates over the triangle
    0 <= theta <= pi/4, 0 <= r <= a / cos(theta) (a = h/2),
      int_square log(x^2 + y^2) = 8 a^2 (log a + log(2)/2 - 3/2 + pi/4),
    and K = -(1/(4 pi)) log(x^2 + y^2).
    """
    a = 0.5 / float(n)
    return -(8.0 * a * a / (4.0 * np.pi)) * (np.log(a) + 0.5 * np.log(2.0) - 1.5 + 0.25 * np.pi)


def problem_first_kind(n: int, tol: float = 1e-6, leaf_size: int = 64, n_proxy: int = 16,
                       proxy_radius: float = 1.25) -> dict:
    """The first-kind volume integral equation of Example 1 (Section 4.1) on the n x n grid:
    A_ij = h^2 K(x_i - x_j) for i != j and A_ii = the integral of K over one cell."""
    d = problem(n, tol, leaf_size, n_proxy, proxy_radius)
    d["diag"] = laplace2d_cell_self_term(n)
    return d
