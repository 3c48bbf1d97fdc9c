"""Example 1 of Section 4.1 (first-kind equation on the unit square) on the CPU: the cell
self-term against numerical quadrature, and the oracle's e_a, e_s, n_i against the
paper's RS-S accuracy table (order of magnitude: the paper used n_occ = 256 and 64
proxies, this configuration 64 and 16)."""
import numpy as np
import pytest
from scipy import integrate

from oracle import rss_oracle as O
from paper_1609_08130_amd import workloads as W
from tests.example1_util import paper_row, power_norm


@pytest.mark.parametrize("n", [64, 512, 4096])
def test_cell_self_term_matches_quadrature(n):
    # the cell [-h/2, h/2]^2 is eight copies of the triangle 0 <= y <= x <= h/2, whose only
    # singular point (the origin) is a vertex, where adaptive quadrature converges
    a = 0.5 / n
    f = lambda y, x: -np.log(x * x + y * y) / (4.0 * np.pi)
    tri, _ = integrate.dblquad(f, 0.0, a, lambda x: 0.0, lambda x: x, epsabs=0.0, epsrel=1e-13)
    assert abs(W.laplace2d_cell_self_term(n) - 8.0 * tri) <= 1e-12 * abs(8.0 * tri)


def test_first_kind_problem_definition():
    n = 64
    d = W.problem_first_kind(n, 1e-6)
    assert d["weight"] == 1.0 / (n * n)
    assert d["diag"] == W.laplace2d_cell_self_term(n)
    # the self-term is positive and close to h^2 (log h dominates)
    assert 0.5 / (n * n) < d["diag"] < 2.0 / (n * n)


@pytest.mark.parametrize("tol", [1e-6, 1e-9])
def test_oracle_first_kind_accuracy_against_paper(tol):
    n = 64
    p = O.Params(**W.problem_first_kind(n, tol))
    pts = W.grid_points(n)
    F = O.factor(pts, p)
    A = O.dense_matrix(pts, p)
    rng = np.random.default_rng(1)
    x0 = rng.standard_normal(len(pts))
    nA = power_norm(lambda v: A @ v, x0)
    e_a = power_norm(lambda v: A @ v - O.apply(F, v), x0) / nA
    e_s = power_norm(lambda v: v - A @ O.solve(F, v), x0)
    x = rng.standard_normal(len(pts))
    b = A @ x
    _, n_i, relres = O.gmres(lambda v: A @ v, lambda v: O.solve(F, v), b, rtol=1e-12)
    ref = paper_row(tol, 512)
    print(f"oracle first kind n={n} tol={tol}: e_a={e_a:.2e} e_s={e_s:.2e} n_i={n_i} "
          f"(paper RS-S at 512^2: {ref['e_a']:.1e} {ref['e_s']:.1e} {ref['n_i']})")
    assert relres <= 1e-12
    assert e_a <= 10 * tol
    assert ref["e_a"] / 100 <= e_a <= ref["e_a"] * 100
    assert e_s <= ref["e_s"] * 100
    assert n_i <= ref["n_i"] + 2
