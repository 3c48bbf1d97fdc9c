"""GPU: the exact operator, GMRES refinement, and properties at the full workload sizes."""
import numpy as np
import pytest

from oracle import rss_oracle as O
from paper_1609_08130_amd import workloads as W
from tests.parity_util import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rss():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1609_08130_amd import rss as mod
    return mod


def _factor(rss, pts, prm, precision="fp64"):
    prm = dict(prm)
    prm.pop("dim", None)
    return rss.Factor(torch.tensor(pts, device="cuda"), precision=precision, **prm)


@pytest.mark.parametrize("n", [64, 100])
def test_fft_operator_matches_oracle(rss, n):
    pts = W.grid_points(n)
    prm = W.problem(n, 1e-6)
    F = _factor(rss, pts, prm)
    assert F.info()["exact_operator"] == "fft"
    x = W.rhs(n * n, seed=4, nrhs=2)
    y = F.matvec(torch.tensor(x, device="cuda")).cpu().numpy()
    yr = O.dense_matrix(pts, O.Params(**prm)) @ x
    err = np.abs(y - yr).max() / np.abs(yr).max()
    say(f"[operator] fft n={n} max rel err {err:.2e}")
    assert err <= 1e-13
    F.close()


def test_direct_operator_on_scattered_points(rss):
    pts = W.random_points(3000, seed=9)
    prm = dict(weight=1.0 / 3000, tol=1e-6, leaf_size=32)
    F = _factor(rss, pts, prm)
    assert F.info()["exact_operator"] == "direct"
    x = W.rhs(3000, seed=2)
    y = F.matvec(torch.tensor(x, device="cuda")).cpu().numpy()
    yr = O.dense_matrix(pts, O.Params(**prm)) @ x
    assert np.abs(y - yr).max() <= 1e-13 * np.abs(yr).max()
    F.close()


def _colour0_leaf_sample(F, pts, prm, count):
    """Skeletons of colour-0 leaf boxes: their ID input is untouched kernel data, so the
    oracle computes them from scratch (Section 3.2, eq. smallid)."""
    p = O.Params(**prm)
    tree = O.build_tree(pts, p)
    D, nb = tree.depth, 2 ** tree.depth
    rng = np.random.default_rng(0)
    cands = [b for b in range(nb * nb) if O.colour(b, nb) == 0]
    for b in rng.choice(cands, size=min(count, len(cands)), replace=False):
        b = int(b)
        B = tree.leaf_lists[b]
        rows = [O.matrix_block(pts, tree.leaf_lists[o], B, p) for o in O.ring(b, nb, 2)]
        rows.append(O.kernel_block(O.proxy_points(b, D, tree, p), pts[B], p))
        s, r, _ = O.id_sorted(O.cpqr_id(np.vstack(rows), p.tol))
        Sg, Rg = F.box_sets(D, b)
        assert np.array_equal(Sg, B[s]) and np.array_equal(Rg, B[r]), b


@pytest.mark.parametrize("n,precision,tol", [(512, "mixed", 1e-6), (1024, "mixed", 1e-6), (1024, "fp64", 1e-6),
                                             (1024, "mixed", 1e-3), (1024, "mixed", 1e-9)])
def test_full_size_properties(rss, n, precision, tol):
    pts = W.grid_points(n)
    prm = W.problem(n, tol)
    say(f"[fullsize] n={n} precision={precision} tol={tol} factor")
    F = _factor(rss, pts, prm, precision)
    _colour0_leaf_sample(F, pts, prm, 6)
    b = torch.tensor(W.rhs(n * n, seed=0), device="cuda")
    use32 = precision == "mixed"
    # F^{-1} F = I up to the precision of the factor copy used by the solve
    z = F.solve(F.apply(b), use_fp32=use32)
    e = float(torch.linalg.norm(z - b) / torch.linalg.norm(b))
    say(f"[fullsize] n={n} |F^-1 F b - b|/|b| = {e:.2e}")
    assert e <= (2e-6 if use32 else 1e-13)
    x, it, rr = F.gmres(b, rtol=1e-10, maxit=30, use_fp32=use32)
    # independent residual: the oracle's numpy FFT operator on the CPU
    xr = x.cpu().numpy()
    res = np.linalg.norm(W.rhs(n * n, seed=0) - O.matvec_grid_fft(n, O.Params(**prm), xr))
    rel = res / np.linalg.norm(W.rhs(n * n, seed=0))
    say(f"[fullsize] n={n} gmres iters={it} relres(gpu)={rr:.2e} relres(oracle operator)={rel:.2e}")
    assert rr <= 1e-10 and rel <= 2e-10 and it <= 8
    if precision == "fp64":
        # generalized square root at full size: F^{1/2} (F^{1/2})^* b = F b
        y2 = F.sqrt_apply(F.sqrt_apply(b, adjoint=True))
        e2 = float(torch.linalg.norm(y2 - F.apply(b)) / torch.linalg.norm(F.apply(b)))
        say(f"[fullsize] n={n} |C C^* b - F b|/|F b| = {e2:.2e}")
        assert e2 <= 1e-12
    F.close()
