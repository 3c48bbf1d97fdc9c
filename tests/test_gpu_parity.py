"""GPU parity: librss (through the C ABI) against the oracle on the same seeded inputs."""
import numpy as np
import pytest

from oracle import rss_oracle as O
from paper_1609_08130_amd import workloads as W
from tests.parity_util import factor_tol, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rss():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1609_08130_amd import rss as mod
    return mod


def _gpu_factor(rss, pts, p: O.Params, precision="fp64"):
    d = torch.tensor(pts, dtype=torch.float64, device="cuda")
    return rss.Factor(d, diag=p.diag, weight=p.weight, tol=p.tol, leaf_size=p.leaf_size, n_proxy=p.n_proxy,
                      proxy_radius=p.proxy_radius, root_lo=p.root_lo, root_side=p.root_side,
                      precision=precision)


def _compare(rss, name, pts, p, nrhs=1, precision="fp64"):
    say(f"[parity] case={name} N={len(pts)} tol={p.tol} leaf={p.leaf_size} precision={precision}")
    F = _gpu_factor(rss, pts, p, precision)
    R = O.factor(pts, p)
    depth, ntop = F.shape()
    assert depth == R.depth
    # skeleton index sets: exact, every box of every level
    mism = []
    for (t, box), (S, Rr) in R.skeletons.items():
        Sg, Rg = F.box_sets(t, box)
        if not (np.array_equal(Sg, S) and np.array_equal(Rg, Rr)):
            mism.append((t, box, len(S), len(Sg)))
    assert not mism, f"skeleton mismatches (depth, box, |S| oracle, |S| gpu): {mism[:10]}"
    assert np.array_equal(F.top_set(), R.top)
    b = W.rhs(len(pts), seed=0, nrhs=nrhs)
    bt = torch.tensor(b, device="cuda")
    tol = factor_tol(p.tol)
    x = F.solve(bt).cpu().numpy()
    xr = O.solve(R, b)
    ex = np.linalg.norm(x - xr) / np.linalg.norm(xr)
    y = F.apply(bt).cpu().numpy()
    yr = O.apply(R, b)
    ey = np.linalg.norm(y - yr) / np.linalg.norm(yr)
    sg, ld = F.logdet()
    sr, lr = O.logdet(R)
    say(f"[parity] case={name} solve_rel={ex:.2e} apply_rel={ey:.2e} logdet gpu={ld:.15e} oracle={lr:.15e} tol={tol:.1e}")
    assert ex <= tol and ey <= tol
    assert sg == sr and abs(ld - lr) <= tol * max(1.0, abs(lr)) + 1e-13 * len(pts)
    F.close()
    return ex, ey


def test_parity_grid64_tol1e6(rss):
    n = 64
    _compare(rss, "grid64", W.grid_points(n), O.Params(**W.problem(n, 1e-6)))


@pytest.mark.parametrize("tol", [1e-3, 1e-9])
def test_parity_grid64_other_tolerances(rss, tol):
    n = 64
    _compare(rss, f"grid64_tol{tol}", W.grid_points(n), O.Params(**W.problem(n, tol)))


def test_parity_ragged_grid100_three_levels(rss):
    # 100 x 100 grid with leaf 64: boxes of 36..49 points, depth 4 (levels 4, 3, 2)
    n = 100
    _compare(rss, "grid100", W.grid_points(n), O.Params(**W.problem(n, 1e-6)), nrhs=3)


def test_parity_random_points_uneven_boxes(rss):
    pts = W.random_points(3000, seed=7)
    p = O.Params(weight=1.0 / 3000, tol=1e-6, leaf_size=24)
    _compare(rss, "random3000", pts, p)


def test_parity_jittered_grid_small_leaf(rss):
    pts = W.jittered_grid_points(48, 0.1, seed=3)
    p = O.Params(weight=1.0 / 48 ** 2, tol=1e-7, leaf_size=16)
    _compare(rss, "jitter48_leaf16", pts, p)


@pytest.mark.parametrize("n_proxy,radius", [(64, 2.5), (32, 1.0)])
def test_parity_proxy_surfaces(rss, n_proxy, radius):
    # the paper's proxy circle (64 points at 2.5 box sides, Section 4) and a tight one
    n = 64
    d = W.problem(n, 1e-6)
    d.update(n_proxy=n_proxy, proxy_radius=radius)
    _compare(rss, f"grid64_proxy{n_proxy}_r{radius}", W.grid_points(n), O.Params(**d))


@pytest.mark.parametrize("root_side", [3.0, 0.0])
def test_parity_translated_domain(rss, root_side):
    # points in [2, 5] x [-1, 2]: an explicit root box, or (root_side 0) the bounding
    # square of the points, so box geometry and proxy circles are not those of [0, 1]^2
    rng = np.random.default_rng(21)
    pts = np.column_stack([2.0 + 3.0 * rng.random(2500), -1.0 + 3.0 * rng.random(2500)])
    p = O.Params(weight=9.0 / 2500, tol=1e-6, leaf_size=32, root_lo=(2.0, -1.0), root_side=root_side)
    _compare(rss, f"translated_root{root_side}", pts, p)


@pytest.mark.parametrize("npts,leaf", [(1, 64), (50, 64), (200, 64), (300, 40)])
def test_small_and_degenerate_trees(rss, npts, leaf):
    pts = W.random_points(npts, seed=npts)
    p = O.Params(weight=1.0 / max(npts, 1), tol=1e-6, leaf_size=leaf)
    say(f"[parity] case=small N={npts} leaf={leaf}")
    F = _gpu_factor(rss, pts, p)
    R = O.factor(pts, p)
    assert F.shape()[0] == R.depth
    A = O.dense_matrix(pts, p)
    b = W.rhs(npts, seed=1)
    x = F.solve(torch.tensor(b, device="cuda")).cpu().numpy()
    np.testing.assert_allclose(x, O.solve(R, b), rtol=0, atol=factor_tol(p.tol) * np.abs(x).max())
    if R.depth <= 1:
        np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=0, atol=1e-12 * np.abs(x).max())
        sg, ld = F.logdet()
        sr, lr = np.linalg.slogdet(A)
        assert sg == sr and abs(ld - lr) <= 1e-12 * max(1.0, abs(lr)) + 1e-14 * npts
    F.close()


@pytest.mark.parametrize("diag,weight", [(1.0, None), (1e-3, 1.0)])
def test_unskeletonized_top_block_961(rss, diag, weight):
    # 31 x 31 grid, leaf 256: depth 1, nothing is skeletonized and the top block is the whole
    # 961 x 961 matrix, so the blocked top LU runs its first panels from global memory and
    # the later ones from LDS.  With diag 1e-3 and weight 1 the diagonal is small against the
    # kernel, partial pivoting interchanges 290 rows and cond(A) is about 7.7e4.
    n = 31
    pts = W.grid_points(n)
    d = W.problem(n, 1e-6, leaf_size=256)
    d["diag"] = diag
    if weight is not None:
        d["weight"] = weight
    p = O.Params(**d)
    say(f"[parity] case=top961 diag={diag} N={n * n}")
    F = _gpu_factor(rss, pts, p)
    assert F.shape() == (1, n * n)
    A = O.dense_matrix(pts, p)
    b = W.rhs(n * n, seed=2)
    x = F.solve(torch.tensor(b, device="cuda")).cpu().numpy()
    xr = np.linalg.solve(A, b)
    bound = 1e-12 if diag == 1.0 else 2e-10          # ~ 10 cond(A) eps
    assert np.linalg.norm(x - xr) <= bound * np.linalg.norm(xr)
    sg, ld = F.logdet()
    sr, lr = np.linalg.slogdet(A)
    assert sg == sr and abs(ld - lr) <= (1e-12 if diag == 1.0 else 1e-10) * max(1.0, abs(lr))
    F.close()


@pytest.mark.parametrize("precision,nrhs", [("fp64", 4), ("fp64", 6), ("mixed", 7)])
def test_solve_nrhs_matches_single(rss, precision, nrhs):
    # right-hand sides go through the sweeps in groups of four (the last group partial):
    # every column equals its single-vector solve bit for bit
    n = 64
    p = O.Params(**W.problem(n, 1e-6))
    F = _gpu_factor(rss, W.grid_points(n), p, precision)
    B = torch.tensor(W.rhs(n * n, seed=5, nrhs=nrhs), device="cuda")
    u32 = precision == "mixed"
    X = F.solve(B, use_fp32=u32)
    for j in range(nrhs):
        xj = F.solve(B[:, j].contiguous(), use_fp32=u32)
        assert torch.equal(X[:, j], xj), j
    # F^{-1} F = I
    Y = F.apply(B)
    Z = F.solve(Y)
    assert float((Z - B).abs().max()) <= 1e-12 * float(B.abs().max())
    F.close()


def test_gmres_refined_solution_matches_dense(rss):
    n = 64
    pts = W.grid_points(n)
    p = O.Params(**W.problem(n, 1e-6))
    A = O.dense_matrix(pts, p)
    b = W.rhs(n * n, seed=0)
    xe = np.linalg.solve(A, b)
    for prec in ("fp64", "mixed"):
        say(f"[parity] case=gmres precision={prec}")
        F = _gpu_factor(rss, pts, p, prec)
        x, it, rr = F.gmres(torch.tensor(b, device="cuda"), rtol=1e-12, maxit=20, use_fp32=(prec == "mixed"))
        x = x.cpu().numpy()
        err = np.linalg.norm(x - xe) / np.linalg.norm(xe)
        say(f"[parity] gmres {prec}: iters={it} relres={rr:.2e} err_vs_dense={err:.2e}")
        assert rr <= 1e-12 and it <= 6 and err <= 1e-10
        F.close()


def test_mixed_factor_is_accurate(rss):
    n = 64
    pts = W.grid_points(n)
    p = O.Params(**W.problem(n, 1e-6))
    F = _gpu_factor(rss, pts, p, "mixed")
    R = O.factor(pts, p)
    b = W.rhs(n * n, seed=0)
    x64 = F.solve(torch.tensor(b, device="cuda")).cpu().numpy()
    x32 = F.solve(torch.tensor(b, device="cuda"), use_fp32=True).cpu().numpy()
    xr = O.solve(R, b)
    e64 = np.linalg.norm(x64 - xr) / np.linalg.norm(xr)
    e32 = np.linalg.norm(x32 - xr) / np.linalg.norm(xr)
    say(f"[parity] mixed factor: fp64-apply err={e64:.2e} fp32-apply err={e32:.2e}")
    # The skeleton-skeleton Schur update is O(1) (X_SR ~ -T, X_RR ~ I + T^T T), so FP32
    # products perturb F by a few u32 = 6e-8 relative; the FP32 factor copy used by the
    # preconditioner solve adds the same order again.  cond(A) ~ 1.13 here.
    u32 = float(np.finfo(np.float32).eps) / 2
    assert e64 <= 40 * u32 and e32 <= 80 * u32
    F.close()


def test_argument_errors_on_device(rss):
    pts = W.grid_points(16)
    pts[3] = pts[7]
    with pytest.raises(rss.RSSError) as ei:
        _gpu_factor(rss, pts, O.Params(**W.problem(16, 1e-6)))
    assert ei.value.name == "RSS_E_ARG"
    pts = W.grid_points(16) + 2.0
    with pytest.raises(rss.RSSError) as ei:
        _gpu_factor(rss, pts, O.Params(**W.problem(16, 1e-6)))
    assert ei.value.name == "RSS_E_ARG"


# ---- generalized square root F^{1/2} = (prod V_i) P_t D^{1/2} (Section 3.3) ---------------

@pytest.mark.parametrize("n,tol,precision", [(64, 1e-6, "fp64"), (64, 1e-9, "mixed"), (100, 1e-6, "fp64")])
def test_sqrt_apply_matches_oracle(rss, n, tol, precision):
    pts = W.grid_points(n)
    p = O.Params(**W.problem(n, tol))
    say(f"[parity] case=sqrt grid{n} tol={tol} precision={precision}")
    F = _gpu_factor(rss, pts, p, precision)
    R = O.factor(pts, p)
    b = W.rhs(n * n, seed=5, nrhs=2)
    bt = torch.tensor(b, device="cuda")
    # mixed: the FP32 Schur products perturb F by a few u32 (as for F^{-1} b above)
    ftol = factor_tol(tol) if precision == "fp64" else 40 * float(np.finfo(np.float32).eps) / 2
    for adj in (False, True):
        y = F.sqrt_apply(bt, adjoint=adj).cpu().numpy()
        yr = O.sqrt_apply(R, b, adjoint=adj)
        e = np.linalg.norm(y - yr) / np.linalg.norm(yr)
        say(f"[parity] sqrt adjoint={adj} rel={e:.2e}")
        assert e <= ftol
    # F = F^{1/2} (F^{1/2})^* on the device itself.  FP64: to rounding.  Mixed: the FP32
    # Schur products leave the stored blocks symmetric only to a few u32, so V_i^* = W_i
    # (E^T = G) holds to that order (measured 6e-6, about 100 u32, at N = 4096 and tol 1e-9).
    y2 = F.sqrt_apply(F.sqrt_apply(bt, adjoint=True)).cpu().numpy()
    yf = F.apply(bt).cpu().numpy()
    e2 = np.linalg.norm(y2 - yf) / np.linalg.norm(yf)
    say(f"[parity] sqrt C C^* vs F rel={e2:.2e}")
    assert e2 <= (1e-12 if precision == "fp64" else 400 * float(np.finfo(np.float32).eps) / 2)
    F.close()


def test_sqrt_apply_without_skeletonization_is_cholesky(rss):
    # depth <= 1: F = A and F^{1/2} is the Cholesky factor of A
    pts = W.random_points(200, seed=11)
    p = O.Params(weight=1.0 / 200, tol=1e-6, leaf_size=256)
    F = _gpu_factor(rss, pts, p)
    assert F.shape()[0] <= 1
    A = O.dense_matrix(pts, p)
    Lc = np.linalg.cholesky(A)
    b = W.rhs(200, seed=3)
    bt = torch.tensor(b, device="cuda")
    np.testing.assert_allclose(F.sqrt_apply(bt).cpu().numpy(), Lc @ b, rtol=0, atol=1e-13 * np.abs(Lc @ b).max())
    np.testing.assert_allclose(F.sqrt_apply(bt, adjoint=True).cpu().numpy(), Lc.T @ b, rtol=0,
                               atol=1e-13 * np.abs(Lc.T @ b).max())
    F.close()


def test_sqrt_apply_argument_errors(rss):
    import ctypes
    pts = W.grid_points(16)
    F = _gpu_factor(rss, pts, O.Params(**W.problem(16, 1e-6, leaf_size=16)))
    x = torch.ones(256, dtype=torch.float64, device="cuda")
    lib = rss.lib()
    p = ctypes.c_void_p(x.data_ptr())
    # aliasing input and output, nrhs < 1, ld < N: RSS_E_ARG, nothing written
    assert lib.rss_sqrt_apply(F._h, p, p, 1, 256, 0, None) == 1
    y = torch.zeros(256, dtype=torch.float64, device="cuda")
    q = ctypes.c_void_p(y.data_ptr())
    assert lib.rss_sqrt_apply(F._h, p, q, 0, 256, 0, None) == 1
    assert lib.rss_sqrt_apply(F._h, p, q, 1, 255, 1, None) == 1
    torch.cuda.synchronize()
    assert float(y.abs().max()) == 0.0
    F.close()


def test_sqrt_apply_rejects_indefinite_blocks(rss):
    pts = W.grid_points(16)
    p = O.Params(diag=-1.0, weight=1.0 / 256, tol=1e-6, leaf_size=16)
    F = _gpu_factor(rss, pts, p)
    with pytest.raises(rss.RSSError) as ei:
        F.sqrt_apply(torch.ones(256, dtype=torch.float64, device="cuda"))
    assert ei.value.name == "RSS_E_SINGULAR"
    # the factor itself stays usable
    x = F.solve(torch.ones(256, dtype=torch.float64, device="cuda")).cpu().numpy()
    assert np.all(np.isfinite(x))
    F.close()
