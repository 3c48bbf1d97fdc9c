"""GPU parity: librss (through the C ABI) against the oracle on the same seeded inputs."""
import numpy as np
import pytest

from oracle import rss_oracle as O
from paper_1609_08130_amd import workloads as W
from tests.parity_util import (compare_record, compare_skeletons, plan_override, record_bound, rel_maxdiff, say,
                               vec_bound)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rss():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1609_08130_amd import rss as mod
    return mod


# Mixed precision against the FP64 oracle.  u32 = 2^-24.  The mixed factor keeps every self
# block A(B_a, B_a) in FP64 and forms the S x S products of each step in FP64 (they carry the
# O(1) skeleton-skeleton entries); FP32 rounding touches only the blocks between different
# boxes, whose entries are w K (~1e-5 here), and the Schur products into them.  Independent
# roundings of those entries move F b by about u32 ||A - diag(A)||_F / sqrt(N) per set of
# roundings; a few sets (store, one per level) with a factor 10 of margin give the bound
# (7.4e-11 measured at N = 4096 against a bound of ~3e-10).
U32 = 2.0 ** -24


def mixed_factor_bound(pts, p) -> float:
    A = O.dense_matrix(pts, p)
    off = np.linalg.norm(A - np.diag(np.diag(A)), "fro") / np.sqrt(len(pts))
    return 10 * U32 * off


# The FP32 factor copy used by the preconditioner solve rounds each record to FP32 and
# accumulates the sweep dot products in FP32: errors of order u32 relative to x (1.3 u32
# measured), bounded by 4 u32.
MIXED_SOLVE32_BOUND = 4 * U32
# F^{1/2} is not unique: it follows the factorization's own T through the Cholesky factors
# of X_RR, and at tol 1e-9 T moves with the FP32-rounded products in the ID inputs, its
# rounding amplified by cond(R11) ~ 1 / tol (2.8 u32 measured), bounded by 8 u32.
MIXED_SQRT_BOUND = 8 * U32


def _gpu_factor(rss, pts, p: O.Params, precision="fp64"):
    d = torch.tensor(pts, dtype=torch.float64, device="cuda")
    return rss.Factor(d, diag=p.diag, weight=p.weight, tol=p.tol, leaf_size=p.leaf_size, n_proxy=p.n_proxy,
                      proxy_radius=p.proxy_radius, root_lo=p.root_lo, root_side=p.root_side,
                      precision=precision, max_box=p.max_box)


def _compare(rss, name, pts, p, nrhs=1, precision="fp64", records=True, bound=None):
    """Skeleton sets of every box and the top set exactly; every record's T, X_RR, X_JR, G
    and J; F^{-1} b, F b element-wise and log|det F| (Section 3.3)."""
    say(f"[parity] case={name} N={len(pts)} tol={p.tol} leaf={p.leaf_size} precision={precision}")
    F = _gpu_factor(rss, pts, p, precision)
    R = O.factor(pts, p)
    depth, ntop = F.shape()
    assert depth == R.depth and F.info()["top_depth"] == R.top_depth
    compare_skeletons(F, R.skeletons)
    assert np.array_equal(F.top_set(), R.top)
    worst = 0.0
    if records:
        for r in R.records:
            worst = max(worst, compare_record(F, r.depth, r.box, dict(T=r.T, XRR=r.XRR, XJR=r.E @ r.XRR, G=r.G, J=r.J),
                                              p.tol))
    b = W.rhs(len(pts), seed=0, nrhs=nrhs)
    bt = torch.tensor(b, device="cuda")
    bound = vec_bound(p.tol) if bound is None else bound
    x = F.solve(bt).cpu().numpy()
    xr = O.solve(R, b)
    y = F.apply(bt).cpu().numpy()
    yr = O.apply(R, b)
    ex, ey = rel_maxdiff(x, xr), rel_maxdiff(y, yr)
    sg, ld = F.logdet()
    sr, lr = O.logdet(R)
    say(f"[parity] case={name} records={len(R.records)} worst_record_rel={worst:.2e} solve_maxrel={ex:.2e} "
        f"apply_maxrel={ey:.2e} logdet gpu={ld:.15e} oracle={lr:.15e} bound={bound:.1e}")
    np.testing.assert_allclose(x, xr, rtol=0, atol=bound * np.abs(xr).max())
    np.testing.assert_allclose(y, yr, rtol=0, atol=bound * np.abs(yr).max())
    assert sg == sr and abs(ld - lr) <= bound * max(1.0, abs(lr)) + 1e-14 * len(pts)
    info = F.info()
    F.close()
    return ex, ey, info


def test_parity_grid64_tol1e6(rss):
    n = 64
    _compare(rss, "grid64", W.grid_points(n), O.Params(**W.problem(n, 1e-6)))


@pytest.mark.parametrize("tol", [1e-3, 1e-9])
def test_parity_grid64_other_tolerances(rss, tol):
    n = 64
    _compare(rss, f"grid64_tol{tol}", W.grid_points(n), O.Params(**W.problem(n, tol)))


# Box-size limit: level-start box maxima without a limit are 16, 48, 93 (grid 64, leaf 16,
# tol 1e-6), 16, 64, 122 (tol 1e-9) and 49, 85, 97 (grid 100, leaf 64) at depths 4, 3, 2.
@pytest.mark.parametrize("name,n,leaf,tol,max_box,precision,top_depth", [
    ("grid64_leaf16_max40", 64, 16, 1e-6, 40, "fp64", 4),       # top: the 256 leaf boxes
    ("grid64_leaf16_max40_mixed", 64, 16, 1e-6, 40, "mixed", 4),
    ("grid64_leaf16_tol1e-9_max100", 64, 16, 1e-9, 100, "fp64", 3),
    ("grid64_leaf16_tol1e-9_max122", 64, 16, 1e-9, 122, "fp64", 2),   # at the limit: no stop
    ("grid100_max90", 100, 64, 1e-6, 90, "fp64", 3),
    # boxes of at most 9 points keep every DOF at the leaves: the top block is all 5184
    # DOFs (the inverse with 16 columns per workgroup, tall panels, 1024 boxes in the lists)
    ("grid72_leaf16_max20", 72, 16, 1e-6, 20, "fp64", 5),
])
def test_parity_box_limit_ends_the_recursion(rss, name, n, leaf, tol, max_box, precision, top_depth):
    p = O.Params(**W.problem(n, tol, leaf_size=leaf), max_box=max_box)
    assert O.factor(W.grid_points(n), p).top_depth == top_depth
    # mixed: the FP32 store rounds the ID inputs, so the records are not compared element
    # by element and F b, F^{-1} b take the mixed factor's bound (as for the full depth)
    mixed = precision == "mixed"
    _, _, info = _compare(rss, name, W.grid_points(n), p, nrhs=2, precision=precision, records=not mixed,
                          bound=mixed_factor_bound(W.grid_points(n), p) if mixed else None)
    assert info["top_depth"] == top_depth
    assert min(l["depth"] for l in info["levels"]) == top_depth


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


def test_parity_gauss_jordan_1024_threads_r_over_128(rss):
    # 64 x 64 grid, leaf 256: 16 boxes of 256 points at depth 2, |R| ~ 220 > 128, beyond the
    # register form of the 1024-thread inverse: X_RR goes through the workspace to the
    # pivoting Gauss-Jordan of the general form
    n = 64
    ex, ey, info = _compare(rss, "grid64_leaf256", W.grid_points(n), O.Params(**W.problem(n, 1e-6, leaf_size=256)))
    say(f"[parity] grid64_leaf256 shapes={info['shapes']}")
    assert "elim_inv_gauss_jordan_lds" in info["shapes"] and any(s.startswith("elim_inv_1024") for s in info["shapes"])


def mixed_density_points(seed: int = 4):
    """4 random points in every box of the 64 x 64 box grid plus 106 more in 12 boxes (of
    every colour): a uniform depth-6 tree with ~455 boxes per colour whose dense boxes have
    |B| = 110 and |R| ~ 80 (their O-ring boxes hold 4 points each, so the ID input has
    16 * 4 + 16 rows)."""
    rng = np.random.default_rng(seed)
    nb = 64
    cells = np.stack(np.meshgrid(np.arange(nb), np.arange(nb), indexing="xy"), axis=-1).reshape(-1, 2)
    pts = [(np.repeat(cells, 4, axis=0) + rng.uniform(0.05, 0.95, (4 * nb * nb, 2))) / nb]
    dense = [(9 + 7 * i, 11 + 5 * i) for i in range(6)] + [(40 + 2 * i, 8 + 9 * i) for i in range(6)]
    for bx, by in dense:
        pts.append((np.array([bx, by]) + rng.uniform(0.02, 0.98, (106, 2))) / nb)
    return np.concatenate(pts)


def test_parity_gauss_jordan_256_threads_many_boxes(rss):
    # ~455 boxes per colour take the 256-thread inverse; the dense boxes have |R| > 64,
    # beyond its register form, and nmax = 110 lets X_RR sit in LDS for the pivoting
    # Gauss-Jordan
    pts = mixed_density_points()
    p = O.Params(weight=1.0 / len(pts), tol=1e-6, leaf_size=110)
    # the 256-thread inverse for colours of 256..511 boxes, whatever the tuned table picks
    with plan_override("b2.inv_threads=256"):
        ex, ey, info = _compare(rss, "mixed_density_leaf110", pts, p, records=True)
    say(f"[parity] mixed_density shapes={info['shapes']}")
    assert "elim_inv_gauss_jordan_lds" in info["shapes"] and "elim_inv_256_xlds_zs" in info["shapes"]


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
    np.testing.assert_allclose(x, O.solve(R, b), rtol=0, atol=vec_bound(p.tol) * np.abs(x).max())
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
        # GMRES without the factor needs 6 iterations here (tests/test_oracle_pins.py pins
        # that), so these bounds fail unless F^{-1} preconditions
        assert rr <= 1e-12 and it <= (2 if prec == "fp64" else 3) and err <= 1e-10
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
    bound = mixed_factor_bound(pts, p)
    say(f"[parity] mixed factor: fp64-solve err={e64:.2e} (bound {bound:.1e}) fp32-solve err={e32:.2e} "
        f"({e32 / U32:.2f} u32)")
    assert e64 <= bound and e32 <= MIXED_SOLVE32_BOUND
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
    # FP64: F^{1/2} is not unique (it depends on the factorization's own T through the
    # Cholesky factors of X_RR), so it inherits the record bound (rounding in T amplified by
    # cond(R11) ~ 1 / tol; measured 2.4e-11 at tol 1e-6), unlike F and F^{-1}.
    ftol = record_bound(tol) if precision == "fp64" else MIXED_SQRT_BOUND
    for adj in (False, True):
        y = F.sqrt_apply(bt, adjoint=adj).cpu().numpy()
        yr = O.sqrt_apply(R, b, adjoint=adj)
        e = np.linalg.norm(y - yr) / np.linalg.norm(yr)
        say(f"[parity] sqrt adjoint={adj} rel={e:.2e} ({e / U32:.2f} u32)")
        assert e <= ftol
    # F = F^{1/2} (F^{1/2})^* on the device itself.  FP64: to rounding.  Mixed: the FP32
    # Schur products into blocks between boxes leave them symmetric only to u32 |w K|, and
    # C C^* uses W_i^* in place of V_i: E - G^T = ((A_JR - A_RJ^T) - (A_JS - A_SJ^T) T)
    # X_RR^{-1}, that asymmetry times (1 + |T|); measured 4.9e-13 at N = 4096, tol 1e-9.
    y2 = F.sqrt_apply(F.sqrt_apply(bt, adjoint=True)).cpu().numpy()
    yf = F.apply(bt).cpu().numpy()
    e2 = np.linalg.norm(y2 - yf) / np.linalg.norm(yf)
    say(f"[parity] sqrt C C^* vs F rel={e2:.2e} ({e2 / U32:.1f} u32)")
    assert e2 <= (1e-12 if precision == "fp64" else 1e-11)
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
