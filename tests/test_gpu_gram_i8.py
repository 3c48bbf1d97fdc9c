"""Exact Gram sums of the ID rows on the int8 matrix cores (k_gram_i8) in mixed precision.

The ID of a box (Section 3.1, eq. skelid: a pivoted QR of the rows M of the box's columns)
runs through the Gram matrix G = M^T M in double-double and its pivoted Cholesky.  With an
FP32 store, k_gram_i8 forms the sums of the FP32 rows exactly (base-128 digits per column on
v_mfma_i32_16x16x64_i8, proxy rows by TwoProd; a slice with too wide an exponent spread sums
in double-double), where k_gram accumulates them in compensated FP64.  Both are accurate to
double-double, so the factorization must come out the same.  Per case, with the plan field
gram_i8 forced on and off in every bucket (RSS_TUNE):
  * the skeleton / redundant sets of every box of every level and the top set are identical;
  * every record (T, X_RR, X_JR, G, J) agrees element-wise within 1e-12 of its largest entry;
  * F^{-1} b and F b agree within 1e-12, log|det F| within 1e-12;
  * F^{-1} b is within the mixed-precision bound of the FP64 oracle's (N <= 5000);
and the cases together take the 4- and 8-wave kernels, 256-row and shorter slices, and the
double-double form (boxes above 96 DOFs keep the double-double Gram kernel).
"""
import numpy as np
import pytest

from oracle import rss_oracle as O
from paper_1609_08130_amd import workloads as W
from tests.example1_util import power_norm
from tests.parity_util import plan_override, rel_maxdiff, say
from tests.test_gpu_parity import mixed_density_points, mixed_factor_bound

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ALL_I8 = ",".join(f"b{b}.gram_i8=1" for b in range(5))
NO_I8 = ",".join(f"b{b}.gram_i8=0" for b in range(5))
SEEN = set()


@pytest.fixture(scope="module")
def rss():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1609_08130_amd import rss as mod
    return mod


def _factor(rss, pts, p: O.Params, spec):
    with plan_override(spec):
        return rss.Factor(torch.tensor(pts, dtype=torch.float64, device="cuda"), diag=p.diag, weight=p.weight,
                          tol=p.tol, leaf_size=p.leaf_size, n_proxy=p.n_proxy, proxy_radius=p.proxy_radius,
                          root_lo=p.root_lo, root_side=p.root_side, precision="mixed",
                          method="rs-ws" if p.hybrid else "rs-s")


def _levels_and_boxes(F, weak, per_level=300):
    """Every box of every level with records (weak records reach depth 1), at most
    per_level boxes per level (a seeded sample)."""
    depth, _ = F.shape()
    rng = np.random.default_rng(0)
    for t in range(depth, 0 if weak else 1, -1):
        boxes = np.arange(4 ** t)
        if len(boxes) > per_level:
            boxes = np.sort(rng.choice(boxes, per_level, replace=False))
        for b in boxes:
            yield t, int(b)


CASES = {
    "grid64": lambda: (W.grid_points(64), O.Params(**W.problem(64, 1e-6))),
    "grid100_tol1e-5": lambda: (W.grid_points(100), O.Params(**W.problem(100, 1e-5))),
    "mixed_density_leaf110": lambda: (lambda pts: (pts, O.Params(weight=1.0 / len(pts), tol=1e-6, leaf_size=110)))(
        mixed_density_points()),
    "grid64_rsws": lambda: (W.grid_points(64), O.Params(**W.problem(64, 1e-6), hybrid=True)),
    "translated_root3": lambda: (np.column_stack([2.0 + 3.0 * np.random.default_rng(21).random(2500),
                                                  -1.0 + 3.0 * np.random.default_rng(22).random(2500)]),
                                 O.Params(weight=9.0 / 2500, tol=1e-6, leaf_size=32, root_lo=(2.0, -1.0),
                                          root_side=3.0)),
}


# boxes above 96 DOFs (here most levels) keep the double-double Gram kernel
WIDE_BOXES = {"mixed_density_leaf110"}
# plan fields set besides gram_i8: the many-box Gram form (256-row slices, one thread per
# column in the pivoted Cholesky) for one case, whatever the tuned table picks
EXTRA = {"grid100_tol1e-5": "," + ",".join(f"b{b}.gram_many=1" for b in range(5))}


@pytest.mark.parametrize("case", sorted(CASES))
def test_gram_i8_matches_double_double(rss, case):
    pts, p = CASES[case]()
    assert len(pts) == len(np.unique(pts, axis=0))
    say(f"[gram_i8] case={case} N={len(pts)} tol={p.tol} leaf={p.leaf_size} hybrid={p.hybrid}")
    extra = EXTRA.get(case, "")
    Fi = _factor(rss, pts, p, ALL_I8 + extra)
    Fd = _factor(rss, pts, p, NO_I8 + extra)
    shapes = Fi.info()["shapes"]
    assert not any(s.startswith("gram_i8") for s in Fd.info()["shapes"])
    if case not in WIDE_BOXES:
        assert any(s.startswith("gram_i8_w") for s in shapes), shapes
    SEEN.update(s for s in shapes if s.startswith("gram_i8"))
    assert Fi.shape() == Fd.shape()
    assert np.array_equal(Fi.top_set(), Fd.top_set())
    worst, nrec = 0.0, 0
    for weak in ((False, True) if p.hybrid else (False,)):
        for t, b in _levels_and_boxes(Fi, weak):
            Si, Ri = Fi.box_sets(t, b, weak=weak)
            Sd, Rd = Fd.box_sets(t, b, weak=weak)
            assert np.array_equal(Si, Sd) and np.array_equal(Ri, Rd), (t, b, weak)
            if len(Ri) == 0:
                continue
            gi, gd = Fi.box_record(t, b, weak=weak), Fd.box_record(t, b, weak=weak)
            assert np.array_equal(gi["J"], gd["J"])
            for key in ("T", "XRR", "XJR", "G"):
                e = rel_maxdiff(gi[key], gd[key])
                worst = max(worst, e)
                assert e <= 1e-12, (t, b, weak, key, e)
            nrec += 1
    b = W.rhs(len(pts), seed=0)
    bt = torch.tensor(b, device="cuda")
    xi, xd = Fi.solve(bt).cpu().numpy(), Fd.solve(bt).cpu().numpy()
    yi, yd = Fi.apply(bt).cpu().numpy(), Fd.apply(bt).cpu().numpy()
    li, ld = Fi.logdet()[1], Fd.logdet()[1]
    # against the FP64 oracle where its dense bound is affordable (N <= 5000)
    e_or, bound = 0.0, 1.0
    if len(pts) <= 5000:
        xr = O.solve(O.factor(pts, p), b)
        e_or = np.linalg.norm(xi - xr) / np.linalg.norm(xr)
        bound = mixed_factor_bound(pts, p)
    say(f"[gram_i8] case={case} records={nrec} worst_record_rel={worst:.2e} solve={rel_maxdiff(xi, xd):.2e} "
        f"apply={rel_maxdiff(yi, yd):.2e} logdet {li:.15e} vs {ld:.15e} oracle_err={e_or:.2e} (bound {bound:.1e}) "
        f"shapes={[s for s in shapes if s.startswith('gram')]}")
    assert rel_maxdiff(xi, xd) <= 1e-12 and rel_maxdiff(yi, yd) <= 1e-12
    assert abs(li - ld) <= 1e-12 * max(1.0, abs(ld))
    assert e_or <= bound
    Fi.close()
    Fd.close()


def test_gram_i8_accuracy_512(rss):
    # the 512 x 512 grid (~455 boxes per colour at the leaves): e_a <= 10 tol and GMRES within
    # the iteration bound of the mixed-precision factor
    n, tol = 512, 1e-6
    p = O.Params(**W.problem(n, tol))
    F = _factor(rss, W.grid_points(n), p, ALL_I8)
    gen = torch.Generator(device="cpu").manual_seed(1)
    x0 = torch.randn(n * n, generator=gen, dtype=torch.float64).cuda()
    tn = lambda t: float(torch.linalg.norm(t))
    e_a = power_norm(lambda v: F.matvec(v) - F.apply(v), x0, norm=tn) / power_norm(F.matvec, x0, norm=tn)
    b = torch.tensor(W.rhs(n * n, seed=0), device="cuda")
    _, it, rr = F.gmres(b, rtol=1e-10, maxit=30, use_fp32=True)
    shapes = F.info()["shapes"]
    SEEN.update(s for s in shapes if s.startswith("gram_i8"))
    say(f"[gram_i8] N={n * n} e_a={e_a:.2e} gmres iters={it} relres={rr:.2e} shapes={[s for s in shapes if s.startswith('gram')]}")
    assert e_a <= 10 * tol and it <= 3 and rr <= 1e-10
    F.close()


def test_gram_i8_forms_covered():
    # runs after the cases above (pytest keeps file order)
    if not SEEN:
        pytest.skip("no int8 Gram case ran")
    say(f"[gram_i8] forms seen: {sorted(SEEN)}")
    for form in ("gram_i8_w4_", "gram_i8_w8_", "gram_i8_wide"):
        assert any(s.startswith(form) for s in SEEN), (form, sorted(SEEN))
    # 256-row slices (many boxes, or few with a large workgroup count) and shorter slices
    # of few-box colours
    assert any(s.endswith("_rows256") for s in SEEN) and any(s.endswith(("_rows64", "_rows128")) for s in SEEN), SEEN
