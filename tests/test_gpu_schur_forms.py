"""The two forms of the FP32 Schur products of a mixed factorization (plan field schur_form:
vector FMAs or matrix cores) with the S x S block of each step in FP64 products and the self
blocks A(B_a, B_a) in FP64 entries (Section 2.1, S_JJ = A_JJ - A_JR A_RR^{-1} A_RJ, over the
3x3 neighbourhood of Section 3.1).

Each form is within the mixed-precision bound of the FP64 oracle (F^{-1} b with the FP64
records), at one and three skeletonized levels, with an FP32 store (tol 1e-6) and with an
FP64 store (tol 1e-9); the two forms agree to FP32 rounding of the products at N = 512^2.
"""
import numpy as np
import pytest

from oracle import rss_oracle as O
from paper_1609_08130_amd import workloads as W
from tests.parity_util import plan_override, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def form_spec(v: int) -> str:
    return ",".join(f"b{b}.schur_form={v}" for b in range(5))


@pytest.fixture(scope="module")
def rss():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1609_08130_amd import rss as mod
    return mod


def _factor(rss, n, tol, form):
    prm = W.problem(n, tol)
    prm.pop("dim")
    pts = torch.tensor(W.grid_points(n), device="cuda")
    with plan_override(form_spec(form)):
        return rss.Factor(pts, precision="mixed", **prm)


@pytest.mark.parametrize("n,tol", [(64, 1e-6), (100, 1e-6), (64, 1e-9)])
def test_schur_forms_against_oracle(rss, n, tol):
    pts = W.grid_points(n)
    p = O.Params(**W.problem(n, tol))
    R = O.factor(pts, p)
    b = W.rhs(n * n, seed=0)
    xr = O.solve(R, b)
    # the mixed-precision bound of the parity tests: FP32 rounding of the entries between
    # different boxes (w K), a few sets of roundings, a factor 10 of margin
    A = O.dense_matrix(pts, p)
    bound = 10 * U32 * np.linalg.norm(A - np.diag(np.diag(A)), "fro") / np.sqrt(len(pts))
    xs = {}
    for form, tag in ((0, ""), (1, "_mfma")):
        say(f"[schur_forms] N={n * n} tol={tol} form={form}")
        F = _factor(rss, n, tol, form)
        shapes = F.info()["shapes"]
        f32 = [s for s in shapes if s.startswith("schur_f32")]
        assert f32 and all(s.endswith("_mfma") == (form == 1) for s in f32), shapes
        assert "schur_self_sxs_f64" in shapes
        x = F.solve(torch.tensor(b, device="cuda")).cpu().numpy()
        err = float(np.linalg.norm(x - xr) / np.linalg.norm(xr))
        say(f"[schur_forms] N={n * n} tol={tol} form={form}: solve err vs oracle {err:.2e} (bound {bound:.1e})")
        assert err <= bound
        F.close()


def test_schur_forms_agree_many_boxes(rss):
    # 512 x 512 grid: colours of up to 484 leaf boxes, several tile rows per box
    n = 512
    say(f"[schur_forms] N={n * n} forms 0 and 1")
    F0 = _factor(rss, n, 1e-6, 0)
    F1 = _factor(rss, n, 1e-6, 1)
    b = torch.tensor(W.rhs(n * n, seed=0), device="cuda")
    x0, x1 = F0.solve(b), F1.solve(b)
    e = float((x0 - x1).abs().max() / x1.abs().max())
    t0, t1 = F0.info()["phase_ms"]["schur"], F1.info()["phase_ms"]["schur"]
    say(f"[schur_forms] N={n * n}: forms 0 and 1 differ by {e:.2e}; Schur {t0:.2f} ms vs {t1:.2f} ms")
    assert e <= 16 * U32
    F0.close()
    F1.close()
