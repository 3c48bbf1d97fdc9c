"""GPU parity on the 512 x 512 grid against the oracle's stored results.

Two cases whose colours hold hundreds to thousands of boxes, so that every launch shape the
factorization and the sweeps switch to with the box count of a colour runs (rss_info lists
the shapes taken):
  * leaf 16: 16384 leaves, ~1820 boxes per colour at depth 7, ~455 at depth 6;
  * leaf 64: the 512 x 512 workload itself, ~455 boxes per colour at its leaves.
The oracle's outputs (tests/golden/make_oracle_fixtures.py, which calls only the oracle)
are compared with the GPU's: the skeleton and redundant sets of every box of every level
and the top set exactly (Section 3.1 eq. skelid, Algorithm 1), F^{-1} b and F b element-wise
and log|det F| (Section 3.3), and the full records of one interior box of the last colour
per level (T, X_RR, X_JR, G, J; Section 3.1 eqs. zab, skelop).
"""
import fnmatch

import numpy as np
import pytest

from paper_1609_08130_amd import workloads as W
from tests.golden.make_oracle_fixtures import CASES, load
from tests.parity_util import compare_record, compare_skeletons, plan_override, rel_maxdiff, say, vec_bound

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rss():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1609_08130_amd import rss as mod
    return mod


@pytest.mark.parametrize("name,shapes", [
    # leaf 16: >= 1024 boxes per colour (4 tiles per elimination workgroup, 64-thread pivoted
    # Cholesky with 16 LDS rows, 256-thread inverse) and the few-box shapes of the upper levels
    ("grid512_leaf16_tol1e-6", ["elim_rows_w*_tpw4", "elim_inv_256*", "elim_inv_1024*", "pchol_64x1_kc16",
                                "solve_fwd_256_f64", "solve_fwd_1024_f64", "gram_reduce"]),
    # leaf 64: 455 boxes per colour at the leaves (the tuned plans of 256..511 boxes: four
    # 32-line tiles per elimination workgroup, 1024-thread inverse, 256-thread sweeps)
    ("grid512_leaf64_tol1e-6", ["elim_rows_w32_tpw4", "elim_inv_1024*", "solve_fwd_256_f64", "solve_bwd_256_f64"]),
    # the same with two 16-line tiles per workgroup (an earlier tuned plan of those colours)
    ("grid512_leaf64_tol1e-6@b2.elim_tpw=2,b2.elim_tw=16", ["elim_rows_w16_tpw2", "elim_inv_1024*"]),
    # the same with the former plans of those colours forced (256-thread inverse, one tile per
    # workgroup, 16-line tiles), so both variants stay checked
    ("grid512_leaf64_tol1e-6@b2.inv_threads=256,b2.elim_tpw=1,b2.elim_tw=16",
     ["elim_rows_w16_tpw1", "elim_inv_256*", "solve_fwd_256_f64"]),
])
def test_parity_512_grid_against_stored_oracle(rss, name, shapes):
    name, _, spec = name.partition("@")
    with plan_override(spec):
        _run_case(rss, name, shapes)


def _run_case(rss, name, shapes):
    c = CASES[name]
    n = c["n"]
    ref = load(name)
    say(f"[parity-large] case={name} N={n * n} leaf={c['leaf']} tol={c['tol']} "
        f"(oracle factor {ref['meta']['oracle_factor_seconds']} s, stored)")
    prm = W.problem(n, c["tol"], leaf_size=c["leaf"])
    prm.pop("dim")
    F = rss.Factor(torch.tensor(W.grid_points(n), device="cuda"), precision="fp64", **prm)
    depth, ntop = F.shape()
    assert depth == int(ref["depth"])
    nsk = compare_skeletons(F, ref["skeletons"])
    assert np.array_equal(F.top_set(), ref["top"].astype(np.int64))
    worst = 0.0
    for r in ref["records"]:
        worst = max(worst, compare_record(F, r["depth"], r["box"], r, c["tol"]))
    b = torch.tensor(W.rhs(n * n, seed=0), device="cuda")
    x = F.solve(b).cpu().numpy()
    y = F.apply(b).cpu().numpy()
    sg, ld = F.logdet()
    ex, ey = rel_maxdiff(x, ref["x"]), rel_maxdiff(y, ref["y"])
    info = F.info()
    say(f"[parity-large] case={name} boxes={nsk} records_checked={len(ref['records'])} worst_record_rel={worst:.2e} "
        f"solve_maxrel={ex:.2e} apply_maxrel={ey:.2e} logdet gpu={ld:.15e} oracle={ref['logdet'][1]:.15e}")
    say(f"[parity-large] case={name} shapes={info['shapes']}")
    bound = vec_bound(c["tol"])
    np.testing.assert_allclose(x, ref["x"], rtol=0, atol=bound * np.abs(ref["x"]).max())
    np.testing.assert_allclose(y, ref["y"], rtol=0, atol=bound * np.abs(ref["y"]).max())
    assert sg == ref["logdet"][0] and abs(ld - ref["logdet"][1]) <= bound * max(1.0, abs(ref["logdet"][1])) + 1e-14 * n * n
    # glob patterns (a pattern without "*" matches as a prefix)
    missing = [s for s in shapes if not any(fnmatch.fnmatch(t, s if "*" in s else s + "*") for t in info["shapes"])]
    assert not missing, (missing, info["shapes"])
    F.close()
