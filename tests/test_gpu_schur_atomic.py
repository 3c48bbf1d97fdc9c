"""The Schur update by no-return atomic adds (plan field schur_atomic) against the
load-subtract-store form.

Within one launch every store entry has exactly one writer (the 3 x 3 neighbourhoods of the
boxes of one colour are disjoint, Section 3.1 and the 3^d colouring), so adding -(X_JR G)_e
atomically rounds once, exactly as old - (X_JR G)_e: the two factorizations must be equal
bit for bit (F^{-1} b, F b, log|det F|, every skeleton set), in FP64 and in mixed precision
(FP32 store with FP64 self blocks, second pass included, and FP64 S x S products).
"""
import numpy as np
import pytest

from paper_1609_08130_amd import workloads as W
from tests.parity_util import plan_override, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ON = ",".join(f"b{b}.schur_atomic=1" for b in range(5))
OFF = ",".join(f"b{b}.schur_atomic=0" for b in range(5))


@pytest.fixture(scope="module")
def rss():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1609_08130_amd import rss as mod
    return mod


@pytest.mark.parametrize("n,precision,method", [(64, "fp64", "rs-s"), (100, "mixed", "rs-s"), (512, "mixed", "rs-s"),
                                                (64, "mixed", "rs-ws")])
def test_atomic_schur_equals_read_modify_write(rss, n, precision, method):
    say(f"[schur_atomic] N={n * n} precision={precision} method={method}")
    prm = W.problem(n, 1e-6)
    prm.pop("dim")
    pts = torch.tensor(W.grid_points(n), device="cuda")
    fs = {}
    for spec in (ON, OFF):
        with plan_override(spec):
            fs[spec] = rss.Factor(pts, precision=precision, method=method, **prm)
    Fa, Fr = fs[ON], fs[OFF]
    assert any(s.endswith("_atomic") for s in Fa.info()["shapes"])
    assert not any(s.endswith("_atomic") for s in Fr.info()["shapes"])
    b = torch.tensor(W.rhs(n * n, seed=0), device="cuda")
    assert torch.equal(Fa.solve(b), Fr.solve(b))
    assert torch.equal(Fa.apply(b), Fr.apply(b))
    assert Fa.logdet() == Fr.logdet()
    assert np.array_equal(Fa.top_set(), Fr.top_set())
    depth, _ = Fa.shape()
    for t in range(depth, 1, -1):
        for box in range(0, 4 ** t, max(1, 4 ** t // 64)):   # up to 64 boxes per level
            (Sa, Ra), (Sr, Rr) = Fa.box_sets(t, box), Fr.box_sets(t, box)
            assert np.array_equal(Sa, Sr) and np.array_equal(Ra, Rr), (t, box)
    ta = Fa.info()["phase_ms"]["schur"]
    tr = Fr.info()["phase_ms"]["schur"]
    say(f"[schur_atomic] N={n * n} {precision} {method}: bitwise equal; Schur {ta:.2f} ms atomic vs {tr:.2f} ms")
    Fa.close()
    Fr.close()
