"""GPU: rss_gmres_noalloc, the GMRES entry point for callers that cannot allocate device
memory, against rss_gmres on the same factors: identical iterates (the same arithmetic in
the same order), on two calls in a row with the second on a smaller problem (the library's
work array keeps the first call's contents), a rejected size that writes nothing, and no
change of the device's free memory across a call."""
import ctypes

import numpy as np
import pytest

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


def _factor(rss, n, precision):
    prm = W.problem(n, 1e-6)
    prm.pop("dim")
    return rss.Factor(torch.tensor(W.grid_points(n), device="cuda"), precision=precision, **prm)


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_matches_allocating_gmres(rss, order):
    for n, precision, restart in ((96, "mixed", 8), (40, "fp64", 5)):
        say(f"[noalloc] N={n * n} {precision} restart={restart}")
        F = _factor(rss, n, precision)
        b = torch.tensor(W.rhs(n * n, seed=3), device="cuda")
        use32 = precision == "mixed"
        x_ref, it_ref, rr_ref = F.gmres(b, rtol=1e-12, maxit=20, restart=restart, use_fp32=use32)
        x = torch.full_like(b, float("nan"))
        st, it, rr = F.gmres_noalloc(b, x, rtol=1e-12, maxit=20, restart=restart, use_fp32=use32)
        torch.cuda.synchronize()
        say(f"[noalloc] N={n * n}: status={st} iters={it} (ref {it_ref}) relres={rr:.2e} (ref {rr_ref:.2e})")
        assert st == 0 and it == it_ref and rr == rr_ref
        assert torch.equal(x, x_ref)
        # a budget of one iteration: RSS_E_NOCONV from both, with the same iterate
        x1_ref, _, rr1_ref = F.gmres(b, rtol=1e-14, maxit=1, restart=restart, use_fp32=use32, raise_on_noconv=False)
        x1 = torch.empty_like(b)
        st1, it1, rr1 = F.gmres_noalloc(b, x1, rtol=1e-14, maxit=1, restart=restart, use_fp32=use32)
        assert st1 == 6 and it1 == 1 and rr1 == rr1_ref and torch.equal(x1, x1_ref)
        F.close()


def test_noalloc_rejects_oversize_and_allocates_nothing(rss):
    n = 512
    F = _factor(rss, n, "fp64")
    b = torch.tensor(W.rhs(n * n, seed=0), device="cuda")
    x = torch.full_like(b, 7.0)
    lib = rss.lib()
    it, rr = ctypes.c_int32(-1), ctypes.c_double(-1.0)
    # (2 * 64 + 3) * 262144 + 1024 doubles exceed the 256 MiB array
    st = lib.rss_gmres_noalloc(F._h, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()), 1e-10, 10, 64,
                               0, None, ctypes.byref(it), ctypes.byref(rr))
    torch.cuda.synchronize()
    assert st == 1 and "noalloc" in lib.rss_last_error().decode()
    assert bool((x == 7.0).all()) and it.value == -1
    # a call that fits leaves the device's free memory unchanged
    rss.trim()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    st2, it2, rr2 = F.gmres_noalloc(b, x, rtol=1e-10, maxit=10, restart=14)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    say(f"[noalloc] N={n * n}: status={st2} iters={it2} relres={rr2:.2e} free memory {free0} -> {free1}")
    assert st2 == 0 and rr2 <= 1e-10 and free1 == free0
    F.close()
