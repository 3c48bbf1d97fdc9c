"""The exact Gram-sum scheme of k_gram_i8, checked on the CPU.

The kernel forms sum_k x_kp x_kq for FP32 entries x from per-column fixed point: with E_q
the largest binary exponent of column q over a slice (frexp convention) and U_q =
E_q - 34, X = x 2^-U_q is an integer below 2^34 whenever the column's exponents span at
most 10; it splits into five base-128 digits (four balanced by rint, in [-64, 64], and the
remainder, |d| <= 64); the products of digit pairs summed over at most 256 rows are exact
int32 values S_s (s = u + v), folded into two int64 words w0 = sum_{s<5} 128^s S_s and
w1 = sum_{s>=5} 128^(s-5) S_s, and the double-double TwoSum(w1 2^35, w0) scaled by
2^(U_p + U_q) equals the exact sum.  Here the same FP32 steps run in numpy and the result
is compared with exact rational arithmetic; the bounds the kernel relies on are asserted
on the way.  (The GPU kernel itself is compared with the double-double Gram kernel in
tests/test_gpu_gram_i8.py.)
"""
from fractions import Fraction

import numpy as np
import pytest

L = 5


def _digits(y):
    out = []
    y = y.astype(np.float32)
    for u in range(L):
        if u < L - 1:
            r = np.rint(y * np.float32(0.0078125)).astype(np.float32)
            d = y.astype(np.float64) - 128.0 * r.astype(np.float64)   # the kernel's fma: exact
            assert np.all(d == d.astype(np.float32))
            y = r
        else:
            d = y.astype(np.float64)
        assert np.all(np.abs(d) <= 64)
        out.append(d.astype(np.int64))
    return out


def _two_sum(a, b):
    s = a + b
    z = s - a
    return s, (a - (s - z)) + (b - z)


@pytest.mark.parametrize("seed", range(6))
def test_digit_gram_is_exact(seed):
    rng = np.random.default_rng(seed)
    checked = 0
    for _ in range(12):
        nro, n = int(rng.integers(1, 257)), int(rng.integers(1, 12))
        spread = int(rng.integers(0, 11))
        # mantissas in [1/2, 1) with random signs, exponents within `spread` of a random top
        mant = rng.uniform(0.5, 1.0, size=(nro, n)) * rng.choice([-1.0, 1.0], size=(nro, n))
        top = rng.integers(-40, 40)
        x = np.ldexp(mant, top - rng.integers(0, spread + 1, size=(nro, n))).astype(np.float32)
        x[rng.random(x.shape) < 0.05] = 0
        ex = np.frexp(x)[1]
        nz = x != 0
        emax = np.where(nz, ex, -100000).max(0)
        emin = np.where(nz, ex, 100000).min(0)
        if np.any((emax > -100000) & (emax - emin > 7 * L - 25)):
            continue   # the kernel sums such a slice in double-double (rounding to 1.0 can widen it)
        U = np.where(emax > -100000, emax - 7 * L + 1, 0)
        y = np.ldexp(x.astype(np.float64), -U[None, :])
        assert np.all(y == np.rint(y)) and np.all(np.abs(y) < 2.0 ** 34)
        D = _digits(y.astype(np.float32))
        S = [sum(D[u].T @ D[s - u] for u in range(L) if 0 <= s - u < L) for s in range(2 * L - 1)]
        assert max(int(np.abs(Si).max()) for Si in S) < 2 ** 23
        w0 = sum(S[s] * 128 ** s for s in range(5))
        w1 = sum(S[s] * 128 ** (s - 5) for s in range(5, 2 * L - 1))
        assert np.abs(w0).max() < 2 ** 53 and np.abs(w1).max() < 2 ** 53
        for p in range(n):
            for q in range(p, n):
                exact = sum(Fraction(float(x[k, p])) * Fraction(float(x[k, q])) for k in range(nro))
                hi, lo = _two_sum(np.ldexp(float(w1[p, q]), 35), float(w0[p, q]))
                e = int(U[p] + U[q])
                assert Fraction(np.ldexp(hi, e)) + Fraction(np.ldexp(lo, e)) == exact
        checked += 1
    assert checked > 0


def test_wide_spread_is_detected():
    # a column spanning 11 binary orders needs a sixth digit: the kernel's test rejects it
    x = np.array([[1.0], [2.0 ** -11]], dtype=np.float32)
    ex = np.frexp(x)[1]
    assert ex.max() - ex.min() > 7 * L - 25
