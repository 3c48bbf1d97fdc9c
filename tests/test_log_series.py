"""The logarithm used for FP32-stored matrix entries (CPU check of its accuracy).

Entries kept in FP32 take log x through x = m 2^e, m in [sqrt(1/2), sqrt(2)), and
log m = 2 atanh(t), t = (m - 1) / (m + 1), by the odd series of atanh to t^13.  The
claim checked here: relative error <= 1.3e-12 over the distances of any unit-square
workload, so FP32 rounding of w K is unchanged but for rare ties.
"""
import numpy as np


def _series_log(x):
    m, e = np.frexp(x)
    low = m < 0.70710678118654752
    m = np.where(low, 2.0 * m, m)
    e = np.where(low, e - 1, e)
    t = (m - 1.0) / (m + 1.0)
    t2 = t * t
    p = np.full_like(t, 1.0 / 13.0)
    for c in (1.0 / 11.0, 1.0 / 9.0, 1.0 / 7.0, 1.0 / 5.0, 1.0 / 3.0, 1.0):
        p = p * t2 + c
    return e * 0.69314718055994531 + 2.0 * t * p


def test_series_log_relative_error():
    rng = np.random.default_rng(0)
    x = np.exp(rng.uniform(np.log(1e-14), np.log(1e3), 1_000_000))
    x = np.concatenate([x, 1.0 + np.linspace(-1e-3, 1e-3, 2001), [0.5, 1.0, 2.0, 0.7071067811865476]])
    ref = np.log(x)
    got = _series_log(x)
    nz = ref != 0.0
    assert np.max(np.abs(got[nz] - ref[nz]) / np.abs(ref[nz])) <= 1.3e-12
    assert np.all(got[~nz] == 0.0)
    # FP32 entries w K = coef log r^2 round to the same value
    coef = -1.0 / (4.0 * np.pi * 1024 ** 2)
    assert np.mean((coef * got).astype(np.float32) != (coef * ref).astype(np.float32)) < 1e-4
