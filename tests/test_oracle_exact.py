"""The oracle's correctly rounded sums: C and Python agree, and both give
the FP64 number nearest the exact (rational) value."""

import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact as X


def _exact_fraction_dot(a, b):
    s = sum((Fraction(float(x)) * Fraction(float(y)) for x, y in zip(a, b)), Fraction(0))
    return float(s)  # Fraction -> float rounds to nearest, ties to even


@pytest.mark.parametrize("seed", range(6))
def test_dot_is_correctly_rounded(seed):
    rng = np.random.default_rng(seed)
    n = 200
    # ill-conditioned: huge cancellation across many scales
    a = rng.standard_normal(n) * np.exp(rng.uniform(-30, 30, n))
    b = rng.standard_normal(n)
    a = np.concatenate([a, -a[:50] * (1 + 1e-12)])
    b = np.concatenate([b, b[:50]])
    want = _exact_fraction_dot(a, b)
    assert X.build_c()
    assert X.exact_dot(a, b) == want
    assert X.py_exact_dot(a, b) == want


def test_sum_half_way_cases():
    # 1 + 2^-53 is exactly half-way between 1 and 1 + 2^-52: ties to even
    assert X.exact_sum([1.0, 2.0 ** -53]) == 1.0
    assert X.exact_sum([1.0, 2.0 ** -53, 2.0 ** -100]) == 1.0 + 2.0 ** -52
    assert X.exact_sum([1.0 + 2.0 ** -52, 2.0 ** -53]) == 1.0 + 2.0 ** -51
    assert X.exact_sum([]) == 0.0


def test_spmv_rows_match_python_and_fractions():
    rng = np.random.default_rng(7)
    m, n = 40, 30
    rp = np.concatenate([[0], np.cumsum(rng.integers(0, 9, m))]).astype(np.int64)
    nnz = int(rp[-1])
    col = rng.integers(0, n, nnz)
    val = rng.standard_normal(nnz) * np.exp(rng.uniform(-20, 20, nnz))
    x = rng.standard_normal(n)
    c = X.exact_spmv(rp, col, val, x)
    p = X.py_exact_spmv(rp, col, val, x)
    assert np.array_equal(c, p)
    for i in range(m):
        s, t = rp[i], rp[i + 1]
        assert c[i] == _exact_fraction_dot(val[s:t], x[col[s:t]])
    rs = X.exact_row_sums(rp, val)
    assert np.array_equal(rs, X.py_exact_row_sums(rp, val))
