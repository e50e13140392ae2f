"""Pins for the oracle's SpMV (Sec. 3.1 definition y = A x).

The oracle is checked against things other than itself: a dense brute-force
product, exact rational sums, and matrices whose product is known in closed
form (identity, permutation, all-ones row, empty rows).
"""
from fractions import Fraction

import numpy as np
import pytest

import graphgen
import oracle


def _dense(row_ptr, col, vals, n_cols):
    n = len(row_ptr) - 1
    A = np.zeros((n, n_cols))
    for r in range(n):
        for k in range(row_ptr[r], row_ptr[r + 1]):
            A[r, col[k]] += vals[k]
    return A


@pytest.mark.parametrize("shape,density,empty,seed", [
    ((1, 1), 1.0, 0.0, 0), ((7, 5), 0.5, 0.0, 1), ((5, 9), 0.3, 0.3, 2),
    ((40, 40), 0.1, 0.2, 3), ((64, 17), 0.6, 0.1, 4), ((33, 64), 0.05, 0.5, 5)])
def test_spmv_dense_bruteforce(shape, density, empty, seed):
    n, nc = shape
    rp, col, vals = graphgen.random_csr(n, nc, density, seed, empty_frac=empty)
    x = np.random.default_rng(seed + 100).uniform(-1, 1, nc)
    y = oracle.spmv(rp, col, vals, x)
    A = _dense(rp, col, vals, nc)
    ref = A @ x
    scale = np.abs(A) @ np.abs(x)
    assert y.shape == (n,)
    assert np.all(np.abs(y - ref) <= 1e-14 * scale + 1e-300)
    # rows with no nonzero are exactly zero
    empty_rows = np.diff(rp) == 0
    assert np.all(y[empty_rows] == 0.0)
    assert np.allclose(oracle.abs_spmv(rp, col, vals, x), scale, rtol=1e-14, atol=0)


def test_spmv_exact_rational():
    # Every product and sum checked against exact rational arithmetic: the
    # long-double result rounded to double is within 1 ulp of the exact value
    # (plus the long-double summation bound).
    rp, col, vals = graphgen.random_csr(12, 30, 0.7, 11, empty_frac=0.2)
    x = np.random.default_rng(12).uniform(-1, 1, 30)
    y = oracle.spmv(rp, col, vals, x)
    for r in range(12):
        terms = [Fraction(float(vals[k])) * Fraction(float(x[col[k]]))
                 for k in range(rp[r], rp[r + 1])]
        exact = sum(terms, Fraction(0))
        abs_sum = sum((abs(t) for t in terms), Fraction(0))
        bound = abs(exact) * Fraction(2) ** -52 + abs_sum * len(terms) * Fraction(2) ** -62
        assert abs(Fraction(float(y[r])) - exact) <= bound


def test_spmv_identity_permutation_ones():
    n = 50
    x = np.random.default_rng(3).uniform(-1, 1, n)
    rp = np.arange(n + 1, dtype=np.int32)
    eye = oracle.spmv(rp, np.arange(n, dtype=np.int32), np.ones(n), x)
    assert np.array_equal(eye, x)
    perm = np.random.default_rng(4).permutation(n).astype(np.int32)
    assert np.array_equal(oracle.spmv(rp, perm, np.ones(n), x), x[perm])
    # one all-ones row followed by empty rows: y[0] = sum(x) (exact, checked
    # with rationals), the rest 0
    rp1 = np.array([0, n] + [n] * 3, np.int32)
    y = oracle.spmv(rp1, np.arange(n, dtype=np.int32), np.ones(n), x)
    exact = sum((Fraction(float(v)) for v in x), Fraction(0))
    assert abs(Fraction(float(y[0])) - exact) <= abs(exact) * Fraction(2) ** -52 + Fraction(
        2) ** -100
    assert np.all(y[1:] == 0.0)


def test_spmv_no_nonzeros():
    rp = np.zeros(6, np.int32)
    y = oracle.spmv(rp, np.zeros(0, np.int32), np.zeros(0), np.ones(4))
    assert np.array_equal(y, np.zeros(5))
