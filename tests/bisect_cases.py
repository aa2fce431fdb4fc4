"""Adversarial symmetric tridiagonals (d, e) for the bisection tests.

Only matrices: no step of the eigensolver is computed here.
"""
import numpy as np

import sbr_inputs as si


def graded(n):
    # diagonal from 1 down to 1e-30, couplings the geometric mean of their
    # neighbours: eigenvalues spread over 30 orders of magnitude
    d = 10.0 ** (-30.0 * np.arange(n) / (n - 1))
    e = 0.5 * np.sqrt(d[:-1] * d[1:])
    return d, e


def glued_wilkinson(copies=10, m=21, glue=1e-14):
    # W_m^+ (diagonal |k - (m-1)/2|, unit couplings) has its largest
    # eigenvalues in pairs that agree to about 1e-13; gluing copies with a
    # tiny coupling makes clusters of 2 * copies nearly equal eigenvalues
    blk = np.abs(np.arange(m) - (m - 1) / 2.0)
    d = np.tile(blk, copies)
    e = np.ones(copies * m - 1)
    e[m - 1::m] = glue
    return d, e


def integer_zero_pivots(n=301):
    # small integer diagonal, couplings 0 or 1: many sub-blocks with exactly
    # representable (often integer) eigenvalues, so count points land on
    # eigenvalues and pivots come out exactly zero
    rng = np.random.default_rng(99)
    d = rng.integers(-2, 3, size=n).astype(np.float64)
    e = rng.integers(0, 2, size=n - 1).astype(np.float64)
    return d, e


def underflowing_pivots(n=200):
    # couplings near the underflow threshold next to O(1) couplings
    d = np.zeros(n)
    e = np.where(np.arange(n - 1) % 2 == 0, 1e-160, 1.0)
    return d, e


def toeplitz_odd(n=1001):
    # tridiag(1, 0, 1) with n odd has the eigenvalue 0: the pivots at x = 0
    # alternate between exact zeros and huge values
    return si.toeplitz_tridiagonal(n, 0.0, 1.0)


CASES = {"graded": graded(400), "glued_wilkinson": glued_wilkinson(), "integer_zero_pivots": integer_zero_pivots(),
         "underflowing_pivots": underflowing_pivots(), "toeplitz_odd": toeplitz_odd()}
