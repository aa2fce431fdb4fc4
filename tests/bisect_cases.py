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


def identity(n=300):
    # one eigenvalue of multiplicity n: every count jumps from 0 to n at 1,
    # so every index shares the same grid cell
    return np.ones(n), np.zeros(n - 1)


def diagonal_only(n=257):
    # no couplings: the count is the number of d_i below x, each step a split
    rng = np.random.default_rng(5)
    return rng.standard_normal(n), np.zeros(n - 1)


def scaled(n, scale, seed):
    # a random tridiagonal scaled far from 1 in either direction (the Sturm
    # data are rescaled by a power of two, so the counts must not move)
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal(n), scale * rng.standard_normal(n - 1)


def pair_clusters(n=400):
    # 2 x 2 blocks [[c, t], [t, c]] with t = 1e-13 |c| glued by 1e-3: tight
    # pairs of eigenvalues c +- t spread over the spectrum
    rng = np.random.default_rng(17)
    c = np.repeat(rng.uniform(-1.0, 1.0, n // 2), 2)
    e = np.empty(n - 1)
    e[0::2] = 1e-13 * np.abs(c[0::2][: (n - 1 + 1) // 2])
    e[1::2] = 1e-3
    return c, e


CASES = {"graded": graded(400), "glued_wilkinson": glued_wilkinson(), "integer_zero_pivots": integer_zero_pivots(),
         "underflowing_pivots": underflowing_pivots(), "toeplitz_odd": toeplitz_odd(), "identity": identity(),
         "diagonal_only": diagonal_only(), "scaled_1e150": scaled(500, 1e150, 3), "scaled_1e-140": scaled(500, 1e-140, 4),
         "pair_clusters": pair_clusters()}
