"""Pins for the CPU oracle (Householder tridiagonalisation + Sturm bisection).

Each test ties the oracle to something other than itself: a closed form, a
prescribed spectrum, an invariant of orthogonal similarity, brute-force
cyclic Jacobi (Golub & Van Loan, Section 8.5) or LAPACK via numpy / scipy.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import sbr_inputs as si


def jacobi_eigvals(A, sweeps=60):
    """Cyclic Jacobi: rotate every off-diagonal pair to zero until converged."""
    A = np.array(A, dtype=np.float64, copy=True)
    n = A.shape[0]
    fro = math.sqrt(float(np.sum(A * A))) or 1.0
    for _ in range(sweeps):
        off = math.sqrt(float(np.sum(np.tril(A, -1) ** 2)))
        if off <= 1e-17 * fro:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                if abs(A[p, q]) <= 1e-300:
                    continue
                theta = (A[q, q] - A[p, p]) / (2.0 * A[p, q])
                if abs(theta) > 1e150:
                    t = 0.5 / theta
                else:
                    t = (1.0 if theta >= 0 else -1.0) / (abs(theta) + math.sqrt(1.0 + theta * theta))
                c = 1.0 / math.sqrt(1.0 + t * t)
                s = t * c
                rp, rq = A[p, :].copy(), A[q, :].copy()
                A[p, :], A[q, :] = c * rp - s * rq, s * rp + c * rq
                cp, cq = A[:, p].copy(), A[:, q].copy()
                A[:, p], A[:, q] = c * cp - s * cq, s * cp + c * cq
    return np.sort(np.diag(A))


def test_jacobi_reference_itself_on_diagonal_and_2x2():
    # The brute-force reference must itself be right on cases solvable by hand.
    assert np.allclose(jacobi_eigvals(np.diag([3.0, -1.0, 2.0])), [-1.0, 2.0, 3.0])
    a, b, c = 2.0, 0.5, -1.0
    disc = math.sqrt(((a - c) / 2) ** 2 + b * b)
    exact = sorted([(a + c) / 2 - disc, (a + c) / 2 + disc])
    assert np.allclose(jacobi_eigvals(np.array([[a, b], [b, c]])), exact, atol=1e-15)


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 500, 1000])
@pytest.mark.parametrize("alpha,beta", [(0.0, 1.0), (1.5, -0.25), (-3.0, 2.0)])
def test_bisection_toeplitz_closed_form(oracle_mod, n, alpha, beta):
    d, e = si.toeplitz_tridiagonal(n, alpha, beta)
    w = oracle_mod.tridiag_eigvals(d, e)
    k = np.arange(1, n + 1)
    exact = np.sort(alpha + 2.0 * beta * np.cos(k * math.pi / (n + 1)))
    scale = abs(alpha) + 2 * abs(beta)
    assert np.max(np.abs(w - exact)) <= 4e-15 * scale * max(1.0, math.log2(n + 1))
    assert np.all(np.diff(w) >= 0)


@pytest.mark.parametrize("n", [4, 9, 16])
def test_sturm_count_matches_jacobi(oracle_mod, n):
    rng = np.random.default_rng(100 + n)
    d = rng.standard_normal(n)
    e = rng.standard_normal(n - 1)
    lam = jacobi_eigvals(si.dense_from_tridiagonal(d, e))
    for x in rng.uniform(lam[0] - 1, lam[-1] + 1, size=40):
        if np.min(np.abs(lam - x)) < 1e-9:
            continue
        assert oracle_mod.sturm_count(d, e, x) == int(np.sum(lam < x))


@pytest.mark.parametrize("n", [2, 5, 11, 16])
def test_eigvalsh_matches_jacobi(oracle_mod, n):
    A = si.gaussian_symmetric(n, np.random.default_rng(7 * n))
    lam = jacobi_eigvals(A)
    w = oracle_mod.eigvalsh(A)
    assert np.max(np.abs(w - lam)) <= 1e-13 * np.max(np.abs(lam))


@pytest.mark.parametrize("n", [50, 300])
@pytest.mark.parametrize("kind", ["geometric", "clustered", "uniform"])
def test_eigvalsh_prescribed_spectrum(oracle_mod, n, kind):
    rng = np.random.default_rng(n)
    lam = {"geometric": si.geometric_spectrum, "clustered": si.clustered_spectrum,
           "uniform": si.uniform_spectrum}[kind](n, rng)
    A = si.spectrum_matrix(lam, rng)
    w = oracle_mod.eigvalsh(A)
    assert np.max(np.abs(w - np.sort(lam))) <= 1e-13 * np.max(np.abs(lam))


@pytest.mark.parametrize("n", [3, 40, 257])
def test_tridiagonalize_invariants(oracle_mod, n):
    A = si.gaussian_symmetric(n, np.random.default_rng(n + 1))
    d, e = oracle_mod.tridiagonalize(A)
    fro2 = float(np.sum(A * A))
    assert abs(d.sum() - np.trace(A)) <= 1e-13 * math.sqrt(fro2) * n
    assert abs(np.sum(d * d) + 2 * np.sum(e * e) - fro2) <= 1e-13 * fro2
    # and the tridiagonal has the spectrum of A (independent route: LAPACK)
    w = scipy.linalg.eigvalsh_tridiagonal(d, e) if n > 1 else d
    assert np.max(np.abs(np.sort(w) - np.linalg.eigvalsh(A))) <= 1e-13 * math.sqrt(fro2)


@pytest.mark.parametrize("n", [1, 2, 3, 10, 128])
def test_eigvalsh_against_lapack(oracle_mod, n):
    A = si.gaussian_symmetric(n, np.random.default_rng(3 * n + 2))
    w = oracle_mod.eigvalsh(A)
    ref = np.linalg.eigvalsh(A)
    assert np.max(np.abs(w - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_bisection_against_scipy_tridiagonal(oracle_mod):
    rng = np.random.default_rng(5)
    d = rng.standard_normal(777)
    e = rng.standard_normal(776)
    w = oracle_mod.tridiag_eigvals(d, e)
    ref = scipy.linalg.eigvalsh_tridiagonal(d, e)
    assert np.max(np.abs(w - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_edge_cases(oracle_mod):
    assert np.allclose(oracle_mod.eigvalsh(np.array([[4.0]])), [4.0])
    Z = np.zeros((6, 6))
    assert np.max(np.abs(oracle_mod.eigvalsh(Z))) <= 1e-300
    I5 = 2.5 * np.eye(5)
    assert np.allclose(oracle_mod.eigvalsh(I5), 2.5, atol=1e-15)
    D = np.diag([5.0, -2.0, 0.0, 7.0])            # already reduced: no reflector applied
    assert np.allclose(oracle_mod.eigvalsh(D), [-2.0, 0.0, 5.0, 7.0], atol=1e-15)
    d, e = si.toeplitz_tridiagonal(30, 1.0, 0.5)  # already tridiagonal
    T = si.dense_from_tridiagonal(d, e)
    d2, e2 = oracle_mod.tridiagonalize(T)
    assert np.allclose(d2, d) and np.allclose(np.abs(e2), np.abs(e))
    # decoupled blocks (an exactly zero off-diagonal)
    d = np.array([1.0, 2.0, 3.0, 4.0])
    e = np.array([0.5, 0.0, 0.25])
    assert np.allclose(oracle_mod.tridiag_eigvals(d, e),
                       scipy.linalg.eigvalsh_tridiagonal(d, e), atol=1e-15)


def test_semicircle_range(oracle_mod):
    n = 400
    A = si.gaussian_symmetric(n, si.make_rng(si.CFG_SMALL, 0))
    w = oracle_mod.eigvalsh(A)
    edge = math.sqrt(2 * n)
    assert -1.15 * edge < w[0] < -0.85 * edge and 0.85 * edge < w[-1] < 1.15 * edge


def test_oracle_bisection_on_adversarial_tridiagonals(oracle_mod):
    # graded, glued Wilkinson, exact zero pivots, underflowing couplings:
    # the oracle's bisection against LAPACK's tridiagonal eigensolver
    from scipy.linalg import eigvalsh_tridiagonal

    from bisect_cases import CASES
    eps = np.finfo(np.float64).eps
    for name, (d, e) in CASES.items():
        ref = oracle_mod.tridiag_eigvals(d, e)
        lap = eigvalsh_tridiagonal(d, e)
        nrm = max(float(np.max(np.abs(lap))), 1e-300)
        assert np.all(np.diff(ref) >= 0.0), name
        assert np.max(np.abs(ref - lap)) <= 8 * len(d) * eps * nrm, name


@pytest.mark.slow
@pytest.mark.parametrize("name", ["n16384", "n32768"])
def test_stored_oracle_eigenvalues(name):
    # the stored eigenvalues of the full-size Gaussian inputs: the generator
    # still produces the matrix they were computed on (SHA-256 of its bytes),
    # and they satisfy what the spectrum of that matrix must: sum = trace,
    # sum of squares = ||A||_F^2, ascending, inside the Gershgorin interval
    import golden_io
    rec, w = golden_io.load(name)
    cfg = {"n16384": si.CFG_FP32, "n32768": si.CFG_LARGE}[name]
    A, _ = si.workload(cfg, 0)
    n = A.shape[0]
    assert w.shape == (n,)
    assert golden_io.matrix_sha256(A) == rec["matrix_sha256"]
    nrm = float(np.max(np.abs(w)))
    eps = np.finfo(np.float64).eps
    assert np.all(np.diff(w) >= 0.0)
    assert abs(float(w.sum()) - float(np.trace(A))) <= n * eps * nrm * 100
    flat = A.reshape(-1)
    fro2 = float(np.dot(flat, flat))
    assert abs(float(np.dot(w, w)) - fro2) <= n * eps * fro2 * 10
    radius = float(np.max(np.sum(np.abs(A), axis=1)))
    assert nrm <= radius
    # Wigner semicircle: the spectrum of (G + G^T)/2 fills about [-sqrt(2n), sqrt(2n)]
    assert 0.97 * math.sqrt(2 * n) <= nrm <= 1.03 * math.sqrt(2 * n)
