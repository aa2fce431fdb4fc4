"""GPU component parity: the MFMA tile kernels, the panel QR (TSQR +
Householder reconstruction) and Sturm bisection, each through the C ABI,
against the CPU oracle / FP64 references on the same seeded inputs."""
import math

import numpy as np
import pytest
import torch

import sbr_inputs as si
from gpu_util import from_col, to_col

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sbr():
    import paper_1604_03703_amd as m
    assert torch.cuda.is_available()
    return m


@pytest.fixture(scope="module")
def plan(sbr):
    return sbr.Plan(0)


EPS64 = np.finfo(np.float64).eps
EPS32 = np.finfo(np.float32).eps


@pytest.mark.parametrize("prec", ["fp64", "fp32_mfma"])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (17, 5, 3), (64, 64, 16), (130, 70, 33), (200, 16, 300),
                                   (96, 128, 128)])
def test_gemm(sbr, prec, ta, tb, M, N, K):
    print("gemm", prec, ta, tb, M, N, K, flush=True)
    rng = np.random.default_rng(M * 1000 + N * 10 + K)
    A = rng.standard_normal((K, M) if ta else (M, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    C = rng.standard_normal((M, N))
    alpha, beta = 1.25, -0.5
    ref = alpha * ((A.T if ta else A) @ (B.T if tb else B)) + beta * C
    lda, ldb, ldc = A.shape[0] + 3, B.shape[0] + 1, M + 2
    Ad, Bd, Cd = to_col(A, lda), to_col(B, ldb), to_col(C, ldc)
    sbr.gemm(ta, tb, M, N, K, alpha, Ad, lda, Bd, ldb, beta, Cd, ldc, precision=prec)
    torch.cuda.synchronize()
    out = from_col(Cd, M)
    scale = np.abs(A).max() * np.abs(B).max() * K + np.abs(C).max()
    tol = (8 * K * EPS64 if prec == "fp64" else 4 * math.sqrt(K) * EPS32 * 4) * scale
    assert np.max(np.abs(out - ref)) <= tol
    # padding rows of C untouched
    assert np.all(Cd.cpu().numpy()[:, M:] == 0.0)


@pytest.mark.parametrize("prec", ["fp64", "fp32_mfma"])
@pytest.mark.parametrize("m,k", [(1, 1), (63, 8), (64, 16), (65, 64), (200, 128), (129, 3)])
def test_syr2k_lower(sbr, prec, m, k):
    print("syr2k", prec, m, k, flush=True)
    rng = np.random.default_rng(m * 7 + k)
    U = rng.standard_normal((m, k))
    V = rng.standard_normal((m, k))
    C = rng.standard_normal((m, m))
    ref = C + U @ V.T + V @ U.T
    Ud, Vd, Cd = to_col(U, m + 1), to_col(V, m), to_col(C, m + 5)
    sbr.syr2k_lower(m, k, Ud, m + 1, Vd, m, Cd, m + 5, precision=prec)
    torch.cuda.synchronize()
    out = from_col(Cd, m)
    low = np.tril_indices(m)
    up = np.triu_indices(m, 1)
    scale = 2 * k * np.abs(U).max() * np.abs(V).max() + np.abs(C).max()
    tol = (8 * k * EPS64 if prec == "fp64" else 8 * math.sqrt(k) * EPS32) * scale
    assert np.max(np.abs(out[low] - ref[low])) <= tol
    assert np.all(out[up] == C[up])           # strict upper triangle not written


@pytest.mark.parametrize("m,k", [(4096, 128), (4224, 64), (8192, 16)])
def test_syr2k_lower_direct_lds_path(sbr, m, k):
    # FP64, m a multiple of 128 with 128 x 128 tiles: with an even leading
    # dimension the operands go from memory straight into LDS, with an odd
    # one through registers; the two forms run the same products in the same
    # order, so C must come out the same bit for bit, and right
    print("syr2k direct lds", m, k, flush=True)
    rng = np.random.default_rng(m + 3 * k)
    U = rng.standard_normal((m, k))
    V = rng.standard_normal((m, k))
    C = rng.standard_normal((m, m))
    outs = []
    for ld in (m + 2, m + 3):
        Ud, Vd, Cd = to_col(U, ld), to_col(V, ld), to_col(C, m + 1)
        sbr.syr2k_lower(m, k, Ud, ld, Vd, ld, Cd, m + 1, precision="fp64")
        torch.cuda.synchronize()
        outs.append(from_col(Cd, m))
    assert np.array_equal(outs[0], outs[1])
    ref = C + U @ V.T + V @ U.T
    low = np.tril_indices(m)
    up = np.triu_indices(m, 1)
    scale = 2 * k * np.abs(U).max() * np.abs(V).max() + np.abs(C).max()
    assert np.max(np.abs(outs[0][low] - ref[low])) <= 8 * k * EPS64 * scale
    assert np.all(outs[0][up] == C[up])


@pytest.mark.parametrize("prec", ["fp64", "fp32_mfma"])
@pytest.mark.parametrize("m,k", [(17, 16), (1000, 64), (4100, 128)])
def test_syr2k_lower_buffer_path(sbr, prec, m, k):
    # U and V with one leading dimension and k a multiple of 16: the
    # buffer-load form the full-to-band uses (64 x 64 tiles below 512 lower
    # tiles, 128 x 128 tiles above: m = 4100 has 33 tile rows, the last
    # ragged); the result goes in by atomic adds, exactly one per element
    print("syr2k buffer", prec, m, k, flush=True)
    rng = np.random.default_rng(m * 11 + k)
    U = rng.standard_normal((m, k))
    V = rng.standard_normal((m, k))
    C = rng.standard_normal((m, m))
    ld = m + 3
    Ud, Vd, Cd = to_col(U, ld), to_col(V, ld), to_col(C, m + 1)
    sbr.syr2k_lower(m, k, Ud, ld, Vd, ld, Cd, m + 1, precision=prec)
    torch.cuda.synchronize()
    out = from_col(Cd, m)
    ref = C + U @ V.T + V @ U.T
    low = np.tril_indices(m)
    up = np.triu_indices(m, 1)
    scale = 2 * k * np.abs(U).max() * np.abs(V).max() + np.abs(C).max()
    tol = (8 * k * EPS64 if prec == "fp64" else 8 * math.sqrt(k) * EPS32) * scale
    assert np.max(np.abs(out[low] - ref[low])) <= tol
    assert np.all(out[up] == C[up])
    # a second call adds the same update again (the epilogue adds, never stores)
    sbr.syr2k_lower(m, k, Ud, ld, Vd, ld, Cd, m + 1, precision=prec)
    torch.cuda.synchronize()
    out2 = from_col(Cd, m)
    ref2 = ref + U @ V.T + V @ U.T
    assert np.max(np.abs(out2[low] - ref2[low])) <= 2 * tol


@pytest.mark.parametrize("prec", ["fp64", "fp32_mfma"])
@pytest.mark.parametrize("m,k", [(1, 1), (50, 16), (64, 64), (130, 128), (257, 32), (1000, 64)])
def test_symm_lower(sbr, prec, m, k):
    print("symm", prec, m, k, flush=True)
    rng = np.random.default_rng(m + 31 * k)
    A = si.gaussian_symmetric(m, rng)
    Aup = np.tril(A) + np.triu(rng.standard_normal((m, m)), 1)   # garbage above: must not be read
    Y = rng.standard_normal((m, k))
    ref = A @ Y
    Ad, Yd = to_col(Aup, m + 2), to_col(Y, m)
    Wd = to_col(np.zeros((m, k)), m + 1)
    sbr.symm_lower(m, k, Ad, m + 2, Yd, m, Wd, m + 1, precision=prec)
    torch.cuda.synchronize()
    out = from_col(Wd, m)
    scale = np.abs(A).max() * np.abs(Y).max() * m
    tol = (8 * m * EPS64 if prec == "fp64" else 8 * math.sqrt(m) * EPS32) * scale
    assert np.max(np.abs(out - ref)) <= tol


@pytest.mark.parametrize("m,b", [(16, 16), (40, 16), (100, 16), (200, 32), (300, 64), (257, 128),
                                 (1000, 64), (37, 8), (9, 4), (5, 2), (2000, 128)])
def test_panel_qr_tsqr_and_reconstruction(sbr, plan, oracle_mod, m, b):
    print("panel_qr", m, b, flush=True)
    rng = np.random.default_rng(m * 3 + b)
    P = rng.standard_normal((m, b))
    Pd = to_col(P)
    Q, R, U, T, S = sbr.panel_qr(Pd, b, plan)
    torch.cuda.synchronize()
    Q, U = from_col(Q, m), from_col(U, m)
    R, T = from_col(R, b), from_col(T, b)
    S = S.cpu().numpy()
    # rect-QR Ensure: P = Q R, orthonormal columns, R upper triangular
    assert np.max(np.abs(np.tril(R, -1))) == 0.0
    assert np.max(np.abs(Q @ R - P)) <= 50 * m * EPS64 * np.abs(P).max()
    assert np.max(np.abs(Q.T @ Q - np.eye(b))) <= 50 * m * EPS64
    # R is LAPACK's R up to the signs of its rows
    s = np.sign(np.diag(R))
    assert np.allclose(s[:, None] * R, oracle_mod.qr_r(P), atol=1e-12 * np.abs(P).max() * math.sqrt(m))
    # Corollary 3.7: U unit lower trapezoidal, (I - U T U^T)[:, :b] = Q S,
    # (I - U T U^T)^T P = [S R; 0], U^T U = T^{-1} + T^{-T}
    assert np.allclose(np.diag(U[:b]), 1.0) and np.max(np.abs(np.triu(U[:b], 1))) == 0.0
    assert np.all(np.abs(S) == 1.0)
    H = np.eye(m) - U @ T @ U.T
    assert np.max(np.abs(H[:, :b] - Q * S[None, :])) <= 200 * m * EPS64
    top = np.zeros((m, b))
    top[:b] = S[:, None] * R
    assert np.max(np.abs(H.T @ P - top)) <= 200 * m * EPS64 * np.abs(P).max()
    Ti = np.linalg.inv(T)
    assert np.max(np.abs(U.T @ U - Ti - Ti.T)) <= 1e-10 * max(1.0, np.abs(Ti).max())


@pytest.mark.parametrize("n", [1, 2, 3, 10, 1000, 4097])
def test_tridiag_eigvals_toeplitz(sbr, n):
    print("toeplitz", n, flush=True)
    d, e = si.toeplitz_tridiagonal(n, 0.0, 1.0)
    w = sbr.tridiag_eigvals(torch.from_numpy(d).cuda(), torch.from_numpy(e).cuda() if n > 1 else None)
    torch.cuda.synchronize()
    k = np.arange(1, n + 1)
    exact = np.sort(2.0 * np.cos(k * math.pi / (n + 1)))
    assert np.max(np.abs(w.cpu().numpy() - exact)) <= 1e-14 * 2 * max(1.0, math.log2(n + 1))


@pytest.mark.parametrize("n", [5, 300, 2048, 3001])
def test_tridiag_eigvals_vs_oracle(sbr, oracle_mod, n):
    print("tridiag", n, flush=True)
    rng = np.random.default_rng(n)
    d = rng.standard_normal(n)
    e = rng.standard_normal(n - 1)
    e[::17] = 0.0                  # decoupled blocks
    w = sbr.tridiag_eigvals(torch.from_numpy(d).cuda(), torch.from_numpy(e).cuda())
    torch.cuda.synchronize()
    ref = oracle_mod.tridiag_eigvals(d, e)
    assert np.max(np.abs(w.cpu().numpy() - ref)) <= 4 * EPS64 * np.max(np.abs(ref))
