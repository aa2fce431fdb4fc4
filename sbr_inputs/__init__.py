"""Seeded synthetic inputs for the SBR symmetric eigensolver.

This module is shared by the CPU oracle's tests, the GPU tests and the
benchmark.  It only draws random numbers and assembles test matrices from
them; it contains none of the eigensolver's own arithmetic (no band
reduction, no bulge chasing, no Sturm counts).

Every generator takes a ``numpy.random.Generator``; ``make_rng(cfg, inp)``
returns the canonical one for workload ``cfg`` (0..4: CFG_SMALL, CFG_MEDIUM,
CFG_LARGE, CFG_FP32, CFG_BATCH below) and input variant ``inp`` (0 = first
input of that workload, 1 = second).

Recipes:

* ``gaussian_symmetric``  A = (G + G^T)/2, G_ij ~ N(0, 1).
* ``spectrum_matrix``     A = Q diag(lam) Q^T, Q = H_1 ... H_64 with
                          H_i = I - 2 v_i v_i^T / |v_i|^2, v_i ~ N(0, I).
* ``geometric_spectrum``  |lam_i| = 10^(-8 (i-1)/(n-1)), random signs.
* ``clustered_spectrum``  64 clusters, centres ~ U[-1, 1], each value
                          centre + 1e-10 * U[-1, 1].
* ``uniform_spectrum``    lam_i ~ U[-1, 1].
* ``scf_like``            M_ij ~ N(0, 0.1^2) exp(-|i-j|/20), A = (M+M^T)/2,
                          diagonal overwritten by sorted U[-20, 5].
* ``batch_sizes``         n_m ~ U{32, ..., 512}.
"""
from __future__ import annotations

import numpy as np

SEED_PREFIX = (1604, 3703)

# Workload indices.
CFG_SMALL = 0        # n = 256, b0 = 16
CFG_MEDIUM = 1       # n = 8192, b0 = 64
CFG_LARGE = 2        # n = 32768, b0 = 128
CFG_FP32 = 3         # n = 16384, FP32-MFMA form
CFG_BATCH = 4        # 4096 SCF-like matrices, n in [32, 512]


def make_rng(cfg: int, inp: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([*SEED_PREFIX, int(cfg), int(inp)]))


def _symmetrize_inplace(G: np.ndarray, block: int = 2048) -> np.ndarray:
    """G <- (G + G^T)/2 blockwise (never through an aliased ``G += G.T``)."""
    n = G.shape[0]
    for i0 in range(0, n, block):
        i1 = min(n, i0 + block)
        for j0 in range(0, i0 + 1, block):
            j1 = min(n, j0 + block)
            if j0 == i0:
                t = 0.5 * (G[i0:i1, j0:j1] + G[j0:j1, i0:i1].T)
                G[i0:i1, j0:j1] = t
            else:
                t = 0.5 * (G[i0:i1, j0:j1] + G[j0:j1, i0:i1].T)
                G[i0:i1, j0:j1] = t
                G[j0:j1, i0:i1] = t.T
    return G


def gaussian_symmetric(n: int, rng: np.random.Generator) -> np.ndarray:
    """(G + G^T)/2 with G_ij i.i.d. N(0, 1), float64, symmetric (any layout)."""
    G = np.empty((n, n), dtype=np.float64)
    rows = max(1, (1 << 24) // max(n, 1))
    for r0 in range(0, n, rows):
        r1 = min(n, r0 + rows)
        G[r0:r1] = rng.standard_normal((r1 - r0, n))
    return _symmetrize_inplace(G)


def householder_factor(n: int, rng: np.random.Generator, count: int = 64):
    """Gaussian reflector vectors v_i (columns of Y, unit length) and the
    triangular factor Tq with H_1 ... H_count = I - Y Tq Y^T (H_i = I - 2 y_i y_i^T)."""
    k = min(count, n)
    Y = rng.standard_normal((n, k))
    Y /= np.linalg.norm(Y, axis=0, keepdims=True)
    Tq = np.zeros((k, k))
    for i in range(k):
        Tq[i, i] = 2.0
        if i:
            Tq[:i, i] = -2.0 * (Tq[:i, :i] @ (Y[:, :i].T @ Y[:, i]))
    return Y, Tq


def spectrum_matrix(lam: np.ndarray, rng: np.random.Generator, count: int = 64) -> np.ndarray:
    """Q diag(lam) Q^T with Q the product of ``count`` Gaussian Householder reflectors.

    With Q = I - K Y^T (K = Y Tq), A = L - K P^T - P K^T + K G K^T where
    L = diag(lam), P = L Y and G = Y^T L Y; assembled as one rank-2k product.
    """
    lam = np.asarray(lam, dtype=np.float64)
    n = lam.shape[0]
    Y, Tq = householder_factor(n, rng, count)
    K = Y @ Tq
    P = lam[:, None] * Y
    G = Y.T @ P
    k = Y.shape[1]
    left = np.concatenate([K, P], axis=1)                      # n x 2k
    mid = np.block([[G, -np.eye(k)], [-np.eye(k), np.zeros((k, k))]])
    A = left @ (mid @ left.T)
    A[np.diag_indices(n)] += lam
    return _symmetrize_inplace(A)


def geometric_spectrum(n: int, rng: np.random.Generator) -> np.ndarray:
    mag = 10.0 ** (-8.0 * np.arange(n) / max(n - 1, 1))
    sign = rng.choice(np.array([-1.0, 1.0]), size=n)
    return mag * sign


def clustered_spectrum(n: int, rng: np.random.Generator, clusters: int = 64,
                       spread: float = 1e-10) -> np.ndarray:
    centres = rng.uniform(-1.0, 1.0, size=clusters)
    per = np.full(clusters, n // clusters)
    per[: n - per.sum()] += 1
    c = np.repeat(centres, per)
    return c + spread * rng.uniform(-1.0, 1.0, size=n)


def uniform_spectrum(n: int, rng: np.random.Generator) -> np.ndarray:
    return rng.uniform(-1.0, 1.0, size=n)


def scf_like(n: int, rng: np.random.Generator) -> np.ndarray:
    i = np.arange(n)
    decay = np.exp(-np.abs(i[:, None] - i[None, :]) / 20.0)
    M = rng.normal(0.0, 0.1, size=(n, n)) * decay
    A = 0.5 * (M + M.T)
    A[np.diag_indices(n)] = np.sort(rng.uniform(-20.0, 5.0, size=n))
    return A


def batch_sizes(count: int, rng: np.random.Generator, lo: int = 32, hi: int = 512) -> np.ndarray:
    return rng.integers(lo, hi + 1, size=count)


def toeplitz_tridiagonal(n: int, alpha: float = 0.0, beta: float = 1.0):
    """(d, e) of tridiag(beta, alpha, beta)."""
    return np.full(n, float(alpha)), np.full(max(n - 1, 0), float(beta))


def dense_from_tridiagonal(d: np.ndarray, e: np.ndarray) -> np.ndarray:
    A = np.diag(np.asarray(d, dtype=np.float64))
    if len(e):
        A += np.diag(e, 1) + np.diag(e, -1)
    return A


def workload(cfg: int, inp: int = 0, n: int | None = None):
    """Matrix (and prescribed spectrum or None) for a named workload.

    ``n`` overrides the size (same recipe at a smaller size, for tests).
    Returns (A, lam_prescribed_or_None).
    """
    rng = make_rng(cfg, inp)
    default_n = {CFG_SMALL: 256, CFG_MEDIUM: 8192, CFG_LARGE: 32768, CFG_FP32: 16384}
    if cfg == CFG_BATCH:
        raise ValueError("use batch_workload for the batched configuration")
    n = int(n or default_n[cfg])
    if inp == 0:
        return gaussian_symmetric(n, rng), None
    if cfg == CFG_MEDIUM:
        lam = geometric_spectrum(n, rng)
    elif cfg == CFG_LARGE:
        lam = clustered_spectrum(n, rng)
    elif cfg == CFG_FP32:
        lam = uniform_spectrum(n, rng)
    else:
        lam = uniform_spectrum(n, rng)
    return spectrum_matrix(lam, rng), np.sort(lam)


def batch_workload(count: int = 4096, inp: int = 0, lo: int = 32, hi: int = 512):
    rng = make_rng(CFG_BATCH, inp)
    sizes = batch_sizes(count, rng, lo, hi)
    return [scf_like(int(m), rng) for m in sizes]
