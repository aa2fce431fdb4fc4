"""NumPy model of the paper's successive band reduction -- TEST INFRASTRUCTURE.

Plain FP64 transcription (dense, both triangles kept) of the algorithms of
Solomonik, Ballard, Demmel & Hoefler, "A communication-avoiding parallel
algorithm for the symmetric eigenvalue problem":

* ``rect_qr``               -- Algorithm 3.2 (rect-QR): row blocks, QR of each,
                               QR of the stacked R factors, Q_i = W_i Z_i.
* ``householder_reconstruct`` -- Corollary 3.7: [U1, W1] = LU(Q1 - S),
                               U = Q W1^{-1}, T from W1 and U1, with the sign
                               matrix the corollary leaves out kept explicit:
                               S_ii = -sign of the current pivot (so no pivot is
                               below 1 in magnitude), (I - U T U^T)[:, :b] = Q S,
                               T = -W1 S U1^{-T}, and the band receives S R.
* ``two_sided_update``       -- Eq. (4.1): Q^T X Q = X + U V^T + V U^T with
                               V = 1/2 U T^T U^T X U T - X U T.
* ``full_to_band``           -- Algorithm 4.1, right-looking (complete trailing
                               update after every panel, allowed by the
                               implementation notes of Section 5).
* ``band_to_band``           -- Algorithm 4.2 with k = 2 and the offsets,
                               loop bounds read as follows: chase (i, j) exists
                               while its QR block's first row is <= n - 2 and
                               sweep i while i h <= n - 2 (the printed floor
                               leaves tail sweeps without chases); the update's
                               column offset for j = 1 is the QR block's first
                               row; the update spans exactly 2b columns for
                               j = 1 and 3b - h for j > 1.

It exists to settle those readings on the CPU (exact zeros outside the band,
eigenvalues preserved) and to describe each chase's touched entries for the
schedule checker.  Only ``tests/`` use it; the GPU path shares nothing with it.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import solve_triangular


# --------------------------------------------------------------------------
# Householder building blocks (sequential QR of Lemma 3.4)
# --------------------------------------------------------------------------
def householder_vector(x: np.ndarray):
    """(v, tau, beta): (I - tau v v^T) x = beta e_0 with v_0 = 1.

    beta = -sgn(x_0) |x| (sgn(0) = +1); if x_1.. = 0 then tau = 0, beta = x_0.
    """
    x = np.asarray(x, dtype=np.float64)
    v = np.zeros_like(x)
    v[0] = 1.0
    if x.shape[0] <= 1:
        return v, 0.0, float(x[0]) if x.shape[0] else 0.0
    tail = np.linalg.norm(x[1:])
    alpha = float(x[0])
    if tail == 0.0:
        return v, 0.0, alpha
    beta = -math.copysign(math.hypot(alpha, tail), alpha)
    tau = (beta - alpha) / beta
    v[1:] = x[1:] / (alpha - beta)
    return v, tau, beta


def householder_qr(A: np.ndarray):
    """Householder QR of an m x c block.

    Returns (U, tau, R): U is m x k unit lower trapezoidal (k = min(m - 1, c)
    reflectors; a column with a single remaining row needs none), R = Q^T A
    (m x c, upper trapezoidal), Q = H_0 ... H_{k-1}.
    """
    R = np.array(A, dtype=np.float64, copy=True)
    m, c = R.shape
    k = max(0, min(m - 1, c))
    U = np.zeros((m, k))
    tau = np.zeros(k)
    for t in range(k):
        v, tt, beta = householder_vector(R[t:, t])
        U[t:, t] = v
        tau[t] = tt
        if tt != 0.0:
            R[t:, t:] -= tt * np.outer(v, v @ R[t:, t:])
        R[t, t] = beta
        R[t + 1:, t] = 0.0
    return U, tau, R


def larft(U: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """Upper triangular T with H_0 ... H_{k-1} = I - U T U^T (forward, columnwise)."""
    k = U.shape[1]
    T = np.zeros((k, k))
    for t in range(k):
        T[t, t] = tau[t]
        if t:
            T[:t, t] = -tau[t] * (T[:t, :t] @ (U[:, :t].T @ U[:, t]))
    return T


def explicit_q(U: np.ndarray, tau: np.ndarray, ncols: int) -> np.ndarray:
    """First ``ncols`` columns of H_0 ... H_{k-1}."""
    m = U.shape[0]
    Q = np.eye(m, ncols)
    for t in reversed(range(U.shape[1])):
        v = U[:, t]
        Q -= tau[t] * np.outer(v, v @ Q)
    return Q


# --------------------------------------------------------------------------
# Algorithm 3.2 (rect-QR) and Corollary 3.7 (Householder reconstruction)
# --------------------------------------------------------------------------
def rect_qr(A: np.ndarray, p: int = 1):
    """[Q, R] <- rect-QR(A, p): thin explicit Q (m x c) and upper triangular R.

    ``p`` plays the role of the processor count (a power of two): the rows are
    split into r = min(p, ceil(m / 2c)) blocks, each factored recursively, then
    the stacked R factors are factored and Q_i = W_i Z_i.
    """
    A = np.asarray(A, dtype=np.float64)
    m, c = A.shape
    if m < c:
        raise ValueError("rect_qr needs m >= c")
    if p == 1 or m <= 2 * c:
        U, tau, R = householder_qr(A)
        return explicit_q(U, tau, c), np.triu(R[:c, :c])
    r = min(p, math.ceil(m / (2 * c)))
    bounds = [round(m * i / r) for i in range(r + 1)]
    Ws, Rs = [], []
    for i in range(r):
        W, R = rect_qr(A[bounds[i]:bounds[i + 1]], max(1, p // r))
        Ws.append(W)
        Rs.append(R)
    Z, R = rect_qr(np.vstack(Rs), p)
    Q = np.vstack([Ws[i] @ Z[i * c:(i + 1) * c] for i in range(r)])
    return Q, R


def householder_reconstruct(Q: np.ndarray):
    """(U, T, S) with (I - U T U^T)[:, :c] = Q S, from the explicit thin Q (m x c).

    LU without pivoting of Q1 - S, S_ii = -sgn of the current pivot (so that
    |pivot| = |.| + 1 >= 1); U1 unit lower, W1 upper; U2 = Q2 W1^{-1};
    T = -W1 S U1^{-T}.
    """
    Q = np.asarray(Q, dtype=np.float64)
    m, c = Q.shape
    F = np.array(Q[:c], copy=True)
    S = np.zeros(c)
    for i in range(c):
        S[i] = -1.0 if F[i, i] >= 0.0 else 1.0
        F[i, i] -= S[i]
        F[i + 1:, i] /= F[i, i]
        F[i + 1:, i + 1:] -= np.outer(F[i + 1:, i], F[i, i + 1:])
    U1 = np.tril(F, -1) + np.eye(c)
    W1 = np.triu(F)
    U2 = solve_triangular(W1, Q[c:].T, trans="T", lower=False).T if m > c else np.zeros((0, c))
    U1inv = solve_triangular(U1, np.eye(c), lower=True, unit_diagonal=True)
    T = -(W1 * S[None, :]) @ U1inv.T
    return np.vstack([U1, U2]), T, S


# --------------------------------------------------------------------------
# Eq. (4.1) and Algorithm 4.1 (full-to-band)
# --------------------------------------------------------------------------
def two_sided_v(X: np.ndarray, U: np.ndarray, T: np.ndarray) -> np.ndarray:
    """V = 1/2 U (T^T (U^T W)) - W with W = X U T (Eq. (4.1))."""
    W = X @ U @ T
    return 0.5 * U @ (T.T @ (U.T @ W)) - W


def two_sided_update(X: np.ndarray, U: np.ndarray, T: np.ndarray) -> np.ndarray:
    V = two_sided_v(X, U, T)
    return X + U @ V.T + V @ U.T


def full_to_band(A: np.ndarray, b: int, leaves: int = 4) -> np.ndarray:
    """Reduce the dense symmetric A to bandwidth b (Algorithm 4.1, right-looking).

    Panel k: QR of A[r0:, c0:c0+b] by rect-QR + reconstruction; the band block
    becomes [S R; 0]; the trailing matrix gets Eq. (4.1).  A panel with fewer
    rows than b (only when b does not divide n) is factored directly by
    Householder QR, giving [U, T] and the trapezoidal R = Q^T panel.
    """
    B = np.array(A, dtype=np.float64, copy=True)
    n = B.shape[0]
    c0 = 0
    while True:
        r0 = c0 + b
        m = n - r0
        if m < 2:
            break
        P = B[r0:, c0:c0 + b]
        if m >= b:
            Q, R = rect_qr(P, leaves)
            U, T, S = householder_reconstruct(Q)
            newP = np.zeros_like(P)
            newP[:b] = S[:, None] * R
        else:
            U, tau, newP = householder_qr(P)
            T = larft(U, tau)
        B[r0:, c0:c0 + b] = newP
        B[c0:c0 + b, r0:] = newP.T
        B[r0:, r0:] = two_sided_update(B[r0:, r0:], U, T)
        c0 += b
    return B


# --------------------------------------------------------------------------
# Algorithm 4.2 (band-to-band), b -> h = b / k
# --------------------------------------------------------------------------
def chase_list(n: int, b: int, h: int | None = None):
    """All chases (i, j) of one reduction b -> h (h = b / k, default k = 2) in
    sequential order, with their offsets and exact index ranges (0-based,
    half-open).

    Loop bounds (reading G4): sweep i exists while i*h <= n - 2; chase j
    exists while o_qr.r <= n - 2 (at least two rows to factor).
    Update columns (G5/G6): j = 1 -> [o_qr.r, o_qr.r + 2b); j > 1 ->
    [o_qr.c + h, o_qr.c + 3b), clipped at n.
    """
    h = b // 2 if h is None else h
    assert 1 <= h < b and b % h == 0
    out = []
    i = 1
    while i * h <= n - 2:
        j = 1
        while True:
            o_blg = (i - 1) * h + (j - 1) * b
            o_qr_r = o_blg + h
            if o_qr_r > n - 2:
                break
            if j == 1:
                o_qr_c = o_qr_r - h
                o_v = 0
                o_up_c = o_qr_r
                nc_exact = 2 * b
            else:
                o_qr_c = o_qr_r - b
                o_v = b - h
                o_up_c = o_qr_c + h
                nc_exact = 3 * b - h
            n_r = min(n - o_qr_r, b)
            n_c = min(n - o_up_c, nc_exact)
            out.append(dict(i=i, j=j, qr_rows=(o_qr_r, o_qr_r + n_r), qr_cols=(o_qr_c, o_qr_c + h),
                            v_rows=(o_v, o_v + n_r), up_cols=(o_up_c, o_up_c + n_c)))
            j += 1
        i += 1
    return out


def chase_touched(ch) -> set:
    """Lower-triangle entries (r, c), r >= c, written by one chase."""
    rs = range(*ch["qr_rows"])
    s = set()
    for r in rs:
        for c in range(*ch["qr_cols"]):
            s.add((max(r, c), min(r, c)))
        for c in range(*ch["up_cols"]):
            s.add((max(r, c), min(r, c)))
    return s


def band_to_band(B: np.ndarray, b: int, check_window: bool = True, h: int | None = None) -> np.ndarray:
    """One reduction b -> h (h = b / k, default k = 2: a halving) of the
    symmetric band matrix B (dense storage).

    For each chase: [U, T, R] = QR(B[I_qr.rs, I_qr.cs]); the block becomes
    [R; 0]; W = B[I_up.cs, I_qr.rs] U T; V = -W;
    V[I_v.rs] += 1/2 U (T^T (U^T W[I_v.rs])); B[I_qr.rs, I_up.cs] += U V^T;
    B[I_up.cs, I_qr.rs] += V U^T.
    """
    B = np.array(B, dtype=np.float64, copy=True)
    n = B.shape[0]
    for ch in chase_list(n, b, h):
        r0, r1 = ch["qr_rows"]
        c0, c1 = ch["qr_cols"]
        u0, u1 = ch["up_cols"]
        v0, v1 = ch["v_rows"]
        if check_window:
            # rows of the QR block carry nothing outside QR columns + update columns
            row = B[r0:r1].copy()
            row[:, c0:c1] = 0.0
            row[:, u0:u1] = 0.0
            if np.any(row != 0.0):
                raise AssertionError("window reading violated at chase %s" % ((ch["i"], ch["j"]),))
        blk = B[r0:r1, c0:c1]
        U, tau, R = householder_qr(blk)
        T = larft(U, tau)
        B[r0:r1, c0:c1] = R
        B[c0:c1, r0:r1] = R.T
        W = B[u0:u1, r0:r1] @ U @ T
        V = -W
        V[v0:v1] += 0.5 * U @ (T.T @ (U.T @ W[v0:v1]))
        B[r0:r1, u0:u1] += U @ V.T
        B[u0:u1, r0:r1] += V @ U.T
    return B


def bandwidth(B: np.ndarray) -> int:
    """Largest |i - j| with B[i, j] != 0 (0 for a diagonal or empty matrix)."""
    idx = np.nonzero(B)
    if len(idx[0]) == 0:
        return 0
    return int(np.max(np.abs(idx[0] - idx[1])))


def sbr_eigvals(A: np.ndarray, b0: int, leaves: int = 4):
    """Full model pipeline: full-to-band b0, halvings to 1, returns (d, e)."""
    B = full_to_band(A, b0, leaves)
    b = b0
    while b > 1:
        B = band_to_band(B, b)
        b //= 2
    n = B.shape[0]
    return np.diag(B).copy(), np.diag(B, -1).copy() if n > 1 else np.zeros(0)
