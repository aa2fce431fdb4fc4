"""Pins for the NumPy model of the paper's algorithms (oracle/sbr_model.py).

Identities of Eq. (4.1), Eq. (4.2) and Corollary 3.7, the Ensure clauses of
Algorithms 3.2, 4.1 and 4.2 (exact band structure, spectrum preserved), and the
chase-ordering rule used by the GPU pipeline.
"""
import itertools
import math

import numpy as np
import pytest

import sbr_inputs as si
from oracle import sbr_model as M

EPS = np.finfo(np.float64).eps


def _random_wy(m, c, seed):
    rng = np.random.default_rng(seed)
    U, tau, _ = M.householder_qr(rng.standard_normal((m, c)))
    return U, M.larft(U, tau)


@pytest.mark.parametrize("m,c", [(12, 3), (40, 8), (33, 16)])
def test_eq_4_1_two_sided_update(m, c):
    U, T = _random_wy(m, c, m + c)
    X = si.gaussian_symmetric(m, np.random.default_rng(m))
    Q = np.eye(m) - U @ T @ U.T
    lhs = Q.T @ X @ Q
    rhs = M.two_sided_update(X, U, T)
    assert np.max(np.abs(lhs - rhs)) <= 50 * m * EPS * np.max(np.abs(X))
    # Q is orthogonal and U^T U = T^{-1} + T^{-T} (Corollary 3.7)
    assert np.max(np.abs(Q.T @ Q - np.eye(m))) <= 50 * m * EPS
    Ti = np.linalg.inv(T)
    assert np.max(np.abs(U.T @ U - Ti - Ti.T)) <= 100 * m * EPS * np.max(np.abs(Ti))


def test_eq_4_2_deferred_application():
    m, c = 30, 6
    U, T = _random_wy(m, c, 3)
    X = si.gaussian_symmetric(m, np.random.default_rng(4))
    Y = np.random.default_rng(5).standard_normal((m, 5))
    Q = np.eye(m) - U @ T @ U.T
    V = M.two_sided_v(X, U, T)
    assert np.allclose(Q.T @ X @ Q @ Y, X @ Y + U @ (V.T @ Y) + V @ (U.T @ Y), atol=1e-12)


@pytest.mark.parametrize("m,c,p", [(64, 8, 1), (64, 8, 4), (200, 16, 8), (130, 16, 4), (48, 16, 2)])
def test_rect_qr(oracle_mod, m, c, p):
    A = np.random.default_rng(m * c + p).standard_normal((m, c))
    Q, R = M.rect_qr(A, p)
    assert Q.shape == (m, c) and R.shape == (c, c)
    assert np.max(np.abs(np.tril(R, -1))) == 0.0
    assert np.max(np.abs(Q @ R - A)) <= 100 * m * EPS * np.max(np.abs(A))
    assert np.max(np.abs(Q.T @ Q - np.eye(c))) <= 100 * m * EPS
    s = np.sign(np.diag(R))
    assert np.allclose(s[:, None] * R, oracle_mod.qr_r(A), atol=1e-12 * np.max(np.abs(A)))


@pytest.mark.parametrize("m,c", [(16, 4), (96, 16), (64, 32)])
def test_householder_reconstruction(m, c):
    P = np.random.default_rng(m + 7 * c).standard_normal((m, c))
    Q, R = M.rect_qr(P, 4)
    U, T, S = M.householder_reconstruct(Q)
    U1 = U[:c]
    assert np.allclose(np.diag(U1), 1.0) and np.max(np.abs(np.triu(U1, 1))) == 0.0
    assert np.max(np.abs(np.tril(T, -1))) <= 1e-14
    H = np.eye(m) - U @ T @ U.T
    assert np.allclose(H[:, :c], Q * S[None, :], atol=1e-13)
    top = np.zeros((m, c))
    top[:c] = S[:, None] * R
    assert np.allclose(H.T @ P, top, atol=1e-12)
    assert np.max(np.abs(H.T @ H - np.eye(m))) <= 1e-13
    Ti = np.linalg.inv(T)
    assert np.allclose(U.T @ U, Ti + Ti.T, atol=1e-11 * np.max(np.abs(Ti)))


@pytest.mark.parametrize("n,b", [(64, 8), (67, 8), (100, 16), (33, 4), (40, 2), (129, 32), (20, 16)])
def test_full_to_band_and_halvings(oracle_mod, n, b):
    A = si.gaussian_symmetric(n, si.make_rng(si.CFG_SMALL, 0))
    ref = oracle_mod.eigvalsh(A)
    fro = math.sqrt(float(np.sum(A * A)))
    B = M.full_to_band(A, b)
    assert M.bandwidth(B) <= b
    assert np.max(np.abs(B - B.T)) <= 1e-13 * fro
    assert abs(np.trace(B) - np.trace(A)) <= 1e-12 * fro
    assert abs(math.sqrt(float(np.sum(B * B))) - fro) <= 1e-13 * fro * n
    assert np.max(np.abs(oracle_mod.eigvalsh(B) - ref)) <= 1e-12 * np.max(np.abs(ref))
    h = b
    while h > 1:
        B = M.band_to_band(B, h)     # also asserts the window reading per chase
        h //= 2
        assert M.bandwidth(B) <= h
        assert np.max(np.abs(oracle_mod.eigvalsh(B) - ref)) <= 1e-12 * np.max(np.abs(ref))
    d, e = np.diag(B), np.diag(B, -1)
    assert np.max(np.abs(oracle_mod.tridiag_eigvals(d, e) - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_model_pipeline_prescribed_spectrum(oracle_mod):
    rng = np.random.default_rng(11)
    lam = si.geometric_spectrum(96, rng)
    A = si.spectrum_matrix(lam, rng)
    d, e = M.sbr_eigvals(A, 16)
    w = oracle_mod.tridiag_eigvals(d, e)
    assert np.max(np.abs(w - np.sort(lam))) <= 1e-13


def _ancestors(chases, lag):
    last = {}
    for c in chases:
        last[c["i"]] = max(last.get(c["i"], 0), c["j"])
    anc = {}
    for c in chases:
        i, j = c["i"], c["j"]
        s = set()
        preds = []
        if j > 1:
            preds.append((i, j - 1))
        if i > 1 and (i - 1) in last:
            preds.append((i - 1, min(j + lag - 1, last[i - 1])))
        for p in preds:
            s |= anc[p]
            s.add(p)
        anc[(i, j)] = s
    return anc


def _conflicts_not_ordered(n, b, lag):
    chases = M.chase_list(n, b)
    touched = [M.chase_touched(c) for c in chases]
    anc = _ancestors(chases, lag)
    bad = 0
    for a, c in itertools.combinations(range(len(chases)), 2):
        if touched[a] & touched[c]:
            ka = (chases[a]["i"], chases[a]["j"])
            kc = (chases[c]["i"], chases[c]["j"])
            bad += ka not in anc[kc]
    return bad


@pytest.mark.parametrize("n,b", [(64, 8), (67, 4), (128, 16), (60, 2), (45, 8)])
def test_chase_schedule_lag3_orders_every_conflict(n, b):
    # chase (i, j) waits for (i, j-1) and (i-1, j+2): every pair of chases
    # that write a common entry is ordered as in the sequential loop nest.
    assert _conflicts_not_ordered(n, b, 3) == 0


def test_chase_schedule_lag2_is_not_enough():
    # Running (i, j) beside (i-1, j+2) (a new panel after the previous bulge
    # moved twice) lets two chases write the same entries.
    assert _conflicts_not_ordered(64, 8, 2) > 0


def test_chase_list_bounds():
    # n not a multiple of b: the last sweeps still get their chases (reading G4)
    ch = M.chase_list(21, 4)
    sweeps = sorted({c["i"] for c in ch})
    assert sweeps == list(range(1, (21 - 2) // 2 + 1))
    for c in ch:
        r0, r1 = c["qr_rows"]
        assert r1 - r0 >= 2 and r1 <= 21


def _phase_touched(ch):
    """Entries of one chase split by phase: the QR block (read, then written
    with [R; 0]) and the rest (left, diagonal and below blocks)."""
    q = set()
    for r in range(*ch["qr_rows"]):
        for c in range(*ch["qr_cols"]):
            q.add((max(r, c), min(r, c)))
    return q, M.chase_touched(ch) - q


def _phase_conflicts_not_ordered(n, b, h=None):
    # chase (i, j): its QR phase waits for (i, j-1) complete and for the QR
    # phase of (i-1, j+2) (the whole sweep i-1 when it has no chase j+2);
    # its other phase follows its own QR phase
    chases = M.chase_list(n, b, h)
    last = {}
    for c in chases:
        last[c["i"]] = max(last.get(c["i"], 0), c["j"])
    anc = {}
    for c in chases:
        i, j = c["i"], c["j"]
        preds = []
        if j > 1:
            preds.append((i, j - 1, "R"))
        if i > 1 and (i - 1) in last:
            if j + 2 <= last[i - 1]:
                preds.append((i - 1, j + 2, "Q"))
            else:
                preds.append((i - 1, last[i - 1], "R"))
        s = set()
        for p in preds:
            s |= anc[p]
            s.add(p)
        anc[(i, j, "Q")] = s
        anc[(i, j, "R")] = s | {(i, j, "Q")}
    nodes, sets = [], []
    for c in chases:
        q, r = _phase_touched(c)
        nodes += [(c["i"], c["j"], "Q"), (c["i"], c["j"], "R")]
        sets += [q, r]
    bad = 0
    for a, c in itertools.combinations(range(len(nodes)), 2):
        if nodes[a][:2] == nodes[c][:2]:
            continue
        if sets[a] & sets[c]:
            bad += nodes[a] not in anc[nodes[c]] and nodes[c] not in anc[nodes[a]]
    return bad


@pytest.mark.parametrize("n,b", [(64, 8), (67, 4), (128, 16), (60, 2), (45, 8), (200, 32)])
def test_chase_schedule_after_previous_qr_orders_every_conflict(n, b):
    # the relaxed pipeline of the wide-band kernel: chase (i, j) may start once
    # chase (i-1, j+2) has finished its QR block (the only entries the two
    # share); every pair of phases that touch a common entry stays ordered
    assert _phase_conflicts_not_ordered(n, b) == 0


@pytest.mark.parametrize("n,b,h", [(64, 16, 4), (67, 16, 2), (130, 32, 8), (100, 32, 4), (129, 64, 8),
                                   (200, 64, 16), (45, 8, 2)])
def test_chase_schedule_after_previous_qr_general_k(n, b, h):
    # the same pipeline for b -> h = b / k with k > 2 (one work-group per
    # sweep, chase (i, j) after the QR phase of (i-1, j+2)): every pair of
    # phases touching a common entry is still ordered as in the loop nest, so
    # the below block a work-group keeps for its next chase is not written by
    # another sweep in between
    assert _phase_conflicts_not_ordered(n, b, h) == 0


def _three_phase_conflicts(n, b, h, lag):
    # the wide-band kernel's schedule: chase (i, j) in three phases, its QR
    # block (Q), its left block (L) and its diagonal and below blocks (D).
    # Q(i, j) follows D(i, j-1) of the same work-group (Q(i, 1) also waits
    # for Q(i-1, 2)); L follows Q; D follows L and the QR phase of
    # (i-1, j+lag) (the whole sweep i-1 when it has no such chase)
    chases = M.chase_list(n, b, h)
    last = {}
    for c in chases:
        last[c["i"]] = max(last.get(c["i"], 0), c["j"])

    def prev_q(i, j):
        return (i, j, "Q") if j <= last[i] else (i, last[i], "D")

    anc = {}

    def add(node, preds):
        s = set()
        for p in preds:
            s |= anc[p]
            s.add(p)
        anc[node] = s

    nodes, sets = [], []
    for c in chases:
        i, j = c["i"], c["j"]
        qp = [(i, j - 1, "D")] if j > 1 else []
        if i > 1 and j == 1:
            qp.append(prev_q(i - 1, 2))
        add((i, j, "Q"), qp)
        add((i, j, "L"), [(i, j, "Q")])
        add((i, j, "D"), [(i, j, "L")] + ([prev_q(i - 1, j + lag)] if i > 1 else []))
        q, r = _phase_touched(c)
        o = c["qr_rows"][0]
        left = {e for e in r if e[1] < o}
        for ph, st in (("Q", q), ("L", left), ("D", r - left)):
            nodes.append((i, j, ph))
            sets.append(st)
    bad = 0
    for a, c in itertools.combinations(range(len(nodes)), 2):
        if nodes[a][:2] == nodes[c][:2]:
            continue
        if sets[a] & sets[c]:
            bad += nodes[a] not in anc[nodes[c]] and nodes[c] not in anc[nodes[a]]
    return bad


@pytest.mark.parametrize("n,b,h", [(64, 8, 4), (67, 4, 2), (128, 16, 8), (200, 32, 16), (130, 32, 8),
                                   (100, 32, 4), (129, 64, 8), (200, 64, 16), (300, 128, 32), (250, 128, 16)])
def test_chase_schedule_early_qr_and_left_block(n, b, h):
    # the QR and left blocks of a chase go ahead of the wait for sweep i-1:
    # every pair of phases touching a common entry is still ordered as in the
    # loop nest; waiting for (i-1, j+1) instead of (i-1, j+2) is not enough
    assert _three_phase_conflicts(n, b, h, 2) == 0
    assert _three_phase_conflicts(n, b, h, 1) > 0


def _lockstep_phase_conflicts(n, b, lag, h=None):
    # the small-band pipeline: at step tau every sweep s of a group does chase
    # j = tau - lag*s, first all the QR blocks (phase 0), then the rest (phase 1);
    # a conflicting pair of phases must run at different times, in the order of
    # the sequential loop nest (sweep-major, QR phase first)
    chases = M.chase_list(n, b, h)
    first_i = min(c["i"] for c in chases)
    nodes = []
    for c in chases:
        q, r = _phase_touched(c)
        tau = c["j"] + lag * (c["i"] - first_i)
        nodes.append(((tau, 0), (c["i"], c["j"], 0), q))
        nodes.append(((tau, 1), (c["i"], c["j"], 1), r))
    bad = 0
    for a, c in itertools.combinations(nodes, 2):
        if a[1][:2] == c[1][:2] or not (a[2] & c[2]):
            continue
        if a[0] == c[0] or (a[0] < c[0]) != (a[1] < c[1]):
            bad += 1
    return bad


@pytest.mark.parametrize("n,b", [(64, 8), (67, 4), (60, 2), (45, 8), (100, 16)])
def test_lockstep_two_phase_lag2_orders_every_conflict(n, b):
    # two phases per step (QR blocks, then the rest) let consecutive sweeps run
    # two chases apart instead of three
    assert _lockstep_phase_conflicts(n, b, 2) == 0


def test_lockstep_two_phase_lag1_is_not_enough():
    assert _lockstep_phase_conflicts(64, 8, 1) > 0


@pytest.mark.parametrize("n,b,h", [(64, 8, 1), (67, 8, 2), (50, 4, 1), (100, 16, 1), (100, 16, 4), (33, 8, 1),
                                   (20, 16, 1), (40, 2, 1), (130, 32, 1)])
def test_band_to_band_general_k(oracle_mod, n, b, h):
    # Algorithm 4.2 with k = b / h > 2: the same offsets and extents with
    # h = b / k; the band shrinks to exactly h (k = b: straight to the
    # tridiagonal) and the spectrum is kept
    rng = np.random.default_rng(n * b + h)
    A = rng.standard_normal((n, n))
    A = 0.5 * (A + A.T)
    i, j = np.indices((n, n))
    A[np.abs(i - j) > b] = 0.0
    ref = oracle_mod.eigvalsh(A)
    B = M.band_to_band(A, b, h=h)       # also asserts the window reading per chase
    assert M.bandwidth(B) <= h
    fro = math.sqrt(float(np.sum(A * A)))
    assert abs(math.sqrt(float(np.sum(B * B))) - fro) <= 1e-13 * fro * n
    assert np.max(np.abs(oracle_mod.eigvalsh(B) - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("n,b", [(35, 4), (67, 8), (100, 16)])
def test_lockstep_two_phase_lag2_direct_to_tridiagonal(n, b):
    # the two-phase lock-step schedule with a lag of two chases also orders
    # every conflict of the direct b -> 1 reduction; a lag of one does not
    assert _lockstep_phase_conflicts(n, b, 2, h=1) == 0
    assert _lockstep_phase_conflicts(n, b, 1, h=1) > 0


def _carry_violations(n, b, h, lag):
    # a sweep keeps its chase's below block (rows [o+b, o+2b) x cols [o, o+b))
    # in registers for its next chase; no phase of another sweep may write
    # those entries between the two (lock-step schedule, two phases per step)
    chases = M.chase_list(n, b, h)
    first_i = min(c["i"] for c in chases)
    when = {}
    written = []
    for c in chases:
        q, r = _phase_touched(c)
        tau = c["j"] + lag * (c["i"] - first_i)
        when[(c["i"], c["j"])] = tau
        written.append(((tau, 0), c["i"], q))
        written.append(((tau, 1), c["i"], r))
    bad = 0
    for c in chases:
        i, j = c["i"], c["j"]
        if (i, j + 1) not in when:
            continue
        r0, r1 = c["qr_rows"]
        o = r0
        blk = {(r, cc) for r in range(o + b, min(n, o + 2 * b)) for cc in range(o, min(n, o + b)) if r >= cc}
        t0, t1 = (when[(i, j)], 1), (when[(i, j + 1)], 0)
        for t, ii, ent in written:
            if ii != i and t0 < t < t1 and (ent & blk):
                bad += 1
    return bad


@pytest.mark.parametrize("n,b,h", [(35, 4, 1), (67, 8, 1), (100, 16, 1), (64, 8, 4), (60, 4, 2)])
def test_lockstep_lag2_keeps_the_carried_below_block(n, b, h):
    assert _carry_violations(n, b, h, 2) == 0
