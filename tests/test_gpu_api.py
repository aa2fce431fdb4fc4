"""GPU tests of the boundary's promises beyond the numbers themselves.

* the plan's status word: a band stage abandoned by a forced wait limit (set
  from the host, so every kernel still exits normally) raises
  SBR_STATUS_STALLED and turns the call's eigenvalues into NaN, and the next
  call on the same plan computes correctly again;
* non-finite input: every eigenvalue NaN and SBR_STATUS_NONFINITE raised;
* leading dimensions beyond n (lda > n for the solver, ldband > 2b + 1 for a
  halving), element by element against the oracle;
* a solve through a plan captured in a HIP graph and replayed on new data,
  each replay against the oracle;
* a plan too large for the device returns SBR_ENOMEM and leaves the device
  usable.
"""
import ctypes

import numpy as np
import pytest
import torch

import sbr_inputs as si
from gpu_util import band_to_dense, random_band

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sbr():
    import paper_1604_03703_amd as m
    assert torch.cuda.is_available()
    return m


def _norm2(ref):
    return max(1e-300, float(np.max(np.abs(ref))))


@pytest.mark.parametrize("n,b0", [(3000, 32), (3000, 8)])
def test_forced_stall_gives_nan_then_next_call_recovers(sbr, oracle_mod, n, b0):
    # a wait limit of one clock tick: the first chase that has to wait for the
    # previous sweep gives up, the stage is abandoned and every block exits
    print("stall", n, b0, flush=True)
    A = si.gaussian_symmetric(n, si.make_rng(si.CFG_SMALL, 5))
    ref = oracle_mod.eigvalsh(A)
    plan = sbr.Plan(n)
    assert plan.status() == 0
    plan.set_wait_limit(1)
    w = sbr.eigvalsh(torch.from_numpy(A).cuda(), b0=b0, plan=plan)
    torch.cuda.synchronize()
    st = plan.status()
    assert st & sbr.STATUS_STALLED, st
    assert torch.isnan(w).all()
    assert plan.status() == 0            # read once, then cleared
    plan.set_wait_limit(0)               # back to the default
    w = sbr.eigvalsh(torch.from_numpy(A).cuda(), b0=b0, plan=plan)
    torch.cuda.synchronize()
    assert plan.status() == 0
    assert np.max(np.abs(w.cpu().numpy() - ref)) <= 1e-11 * _norm2(ref)
    plan.close()


def test_forced_stall_of_a_halving_then_recovery(sbr, oracle_mod):
    n, b = 2000, 64
    rng = np.random.default_rng(21)
    A = random_band(n, b, rng)
    ref = oracle_mod.eigvalsh(A)
    band = np.zeros((n, 2 * b + 1))
    for d in range(b + 1):
        band[: n - d, d] = np.diag(A, -d)
    plan = sbr.Plan(0)
    plan.set_wait_limit(1)
    sbr.band_halve(torch.from_numpy(band.copy()).cuda(), b, plan)
    assert plan.status() & sbr.STATUS_STALLED
    plan.set_wait_limit(0)
    bd = torch.from_numpy(band.copy()).cuda()
    sbr.band_halve(bd, b, plan)
    assert plan.status() == 0
    out = bd.cpu().numpy()
    assert np.all(out[:, b // 2 + 1:] == 0.0)
    w = oracle_mod.eigvalsh(band_to_dense(out, n))
    assert np.max(np.abs(w - ref)) <= 1e-11 * _norm2(ref)


@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_nonfinite_input(sbr, bad):
    n = 200
    A = si.gaussian_symmetric(n, si.make_rng(si.CFG_SMALL, 6))
    A[17, 3] = A[3, 17] = bad
    plan = sbr.Plan(n)
    w = sbr.eigvalsh(torch.from_numpy(A).cuda(), b0=16, plan=plan)
    torch.cuda.synchronize()
    assert torch.isnan(w).all()
    assert plan.status() & sbr.STATUS_NONFINITE
    # the next call on the same plan is clean
    B = si.gaussian_symmetric(n, si.make_rng(si.CFG_SMALL, 7))
    w = sbr.eigvalsh(torch.from_numpy(B).cuda(), b0=16, plan=plan)
    torch.cuda.synchronize()
    assert plan.status() == 0
    ref = np.linalg.eigvalsh(B)
    assert np.max(np.abs(w.cpu().numpy() - ref)) <= 1e-11 * _norm2(ref)
    # the tridiagonal entry point directly
    d = np.arange(10.0)
    e = np.ones(9)
    e[4] = bad
    wt = sbr.tridiag_eigvals(torch.from_numpy(d).cuda(), torch.from_numpy(e).cuda())
    assert torch.isnan(wt).all()


@pytest.mark.parametrize("n,b0,lda", [(300, 32, 317), (1000, 64, 1100), (777, 128, 800), (257, 2, 300)])
def test_eigvalsh_lda_larger_than_n(sbr, oracle_mod, n, b0, lda):
    print("lda", n, b0, lda, flush=True)
    A = si.gaussian_symmetric(n, si.make_rng(si.CFG_SMALL, 8))
    ref = oracle_mod.eigvalsh(A)
    X = torch.full((n, lda), 1e300, dtype=torch.float64, device="cuda")   # padding never read as data
    X[:, :n] = torch.from_numpy(A).cuda()
    view = X[:, :n]
    assert view.stride() == (lda, 1)
    plan = sbr.Plan(n)
    w = sbr.eigvalsh(view, b0=b0, plan=plan, overwrite=True)
    torch.cuda.synchronize()
    assert plan.status() == 0
    err = np.max(np.abs(w.cpu().numpy() - ref))
    print("lda %d: max err %.3e" % (lda, err / _norm2(ref)), flush=True)
    assert err <= 1e-11 * _norm2(ref)


@pytest.mark.parametrize("n", [2432, 4096])
def test_full_tile_product_paths_agree(sbr, oracle_mod, n):
    # b0 = 128 and trailing orders that are multiples of 128: with an even
    # leading dimension the FP64 W = A22 Y reads Y^T and moves its operands
    # straight into LDS, with an odd one it passes them through registers;
    # the products and their order are the same, so the eigenvalues must be
    # the same bit for bit, and right
    print("full-tile product paths", n, flush=True)
    A = si.gaussian_symmetric(n, si.make_rng(si.CFG_SMALL, 12))
    ref = oracle_mod.eigvalsh(A)
    ws = []
    for lda in (n, n + 1):
        X = torch.zeros((n, lda), dtype=torch.float64, device="cuda")
        X[:, :n] = torch.from_numpy(A).cuda()
        plan = sbr.Plan(n)
        w = sbr.eigvalsh(X[:, :n], b0=128, plan=plan, overwrite=True)
        torch.cuda.synchronize()
        assert plan.status() == 0
        ws.append(w.cpu().numpy())
    assert np.array_equal(ws[0], ws[1])
    err = np.max(np.abs(ws[0] - ref))
    print("n %d: max err %.3e" % (n, err / _norm2(ref)), flush=True)
    assert err <= 1e-11 * _norm2(ref)


@pytest.mark.parametrize("b", [2, 4, 8, 16, 32, 64, 128])
def test_band_halve_wide_ldband(sbr, oracle_mod, b):
    n = 600
    ld = 2 * b + 1 + 7
    print("wide ldband", b, ld, flush=True)
    rng = np.random.default_rng(300 + b)
    A = random_band(n, b, rng)
    ref = oracle_mod.eigvalsh(A)
    band = np.zeros((n, ld))
    for d in range(b + 1):
        band[: n - d, d] = np.diag(A, -d)
    plan = sbr.Plan(0)
    bd = torch.from_numpy(band).cuda()
    sbr.band_halve(bd, b, plan)
    torch.cuda.synchronize()
    assert plan.status() == 0
    out = bd.cpu().numpy()
    assert np.all(out[:, b // 2 + 1:] == 0.0)
    w = oracle_mod.eigvalsh(band_to_dense(out, n))
    assert np.max(np.abs(w - ref)) <= 1e-11 * _norm2(ref)


@pytest.mark.parametrize("n,b", [(600, 16), (3000, 16)])
def test_band_halve_b16_group_kernel(sbr, oracle_mod, n, b):
    # b = 16 through the sweep-group kernel instead of the MFMA chase: parity
    # with the oracle and the same bits at any grid size
    print("group b16", n, flush=True)
    rng = np.random.default_rng(410 + n)
    A = random_band(n, b, rng)
    ref = oracle_mod.eigvalsh(A)
    band = np.zeros((n, 2 * b + 1))
    for d in range(b + 1):
        band[: n - d, d] = np.diag(A, -d)
    outs = []
    for blocks in (0, 1):
        p = sbr.Plan(0)
        p.set_group_max_band(16)
        p.set_chase_blocks(blocks)
        bd = torch.from_numpy(band.copy()).cuda()
        sbr.band_halve(bd, b, p)
        torch.cuda.synchronize()
        assert p.status() == 0
        outs.append(bd.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])
    assert np.all(outs[0][:, b // 2 + 1:] == 0.0)
    w = oracle_mod.eigvalsh(band_to_dense(outs[0], n))
    assert np.max(np.abs(w - ref)) <= 1e-11 * _norm2(ref)


@pytest.mark.parametrize("n,b0,precision", [(700, 64, "fp64"), (1030, 128, "fp64"), (700, 64, "fp32_mfma")])
def test_solver_captured_in_hip_graph(sbr, oracle_mod, n, b0, precision):
    # once the plan holds its workspace a call allocates nothing and never
    # waits for the device, so it can be captured; replays on new data in the
    # same input buffer, with eager work and synchronisation between replays
    print("graph", n, b0, precision, flush=True)
    plan = sbr.Plan(n, 0, precision)
    Ad = torch.empty((n, n), dtype=torch.float64, device="cuda")
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    A0 = si.gaussian_symmetric(n, si.make_rng(si.CFG_SMALL, 9))
    Ad.copy_(torch.from_numpy(A0))
    sbr.eigvalsh(Ad, b0=b0, precision=precision, plan=plan, overwrite=True, out=w)   # warm-up, eager
    torch.cuda.synchronize()
    assert plan.status() == 0
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            sbr.eigvalsh(Ad, b0=b0, precision=precision, plan=plan, overwrite=True, out=w)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    tol = 1e-11 if precision == "fp64" else 2e-5
    for rep in range(3):
        A = si.gaussian_symmetric(n, si.make_rng(si.CFG_SMALL, 10 + rep))
        ref = oracle_mod.eigvalsh(A)
        Ad.copy_(torch.from_numpy(A))
        junk = torch.randn(1000, 1000, device="cuda", dtype=torch.float64).sum()   # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert plan.status() == 0
        assert float(junk) == float(junk)
        err = np.max(np.abs(w.cpu().numpy() - ref))
        print("replay %d: max err %.3e" % (rep, err / _norm2(ref)), flush=True)
        assert err <= tol * _norm2(ref)
    del g
    plan.close()


def test_plan_too_large_returns_enomem(sbr, oracle_mod):
    lib = sbr.lib()
    h = ctypes.c_void_p()
    # n = 2^26 needs several n x 128 FP64 buffers of 64 GiB each
    rc = lib.sbr_plan_create(ctypes.byref(h), 1 << 26, 0, 0)
    assert rc == 1, rc            # SBR_ENOMEM
    assert not h.value
    # the device is still usable
    A = si.gaussian_symmetric(100, si.make_rng(si.CFG_SMALL, 11))
    w = sbr.eigvalsh(torch.from_numpy(A).cuda(), b0=16)
    torch.cuda.synchronize()
    ref = oracle_mod.eigvalsh(A)
    assert np.max(np.abs(w.cpu().numpy() - ref)) <= 1e-11 * _norm2(ref)


def test_batched_rejects_strided_views(sbr):
    A = torch.eye(40, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        sbr.eigvalsh_batched([A.t()[::2, ::2]])
    with pytest.raises(ValueError):
        sbr.eigvalsh_batched([torch.zeros((4, 5), dtype=torch.float64, device="cuda")])
