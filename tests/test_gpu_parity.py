"""GPU parity of the stages and of the whole eigensolver against the CPU
oracle on seeded inputs.

Tolerances (the accuracy targets of the method):
FP64 path  max |lam - lam_oracle| <= 1e-11 ||A||_2,
FP32-MFMA  max |lam - lam_oracle| <= 2e-5  ||A||_2,
with ||A||_2 = max |lam_oracle|.  Band structure is checked exactly (entries
outside the band must be exactly zero).
"""
import math

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


@pytest.fixture(scope="module")
def plan(sbr):
    return sbr.Plan(0)


def _norm2(ref):
    return max(1e-300, float(np.max(np.abs(ref))))


def _lower_band_of_colmajor(Ad: torch.Tensor, n: int):
    """Column-major matrix held in the row-major tensor: element (i, j) is Ad[j, i]."""
    M = Ad.detach().cpu().numpy().T          # M[i, j] = column-major (i, j)
    return np.tril(M)


@pytest.mark.parametrize("n,b", [(20, 16), (64, 16), (100, 16), (256, 16), (300, 32), (520, 64),
                                 (700, 128), (50, 2), (77, 8), (130, 64)])
def test_full_to_band(sbr, plan, oracle_mod, n, b):
    print("f2b", n, b, flush=True)
    A = si.gaussian_symmetric(n, si.make_rng(si.CFG_SMALL, 1))
    ref = oracle_mod.eigvalsh(A)
    Ad = torch.from_numpy(A.copy()).cuda()
    sbr.full_to_band(Ad, b, plan)
    torch.cuda.synchronize()
    L = _lower_band_of_colmajor(Ad, n)
    i, j = np.indices((n, n))
    assert np.all(L[(i - j) > b] == 0.0), "entries below the band must be exactly zero"
    B = L + np.tril(L, -1).T
    fro = math.sqrt(float(np.sum(A * A)))
    assert abs(np.trace(B) - np.trace(A)) <= 1e-12 * fro * math.sqrt(n)
    assert abs(math.sqrt(float(np.sum(B * B))) - fro) <= 1e-12 * fro * math.sqrt(n)
    w = oracle_mod.eigvalsh(B)
    assert np.max(np.abs(w - ref)) <= 1e-11 * _norm2(ref)


@pytest.mark.parametrize("b", [2, 4, 8, 16, 32, 64, 128])
@pytest.mark.parametrize("n_rel", ["b+1", "3b+5", "200", "513"])
def test_band_halve(sbr, plan, oracle_mod, b, n_rel):
    n = {"b+1": b + 1, "3b+5": 3 * b + 5, "200": 200, "513": 513}[n_rel]
    print("halve", n, b, flush=True)
    rng = np.random.default_rng(1000 * b + n)
    A = random_band(n, b, rng)
    ref = oracle_mod.eigvalsh(A)
    ld = 2 * b + 1
    band = np.zeros((n, ld))
    for d in range(min(b + 1, n)):
        band[: n - d, d] = np.diag(A, -d)
    bd = torch.from_numpy(band).cuda()
    sbr.band_halve(bd, b, plan)
    torch.cuda.synchronize()
    assert plan.status() == 0
    out = bd.cpu().numpy()
    h = b // 2
    assert np.all(out[:, h + 1:] == 0.0), "entries beyond the new bandwidth must be exactly zero"
    B = band_to_dense(out, n)
    w = oracle_mod.eigvalsh(B)
    assert np.max(np.abs(w - ref)) <= 1e-11 * _norm2(ref)


@pytest.mark.parametrize("n,b", [(600, 4), (600, 16), (600, 32), (600, 64), (700, 128), (3000, 16), (3000, 32),
                                 (3000, 64)])
def test_band_halve_pipelined_equals_sequential(sbr, oracle_mod, n, b):
    # every chase does the same arithmetic on the same data in any schedule
    # that respects the dependencies, so the pipelined grid and a single
    # block (sequential sweep order) must agree bit for bit; the single block
    # always finds the previous sweep done (every chase's blocks are loaded
    # during the chase before it), the grid mixes loads made early and loads
    # made after a wait
    print("race", n, b, flush=True)
    rng = np.random.default_rng(77 + b)
    A = random_band(n, b, rng)
    ld = 2 * b + 1
    band = np.zeros((n, ld))
    for d in range(b + 1):
        band[: n - d, d] = np.diag(A, -d)
    outs = []
    for blocks in (0, 1):
        p = sbr.Plan(0)
        p.set_chase_blocks(blocks)
        bd = torch.from_numpy(band.copy()).cuda()
        sbr.band_halve(bd, b, p)
        torch.cuda.synchronize()
        assert p.status() == 0
        outs.append(bd.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("precision", ["fp64", "fp32_mfma"])
def test_panel_cus_setting_is_bitwise_neutral(sbr, oracle_mod, precision):
    # the CUs kept free for the concurrent panel only change where the bulk
    # trailing update runs, never its arithmetic
    print("panel_cus", precision, flush=True)
    n, b0 = 1536, 64
    A = si.gaussian_symmetric(n, si.make_rng(si.CFG_SMALL, 3))
    outs = []
    for cus in (0, 16, 64):
        p = sbr.Plan(n, 0, precision)
        p.set_panel_cus(cus)
        w = sbr.eigvalsh(torch.from_numpy(A).cuda(), b0=b0, precision=precision, plan=p)
        torch.cuda.synchronize()
        outs.append(w.cpu().numpy())
        p.close()
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    ref = oracle_mod.eigvalsh(A)
    tol = 1e-11 if precision == "fp64" else 2e-5
    assert np.max(np.abs(outs[0] - ref)) <= tol * _norm2(ref)


SIZES = [(1, 0), (2, 0), (3, 0), (4, 2), (5, 0), (17, 4), (33, 8), (64, 16), (100, 16), (256, 16),
         (300, 32), (257, 2), (1000, 64), (777, 128)]


@pytest.mark.parametrize("n,b0", SIZES)
def test_eigvalsh_gaussian(sbr, oracle_mod, n, b0):
    print("eig", n, b0, flush=True)
    A = si.gaussian_symmetric(n, si.make_rng(si.CFG_SMALL, 0))
    ref = oracle_mod.eigvalsh(A)
    w = sbr.eigvalsh(torch.from_numpy(A).cuda(), b0=b0)
    torch.cuda.synchronize()
    assert np.max(np.abs(w.cpu().numpy() - ref)) <= 1e-11 * _norm2(ref)


def test_eigvalsh_config_small(sbr, oracle_mod):
    # the n = 256, b0 = 16 workload: 16 -> 8 -> 4 -> 2 -> 1, all 256 eigenvalues
    A, _ = si.workload(si.CFG_SMALL, 0)
    ref = oracle_mod.eigvalsh(A)
    w = sbr.eigvalsh(torch.from_numpy(A).cuda(), b0=16)
    torch.cuda.synchronize()
    err = np.max(np.abs(w.cpu().numpy() - ref))
    print("n=256 b0=16 max err %.3e (||A||=%.3f)" % (err, _norm2(ref)), flush=True)
    assert err <= 1e-11 * _norm2(ref)


@pytest.mark.parametrize("kind", ["geometric", "clustered", "uniform"])
@pytest.mark.parametrize("n,b0", [(300, 16), (640, 64)])
def test_eigvalsh_prescribed_spectrum(sbr, oracle_mod, kind, n, b0):
    print("spec", kind, n, b0, flush=True)
    rng = np.random.default_rng(n + len(kind))
    lam = {"geometric": si.geometric_spectrum, "clustered": si.clustered_spectrum,
           "uniform": si.uniform_spectrum}[kind](n, rng)
    A = si.spectrum_matrix(lam, rng)
    ref = oracle_mod.eigvalsh(A)
    w = sbr.eigvalsh(torch.from_numpy(A).cuda(), b0=b0).cpu().numpy()
    lam = np.sort(lam)
    assert np.max(np.abs(w - ref)) <= 1e-11 * _norm2(ref)
    assert np.max(np.abs(w - lam)) <= 1e-11 * _norm2(lam)


def test_eigvalsh_toeplitz_embedded(sbr):
    # Q T Q^T with T = tridiag(1, 0, 1): closed-form spectrum 2 cos(k pi / (n + 1))
    n = 400
    rng = np.random.default_rng(3)
    k = np.arange(1, n + 1)
    lam = 2.0 * np.cos(k * math.pi / (n + 1))
    A = si.spectrum_matrix(lam, rng)
    w = sbr.eigvalsh(torch.from_numpy(A).cuda(), b0=32).cpu().numpy()
    assert np.max(np.abs(w - np.sort(lam))) <= 1e-11 * 2.0


def test_eigvalsh_special_matrices(sbr):
    for A in (np.zeros((40, 40)), 3.0 * np.eye(33), np.diag(np.arange(50.0) - 20.0),
              si.dense_from_tridiagonal(*si.toeplitz_tridiagonal(70, 1.0, -2.0))):
        n = A.shape[0]
        ref = np.linalg.eigvalsh(A)
        w = sbr.eigvalsh(torch.from_numpy(A.copy()).cuda(), b0=8).cpu().numpy()
        assert np.max(np.abs(w - ref)) <= 1e-11 * max(1.0, np.max(np.abs(ref))), n


@pytest.mark.parametrize("n,b0", [(256, 16), (700, 64), (1030, 128)])
def test_eigvalsh_fp32_mfma_form(sbr, oracle_mod, n, b0):
    A = si.gaussian_symmetric(n, si.make_rng(si.CFG_FP32, 0))
    ref = oracle_mod.eigvalsh(A)
    w = sbr.eigvalsh(torch.from_numpy(A).cuda(), b0=b0, precision="fp32_mfma").cpu().numpy()
    err = np.abs(w - ref)
    print("fp32 form n=%d: max %.3e rms %.3e (x ||A||)" % (n, err.max() / _norm2(ref),
                                                           math.sqrt(np.mean(err ** 2)) / _norm2(ref)))
    assert err.max() <= 2e-5 * _norm2(ref)


def test_eigvalsh_batched(sbr, oracle_mod):
    mats = si.batch_workload(count=24, lo=32, hi=200)
    refs = [oracle_mod.eigvalsh(M) for M in mats]
    dev = [torch.from_numpy(M.copy()).cuda() for M in mats]
    ws = sbr.eigvalsh_batched(dev)
    torch.cuda.synchronize()
    for w, ref in zip(ws, refs):
        assert np.max(np.abs(w.cpu().numpy() - ref)) <= 1e-11 * _norm2(ref)


BATCH_SIZES = [1, 2, 3, 4, 5, 9, 17, 33, 64, 65, 96, 97, 128, 200, 257, 300, 511, 512, 600]


@pytest.mark.parametrize("b0", [0, 4, 8, 16, 32])
def test_eigvalsh_batched_sizes(sbr, oracle_mod, b0):
    # every size class of the batched kernels (n <= 2: no reduction; n > 512
    # or b0 > 16: the single-matrix path), Gaussian and SCF-like inputs
    print("batched sizes b0", b0, flush=True)
    rng = np.random.default_rng(11 + b0)
    mats = []
    for k, m in enumerate(BATCH_SIZES):
        mats.append(si.scf_like(m, rng) if k % 2 else si.gaussian_symmetric(m, rng))
    refs = [oracle_mod.eigvalsh(M) for M in mats]
    dev = [torch.from_numpy(M.copy()).cuda() for M in mats]
    ws = sbr.eigvalsh_batched(dev, b0=b0)
    torch.cuda.synchronize()
    for M, w, ref in zip(mats, ws, refs):
        err = np.max(np.abs(w.cpu().numpy() - ref))
        assert err <= 1e-11 * max(_norm2(ref), 1e-300) or err == 0.0, (M.shape[0], err)


def test_eigvalsh_batched_replay_and_reshape(sbr, oracle_mod):
    # same buffers twice (the captured launch is replayed on new data), then a
    # different batch on the same plan (descriptors and launch rebuilt)
    rng = np.random.default_rng(5)
    sizes = [40, 300, 150, 512, 70]
    plan = sbr.Plan(512, 8)
    dev = [torch.empty((m, m), dtype=torch.float64, device="cuda") for m in sizes]
    for rep in range(2):
        mats = [si.scf_like(m, rng) for m in sizes]
        for d, M in zip(dev, mats):
            d.copy_(torch.from_numpy(M))
        ws = sbr.eigvalsh_batched(dev, plan=plan)
        torch.cuda.synchronize()
        for M, w in zip(mats, ws):
            ref = oracle_mod.eigvalsh(M)
            assert np.max(np.abs(w.cpu().numpy() - ref)) <= 1e-11 * _norm2(ref), (rep, M.shape[0])
    mats = [si.gaussian_symmetric(m, rng) for m in (100, 31, 257)]
    dev2 = [torch.from_numpy(M.copy()).cuda() for M in mats]
    ws = sbr.eigvalsh_batched(dev2, plan=plan)
    torch.cuda.synchronize()
    for M, w in zip(mats, ws):
        ref = oracle_mod.eigvalsh(M)
        assert np.max(np.abs(w.cpu().numpy() - ref)) <= 1e-11 * _norm2(ref)


def test_batched_solve_prepared_call(sbr, oracle_mod):
    # the prepared call marshals its arguments once; each run() on refilled
    # buffers replays the captured launch and matches the oracle
    rng = np.random.default_rng(8)
    sizes = [33, 512, 129, 200, 64, 7]
    dev = [torch.empty((m, m), dtype=torch.float64, device="cuda") for m in sizes]
    call = sbr.BatchedSolve(dev)
    for rep in range(3):
        mats = [si.scf_like(m, rng) if rep != 1 else si.gaussian_symmetric(m, rng) for m in sizes]
        for d, M in zip(dev, mats):
            d.copy_(torch.from_numpy(M))
        ws = call.run()
        torch.cuda.synchronize()
        for M, w in zip(mats, ws):
            ref = oracle_mod.eigvalsh(M)
            assert np.max(np.abs(w.cpu().numpy() - ref)) <= 1e-11 * _norm2(ref), (rep, M.shape[0])


@pytest.mark.parametrize("b0", [0, 4, 8, 16])
def test_eigvalsh_batched_fp32_form(sbr, oracle_mod, b0):
    # the batched FP32-MFMA form: trailing updates of the batched
    # full-to-band on FP32 MFMA; every matrix within 2e-5 ||A||_2 of the
    # oracle, and not bit-identical to the FP64 form (the FP32 path ran)
    mats = si.batch_workload(count=24, lo=3, hi=512)
    refs = [oracle_mod.eigvalsh(M) for M in mats]
    dev = [torch.from_numpy(M.copy()).cuda() for M in mats]
    ws = sbr.eigvalsh_batched(dev, b0=b0, precision="fp32_mfma")
    dev64 = [torch.from_numpy(M.copy()).cuda() for M in mats]
    ws64 = sbr.eigvalsh_batched(dev64, b0=b0, precision="fp64")
    torch.cuda.synchronize()
    worst, differ = 0.0, 0
    for M, w, w64, ref in zip(mats, ws, ws64, refs):
        e = np.max(np.abs(w.cpu().numpy() - ref)) / _norm2(ref)
        worst = max(worst, e)
        assert e <= 2e-5, (M.shape[0], e)
        assert np.max(np.abs(w64.cpu().numpy() - ref)) <= 1e-11 * _norm2(ref)
        differ += int(not np.array_equal(w.cpu().numpy(), w64.cpu().numpy()))
    print("batched fp32 b0=%d: max err %.3e (x ||A||_2), %d of %d differ from FP64" % (b0, worst, differ, len(mats)),
          flush=True)
    assert differ > len(mats) // 2
