"""GPU parity of the direct band-to-tridiagonal stage (Algorithm 4.2 with
k = b, h = 1; sbr_band_to_tridiag) against the oracle, and of solves that use
it for the last bands.

Bar: entries beyond the first sub-diagonal exactly zero, eigenvalues within
1e-11 ||A||_2 of the oracle's, the same bits at any grid size (every chase
does the same arithmetic on the same data in any schedule that keeps the
dependencies)."""
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


def _band_storage(A, b, ld):
    n = A.shape[0]
    band = np.zeros((n, ld))
    for d in range(min(b + 1, n)):
        band[: n - d, d] = np.diag(A, -d)
    return band


@pytest.mark.parametrize("b", [4, 8, 16])
@pytest.mark.parametrize("n_rel", ["b+1", "b+2", "3b+5", "200", "513", "1000"])
def test_band_to_tridiag(sbr, oracle_mod, b, n_rel):
    n = {"b+1": b + 1, "b+2": b + 2, "3b+5": 3 * b + 5, "200": 200, "513": 513, "1000": 1000}[n_rel]
    print("tridiag stage n=%d b=%d" % (n, b), flush=True)
    rng = np.random.default_rng(7000 + 10 * b + n)
    A = random_band(n, b, rng)
    ref = oracle_mod.eigvalsh(A)
    plan = sbr.Plan(0)
    bd = torch.from_numpy(_band_storage(A, b, 2 * b + 1)).cuda()
    sbr.band_to_tridiag(bd, b, plan)
    torch.cuda.synchronize()
    assert plan.status() == 0
    out = bd.cpu().numpy()
    assert np.all(out[:, 2:] == 0.0), "entries beyond the first sub-diagonal must be exactly zero"
    w = oracle_mod.tridiag_eigvals(out[:, 0].copy(), out[: n - 1, 1].copy())
    err = np.max(np.abs(w - ref))
    assert err <= 1e-11 * _norm2(ref), err


@pytest.mark.parametrize("n,b", [(600, 4), (600, 8), (600, 16), (3000, 4), (3000, 8), (3000, 16)])
def test_band_to_tridiag_grid_independent(sbr, n, b):
    print("tridiag race n=%d b=%d" % (n, b), flush=True)
    rng = np.random.default_rng(17 + b)
    band = _band_storage(random_band(n, b, rng), b, 2 * b + 1)
    outs = []
    for blocks in (0, 1):
        p = sbr.Plan(0)
        p.set_chase_blocks(blocks)
        bd = torch.from_numpy(band.copy()).cuda()
        sbr.band_to_tridiag(bd, b, p)
        torch.cuda.synchronize()
        assert p.status() == 0
        outs.append(bd.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("b", [4, 8, 16])
@pytest.mark.parametrize("n", [300, 2000])
def test_band_to_tridiag_launch_shapes(sbr, oracle_mod, n, b, variant):
    # the other launch shapes (lanes per sweep, sweeps per work-group): the
    # same chases with the team sums grouped differently
    print("tridiag shape n=%d b=%d variant=%d" % (n, b, variant), flush=True)
    rng = np.random.default_rng(500 + n + b)
    A = random_band(n, b, rng)
    ref = oracle_mod.eigvalsh(A)
    plan = sbr.Plan(0)
    plan.set_tridiag_band(0, variant)
    bd = torch.from_numpy(_band_storage(A, b, 2 * b + 1)).cuda()
    sbr.band_to_tridiag(bd, b, plan)
    torch.cuda.synchronize()
    assert plan.status() == 0
    out = bd.cpu().numpy()
    assert np.all(out[:, 2:] == 0.0)
    w = oracle_mod.tridiag_eigvals(out[:, 0].copy(), out[: n - 1, 1].copy())
    assert np.max(np.abs(w - ref)) <= 1e-11 * _norm2(ref)


@pytest.mark.parametrize("b", [4, 8, 16])
def test_band_to_tridiag_wide_ldband(sbr, oracle_mod, b):
    n = 500
    rng = np.random.default_rng(900 + b)
    A = random_band(n, b, rng)
    ref = oracle_mod.eigvalsh(A)
    plan = sbr.Plan(0)
    bd = torch.from_numpy(_band_storage(A, b, 2 * b + 6)).cuda()
    sbr.band_to_tridiag(bd, b, plan)
    torch.cuda.synchronize()
    assert plan.status() == 0
    out = bd.cpu().numpy()
    assert np.all(out[:, 2:] == 0.0)
    w = oracle_mod.eigvalsh(band_to_dense(out, n))
    assert np.max(np.abs(w - ref)) <= 1e-11 * _norm2(ref)


@pytest.mark.parametrize("n,b0,tri", [(1000, 64, 16), (1000, 64, 8), (777, 128, 4), (300, 16, 16), (5000, 64, 16),
                                      (1000, 64, 0), (777, 128, 0)])
def test_solver_with_direct_tridiagonal_stage(sbr, oracle_mod, n, b0, tri):
    print("solve n=%d b0=%d tri=%d" % (n, b0, tri), flush=True)
    A = si.gaussian_symmetric(n, si.make_rng(si.CFG_SMALL, 12))
    ref = oracle_mod.eigvalsh(A)
    plan = sbr.Plan(n)
    plan.set_tridiag_band(tri)
    w = sbr.eigvalsh(torch.from_numpy(A).cuda(), b0=b0, plan=plan)
    torch.cuda.synchronize()
    assert plan.status() == 0
    err = np.max(np.abs(w.cpu().numpy() - ref))
    print("max err %.3e" % (err / _norm2(ref)), flush=True)
    assert err <= 1e-11 * _norm2(ref)
