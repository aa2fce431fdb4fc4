"""Full-to-band with aggregated two-sided updates (Eq. (4.2), the plan's
update depth D > 1), against the oracle.

Inside a group of D panels each panel's W = A22 Y is taken from the matrix
as it stood at the start of the group plus the pending updates'
corrections U (V^T Y) + V (U^T Y); the next panel's columns get the pending
updates before they are factored, and one SYR2K of rank 2 D b per group
updates the trailing matrix.  Cases cover full groups, a last group cut
short by the end of the matrix, ragged n, and groups that end one panel
before the base block.  Bar: max |lam - lam_oracle| <= 1e-11 ||A||_2, the
FP64 solver's bar; the band itself must have the input's eigenvalues.
"""
import numpy as np
import pytest
import torch

import sbr_inputs as si

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sbr():
    import paper_1604_03703_amd as m
    assert torch.cuda.is_available()
    return m


def _norm2(ref):
    return max(1e-300, float(np.max(np.abs(ref))))


@pytest.mark.parametrize("n,b0,depth", [(600, 16, 2), (1000, 32, 3), (777, 64, 4), (2048, 128, 2),
                                        (4100, 128, 3), (300, 128, 2), (257, 32, 4), (1100, 64, 2)])
def test_solver_with_aggregated_updates(sbr, oracle_mod, n, b0, depth):
    print("update depth", n, b0, depth, flush=True)
    A = si.gaussian_symmetric(n, si.make_rng(si.CFG_SMALL, 40 + depth))
    ref = oracle_mod.eigvalsh(A)
    plan = sbr.Plan(n)
    plan.set_update_depth(depth)
    w = sbr.eigvalsh(torch.from_numpy(A).cuda(), b0=b0, plan=plan)
    torch.cuda.synchronize()
    assert plan.status() == 0
    err = np.max(np.abs(w.cpu().numpy() - ref))
    print("depth %d n %d b0 %d: max err %.3e" % (depth, n, b0, err / _norm2(ref)), flush=True)
    assert err <= 1e-11 * _norm2(ref)


@pytest.mark.parametrize("depth", [1, 2, 4])
def test_band_from_aggregated_updates(sbr, oracle_mod, depth):
    # the band the full-to-band call leaves has the input's eigenvalues, and
    # the same call on one plan gives the same band bit for bit
    n, b = 1500, 64
    A = si.gaussian_symmetric(n, si.make_rng(si.CFG_SMALL, 77))
    ref = oracle_mod.eigvalsh(A)
    plan = sbr.Plan(n)
    plan.set_update_depth(depth)
    bands = []
    for _ in range(2):
        X = torch.from_numpy(A.copy()).cuda()
        sbr.full_to_band(X, b, plan)
        torch.cuda.synchronize()
        bands.append(np.tril(X.cpu().numpy().T))      # column-major lower triangle
    assert np.array_equal(bands[0], bands[1])
    L = bands[0]
    i, j = np.indices((n, n))
    assert np.all(L[(i - j) > b] == 0.0), "entries below the band must be exactly zero"
    B = L + np.tril(L, -1).T
    wb = oracle_mod.eigvalsh(B)
    err = np.max(np.abs(wb - ref))
    print("depth %d band eigenvalues: max err %.3e" % (depth, err / _norm2(ref)), flush=True)
    assert err <= 1e-11 * _norm2(ref)


def test_fp32_form_keeps_depth_one(sbr, oracle_mod):
    n = 1200
    A = si.gaussian_symmetric(n, si.make_rng(si.CFG_SMALL, 91))
    ref = oracle_mod.eigvalsh(A)
    plan = sbr.Plan(n, 0, "fp32_mfma")
    plan.set_update_depth(3)
    w = sbr.eigvalsh(torch.from_numpy(A).cuda(), b0=64, precision="fp32_mfma", plan=plan)
    torch.cuda.synchronize()
    err = np.max(np.abs(w.cpu().numpy() - ref))
    assert err <= 2e-5 * _norm2(ref)


def test_update_depth_rejects_out_of_range(sbr):
    plan = sbr.Plan(100)
    for bad in (0, 5, -1):
        with pytest.raises(sbr.SbrError):
            plan.set_update_depth(bad)
