"""GPU parity of the band-to-band reduction b -> h = b / k with k > 2
(Algorithm 4.2 for general k, sbr_band_reduce) against the oracle, and of
solves whose stage sequence uses it.

Bar: entries beyond the h-th sub-diagonal exactly zero, eigenvalues within
1e-11 ||A||_2 of the oracle's, the same bits at any grid size (chase (i, j)
starts after the QR block of chase (i-1, j+2) whatever k is; every conflict
stays ordered as in the loop nest, see test_model.py)."""
import numpy as np
import pytest
import torch

import sbr_inputs as si
from gpu_util import band_to_dense, random_band

pytestmark = pytest.mark.gpu

PAIRS = [(16, 8), (32, 16), (32, 8), (64, 32), (64, 16), (64, 8), (128, 64), (128, 32), (128, 16), (128, 8)]


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


@pytest.mark.parametrize("b,h", PAIRS)
@pytest.mark.parametrize("n_rel", ["b+1", "b+h+3", "3b+5", "700", "1337"])
def test_band_reduce(sbr, oracle_mod, b, h, n_rel):
    n = {"b+1": b + 1, "b+h+3": b + h + 3, "3b+5": 3 * b + 5, "700": 700, "1337": 1337}[n_rel]
    print("band reduce n=%d b=%d h=%d" % (n, b, h), flush=True)
    rng = np.random.default_rng(31000 + 7 * b + h + n)
    A = random_band(n, b, rng)
    ref = oracle_mod.eigvalsh(A)
    plan = sbr.Plan(0)
    bd = torch.from_numpy(_band_storage(A, b, 2 * b + 1)).cuda()
    sbr.band_reduce(bd, b, h, plan)
    torch.cuda.synchronize()
    assert plan.status() == 0
    out = bd.cpu().numpy()
    assert np.all(out[:, h + 1:] == 0.0), "entries beyond the h-th sub-diagonal must be exactly zero"
    w = oracle_mod.eigvalsh(band_to_dense(out, n, keep=h))
    err = np.max(np.abs(w - ref))
    assert err <= 1e-11 * _norm2(ref), err


@pytest.mark.parametrize("b,h", [(32, 8), (64, 16), (64, 8), (128, 32), (128, 16), (128, 8)])
def test_band_reduce_grid_independent(sbr, b, h):
    # one work-group (every sweep in order) and the full grid give the same bits
    n = 3000
    print("band reduce race n=%d b=%d h=%d" % (n, b, h), flush=True)
    rng = np.random.default_rng(77 + b + h)
    band = _band_storage(random_band(n, b, rng), b, 2 * b + 1)
    outs = []
    for blocks in (0, 1):
        p = sbr.Plan(0)
        p.set_chase_blocks(blocks)
        bd = torch.from_numpy(band.copy()).cuda()
        sbr.band_reduce(bd, b, h, p)
        torch.cuda.synchronize()
        assert p.status() == 0
        outs.append(bd.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("b,h", [(64, 16), (128, 16)])
def test_band_reduce_wide_ldband(sbr, oracle_mod, b, h):
    n = 600
    rng = np.random.default_rng(400 + b + h)
    A = random_band(n, b, rng)
    ref = oracle_mod.eigvalsh(A)
    plan = sbr.Plan(0)
    bd = torch.from_numpy(_band_storage(A, b, 2 * b + 9)).cuda()
    sbr.band_reduce(bd, b, h, plan)
    torch.cuda.synchronize()
    assert plan.status() == 0
    out = bd.cpu().numpy()
    assert np.all(out[:, h + 1:] == 0.0)
    w = oracle_mod.eigvalsh(band_to_dense(out, n, keep=h))
    assert np.max(np.abs(w - ref)) <= 1e-11 * _norm2(ref)


def test_band_reduce_rejects_unsupported(sbr):
    plan = sbr.Plan(0)
    bd = torch.zeros((100, 257), dtype=torch.float64, device="cuda")
    for b, h, code in [(32, 12, -5), (32, 32, -5), (32, 4, -5), (64, 2, -5), (24, 8, -5)]:
        rc = sbr.lib().sbr_band_reduce(plan.handle, 100, bd.data_ptr(), 257, b, h, 0, None)
        assert rc == code, (b, h, rc)
    assert sbr.lib().sbr_band_reduce(plan.handle, 100, bd.data_ptr(), 64, 32, 8, 0, None) == -4


@pytest.mark.parametrize("n,b0,widths,expect", [
    (1000, 128, [16, 8, 4, 1], None), (1000, 128, [32, 8, 1], None), (777, 64, [8, 1], None),
    (1500, 128, [64, 8, 4, 2, 1], None), (3000, 128, [], None),
    # 16 -> 4 has no kernel: from 16 the next listed width taken is 1
    (1000, 128, [16, 4, 1], [16, 1])])
def test_solver_with_band_stage_sequence(sbr, oracle_mod, n, b0, widths, expect):
    print("solve n=%d b0=%d widths=%s" % (n, b0, widths), flush=True)
    A = si.gaussian_symmetric(n, si.make_rng(si.CFG_SMALL, 21))
    ref = oracle_mod.eigvalsh(A)
    plan = sbr.Plan(n)
    plan.set_band_stages(widths)
    seq = plan.band_stages(n, b0)
    assert seq[-1] == 1 and all(x > y for x, y in zip([b0] + seq, seq))
    if widths:
        assert seq == (expect or widths), seq
    w = sbr.eigvalsh(torch.from_numpy(A).cuda(), b0=b0, plan=plan)
    torch.cuda.synchronize()
    assert plan.status() == 0
    err = np.max(np.abs(w.cpu().numpy() - ref))
    print("stages %s max err %.3e" % (seq, err / _norm2(ref)), flush=True)
    assert err <= 1e-11 * _norm2(ref)


@pytest.mark.parametrize("b,h", PAIRS)
@pytest.mark.parametrize("n", [300, 1337])
def test_band_reduce_fp32_form(sbr, oracle_mod, b, h, n):
    # the FP32-MFMA form: the WY applications of every chase on FP32 MFMA
    # (QR, tau and T in FP64); the band structure stays exact and the
    # spectrum is kept to the FP32 form's bar
    print("band reduce fp32 n=%d b=%d h=%d" % (n, b, h), flush=True)
    rng = np.random.default_rng(52000 + 3 * b + h + n)
    A = random_band(n, b, rng)
    ref = oracle_mod.eigvalsh(A)
    plan = sbr.Plan(0)
    bd = torch.from_numpy(_band_storage(A, b, 2 * b + 1)).cuda()
    sbr.band_reduce(bd, b, h, plan, precision="fp32_mfma")
    torch.cuda.synchronize()
    assert plan.status() == 0
    out = bd.cpu().numpy()
    assert np.all(out[:, h + 1:] == 0.0)
    w = oracle_mod.eigvalsh(band_to_dense(out, n, keep=h))
    err = np.max(np.abs(w - ref)) / _norm2(ref)
    print("  max err %.3e (x ||A||_2)" % err, flush=True)
    assert err <= 2e-5
