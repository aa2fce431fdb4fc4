"""The batched form with the tuned band per size bucket: the stored tuning
table is well formed (CPU), and a batch solved with it, or with any valid
table, matches the oracle matrix by matrix (GPU)."""
import numpy as np
import pytest

import sbr_inputs as si


def _norm2(ref):
    return max(1e-300, float(np.max(np.abs(ref))))


def test_tuning_database_is_well_formed():
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_1604_03703_amd", "tuning", "batched.json")
    db = json.load(open(path))
    assert db, "no tuning stored"
    for arch, forms in db.items():
        for prec, rec in forms.items():
            assert prec in ("fp64", "fp32_mfma")
            prev = 0
            for b in rec["buckets"]:
                assert b["n_max"] > prev and b["band"] in (4, 8, 16)
                assert str(b["band"]) in b["ms"] and b["ms"][str(b["band"])] == min(b["ms"].values())
                prev = b["n_max"]
            assert prev >= 512


@pytest.mark.gpu
@pytest.mark.parametrize("table", ["tuned", [(64, 4), (200, 8), (512, 16)], [(512, 16)], [(100, 16), (512, 4)]])
def test_batched_with_band_table(oracle_mod, table):
    import torch
    import paper_1604_03703_amd as sbr
    print("batched table", table, flush=True)
    mats = si.batch_workload(count=40, lo=3, hi=512)
    refs = [oracle_mod.eigvalsh(M) for M in mats]
    plan = sbr.Plan(512, len(mats))
    if table == "tuned":
        used = plan.use_tuned_batch_bands()
        assert used, "no tuning stored for this device"
    else:
        plan.set_batch_bands(table)
    dev = [torch.from_numpy(M.copy()).cuda() for M in mats]
    ws = sbr.eigvalsh_batched(dev, b0=0, plan=plan)
    torch.cuda.synchronize()
    for M, w, ref in zip(mats, ws, refs):
        assert np.max(np.abs(w.cpu().numpy() - ref)) <= 1e-11 * _norm2(ref), M.shape[0]


@pytest.mark.gpu
def test_batch_band_table_rejects_malformed():
    import paper_1604_03703_amd as sbr
    plan = sbr.Plan(0, 4)
    with pytest.raises(sbr.SbrError):
        plan.set_batch_bands([(100, 8), (50, 16)])      # n_max not ascending
    with pytest.raises(sbr.SbrError):
        plan.set_batch_bands([(100, 12)])               # not a power of two
    with pytest.raises(sbr.SbrError):
        plan.set_batch_bands([(100, 32)])               # wider than the batched kernels take
    plan.set_batch_bands([])
