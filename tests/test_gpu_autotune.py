"""The autotuner's tables.  Batched form: the tuned band per size bucket is
well formed (CPU), and a batch solved with it, or with any valid table,
matches the oracle matrix by matrix (GPU).  Single-matrix path: the
shortest-path choice of the band-stage sequence equals brute force over
every sequence (CPU), the stored sequences are consistent with their
measured stage times (CPU), and solves with them match the oracle (GPU)."""
import itertools
import json
import os
import numpy as np
import pytest

import sbr_inputs as si


def _norm2(ref):
    return max(1e-300, float(np.max(np.abs(ref))))


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_tuning_database_is_well_formed():
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
                # the band is the fastest on the mixed batch where that
                # refinement ran, else on the bucket's own batch
                ms = b.get("mixed_ms", b["ms"])
                assert str(b["band"]) in ms and ms[str(b["band"])] == min(ms.values())
                prev = b["n_max"]
            assert prev >= 512


def test_coordinate_descent_separable_and_coupled():
    from paper_1604_03703_amd.autotune import coordinate_descent
    cands = (4, 8, 16)
    w = {4: [3.0, 1.0, 2.0], 8: [1.0, 2.0, 1.5], 16: [2.0, 3.0, 1.0]}   # per bucket, per band

    # separable cost: one pass reaches the brute-force optimum from any start
    def sep(bands):
        return sum(w[b][k] for k, b in enumerate(bands))

    full = min(itertools.product(cands, repeat=3), key=sep)
    for start in itertools.product(cands, repeat=3):
        calls = []
        bands, best, t0, tried = coordinate_descent(list(start), cands, lambda b: calls.append(tuple(b)) or sep(b))
        assert bands == list(full) and best == sep(full) and t0 == sep(start)
        # the start, then each other candidate once per bucket, last bucket first
        assert calls[0] == tuple(start) and len(calls) == 1 + 3 * 2
        assert [c for c in calls[1:3]] == [tuple(start[:2]) + (c,) for c in cands if c != start[2]]
        for k, t in enumerate(tried):
            assert t[str(bands[k])] == min(t.values())

    # coupled cost (a phase paid once for the whole batch if any bucket uses
    # b = 16): from [8, 8, 8] the pass moves the last bucket to 16 only if
    # that pays for the shared phase, and then the others follow
    def coupled(bands):
        return sep(bands) + (1.2 if 16 in bands else 0.0)

    bands, best, _, _ = coordinate_descent([8, 8, 8], cands, coupled)
    # bucket 2: 16 gives 1 + 2 + 1 + 1.2 = 5.2 < 4.5? no -> stays 8 (4.5);
    # bucket 1: 4 gives 1 + 1 + 1.5 = 3.5; bucket 0: 8 stays (1 is its best)
    assert bands == [8, 4, 8] and best == coupled([8, 4, 8]) == 3.5


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


def _all_sequences(ms, b0):
    # every chain b0 -> ... -> 1 through measured stages, by enumeration
    out = []
    def walk(b, acc, t):
        if b == 1:
            out.append((t, acc))
            return
        for (bb, h), v in ms.items():
            if bb == b:
                walk(h, acc + [h], t + v)
    walk(b0, [], 0.0)
    return out


def test_stage_sequence_is_the_shortest_path():
    from paper_1604_03703_amd import autotune
    import random
    rng = random.Random(3)
    for trial in range(50):
        ms = {k: rng.uniform(10, 300) for k in autotune.STAGE_PAIRS if rng.random() < 0.8 or k[1] == k[0] // 2}
        for b0 in (16, 32, 64, 128):
            widths, total = autotune.best_sequence(ms, b0)
            brute = min(_all_sequences(ms, b0))
            assert abs(total - brute[0]) < 1e-9
            assert abs(sum(ms[(b, h)] for b, h in zip([b0] + widths, widths)) - total) < 1e-9


def test_stage_table_is_well_formed():
    from paper_1604_03703_amd import autotune
    db = json.load(open(autotune.STAGE_DB))
    assert db, "no stage tuning stored"
    for arch, forms in db.items():
        for prec, per_n in forms.items():
            for n, rec in per_n.items():
                ms = {tuple(int(x) for x in k.split("->")): v for k, v in rec["ms"].items()}
                for b0, seq in rec["sequences"].items():
                    w = seq["widths"]
                    chain = [int(b0)] + w
                    assert w[-1] == 1 and all(x > y for x, y in zip(chain, w))
                    total = sum(ms[(b, h)] for b, h in zip(chain, w))
                    assert abs(total - seq["ms"]) < 1e-2
                    assert total <= min(t for t, _ in _all_sequences(ms, int(b0))) + 1e-2


@pytest.mark.gpu
@pytest.mark.parametrize("n,b0", [(3000, 128), (2000, 64), (1500, 32)])
def test_solver_with_tuned_stages(oracle_mod, n, b0):
    import torch
    import paper_1604_03703_amd as sbr
    A = si.gaussian_symmetric(n, si.make_rng(si.CFG_SMALL, 31))
    ref = oracle_mod.eigvalsh(A)
    plan = sbr.Plan(n)
    widths = plan.use_tuned_stages(n, b0)
    assert widths, "no stage tuning stored for this device"
    assert plan.band_stages(n, b0) == widths
    print("tuned stages n=%d b0=%d: %s" % (n, b0, widths), flush=True)
    w = sbr.eigvalsh(torch.from_numpy(A).cuda(), b0=b0, plan=plan)
    torch.cuda.synchronize()
    assert plan.status() == 0
    assert np.max(np.abs(w.cpu().numpy() - ref)) <= 1e-11 * _norm2(ref)
