"""Autotuner of the batched form: the band width per matrix-size bucket.

The batched solver (`sbr_syev_eigvals_batched` with b0 = 0) reduces each
matrix to a band of width b in {4, 8, 16} before the halvings and the
bisection; which b is fastest depends on the order n (a wider band halves the
number of panels of the full-to-band step but adds a halving stage).  For
every size bucket this module times the captured batched launch on a batch of
synthetic matrices of that bucket (SCF-like: sorted diagonal in [-20, 5],
off-diagonal N(0, 0.1^2) exp(-|i-j|/20), symmetrised) with each candidate b,
and keeps the fastest per bucket.  The phases of a batched call run as
separate kernels over the whole batch, so bucket times measured alone do not
add up to the time of a mixed batch: the per-bucket choice is then refined on
a batch whose orders span every bucket, one bucket at a time (each other
candidate tried with the other buckets' bands fixed, a change kept when the
whole batch gets faster), largest bucket first.  The result is stored in
tuning/batched.json, keyed by the device architecture and the precision form:

    {"gfx950": {"fp64": {"buckets": [{"n_max": 48, "band": 8, "ms": {...}}, ...]}}}

`batch_table()` reads it back as the (n_max, band) list that
`Plan.set_batch_bands` hands to the library; `eigvalsh_batched(b0=0)` applies
it to the plans it creates.  Run on the target GPU:

    python -m paper_1604_03703_amd.autotune [--count 1024] [--reps 5]

The single-matrix path has a second table, tuning/stages.json: the band
widths of its band-to-band stages (the k of each stage of Algorithm 4.3)
and the launch shape of the direct band-to-tridiagonal stage.  For an order
n, `tune_stages` times every stage b -> h the library has a kernel for on a
seeded random band of that order (each direct b -> 1 stage in each launch
shape) and picks, for every starting band b0, the sequence b0 -> ... -> 1
with the least total time (a shortest path over the measured stages):

    python -m paper_1604_03703_amd.autotune --stages [--n 8192 16384 32768]
"""
from __future__ import annotations

import argparse
import json
import os
import time

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
DB = os.path.join(_PKG, "tuning", "batched.json")

BUCKETS = (48, 96, 160, 256, 384, 512)     # upper orders of the size buckets
CANDIDATES = (4, 8, 16)


def device_arch(device: int = 0) -> str:
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def _load_db(path: str = DB) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except OSError:
        return {}


def batch_table(precision="fp64", arch: str | None = None, path: str = DB) -> list:
    """(n_max, band) pairs of the stored tuning for this device, ascending."""
    prec = "fp64" if precision in ("fp64", 0) else "fp32_mfma"
    if arch is None:
        if not torch.cuda.is_available():
            return []
        arch = device_arch()
    rec = _load_db(path).get(arch, {}).get(prec)
    if not rec:
        return []
    return [(int(b["n_max"]), int(b["band"])) for b in rec["buckets"]]


def scf_batch(count: int, lo: int, hi: int, seed: int, device="cuda") -> list:
    """`count` SCF-like symmetric matrices with orders uniform in [lo, hi]."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    sizes = torch.randint(lo, hi + 1, (count,), generator=g).tolist()
    gd = torch.Generator(device=device).manual_seed(seed)
    out = []
    for m in sizes:
        i = torch.arange(m, device=device, dtype=torch.float64)
        decay = torch.exp(-(i[:, None] - i[None, :]).abs() / 20.0)
        M = 0.1 * torch.randn((m, m), dtype=torch.float64, device=device, generator=gd) * decay
        A = 0.5 * (M + M.T)
        d = torch.sort(torch.rand(m, dtype=torch.float64, device=device, generator=gd) * 25.0 - 20.0).values
        A.diagonal().copy_(d)
        out.append(A.contiguous())
    return out


def time_batch(sbr, mats, band: int, precision: str, reps: int, warmup: int) -> float:
    """Median ms of the batched call (its captured launch replayed) with
    every matrix on band width `band`; inputs restored between calls."""
    plan = sbr.Plan(max(int(m.shape[0]) for m in mats), len(mats), precision)
    work = [torch.empty_like(m) for m in mats]
    ws = [torch.empty(m.shape[0], dtype=torch.float64, device=m.device) for m in mats]
    ts = []
    for it in range(warmup + reps):
        for w_, m in zip(work, mats):
            w_.copy_(m)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sbr.eigvalsh_batched(work, b0=band, precision=precision, plan=plan, out=ws)
        torch.cuda.synchronize()
        if it >= warmup:
            ts.append(time.perf_counter() - t0)
    plan.close()
    ts.sort()
    return 1e3 * ts[len(ts) // 2]


def time_batch_table(sbr, mats, table, precision: str, reps: int, warmup: int) -> float:
    """Median ms of one replay of the captured batched launch with the band
    table `table` ((n_max, band) pairs); inputs restored between replays."""
    plan = sbr.Plan(max(int(m.shape[0]) for m in mats), len(mats), precision)
    plan.set_batch_bands(table)
    work = [torch.empty_like(m) for m in mats]
    ws = [torch.empty(m.shape[0], dtype=torch.float64, device=m.device) for m in mats]
    call = sbr.BatchedSolve(work, 0, precision, plan, ws)
    ts = []
    for it in range(warmup + reps):
        for w_, m in zip(work, mats):
            w_.copy_(m)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        call.run()
        torch.cuda.synchronize()
        if it >= warmup:
            ts.append(time.perf_counter() - t0)
    del call
    plan.close()
    ts.sort()
    return 1e3 * ts[len(ts) // 2]


def coordinate_descent(bands: list, candidates, run, log=None):
    """One pass of coordinate descent over the buckets, last (largest) first:
    for bucket k every other candidate is timed with the other buckets fixed
    (`run(bands) -> ms`), and a change is kept when it is faster than the
    best so far.  Returns (bands, best ms, start ms, the times tried per
    bucket as {band: ms})."""
    bands = list(bands)
    start = best = run(bands)
    tried_all = [None] * len(bands)
    for k in reversed(range(len(bands))):
        cur = bands[k]                # the band the bucket had when its turn came
        tried = {str(cur): round(best, 4)}
        for c in candidates:
            if c == cur:
                continue
            trial = list(bands)
            trial[k] = c
            t = run(trial)
            tried[str(c)] = round(t, 4)
            if log:
                log(k, c, t)
            if t < best:
                best, bands = t, trial
        tried_all[k] = tried
    return bands, best, start, tried_all


def refine_mixed(sbr, rec: list, precision: str, count: int, reps: int, warmup: int, candidates=CANDIDATES,
                 lo: int = 32, log=print) -> dict:
    """Coordinate descent of the bucket bands on one mixed batch (orders
    uniform in [lo, largest bucket], the SCF-like size mix); updates rec in
    place, returns a summary."""
    mats = scf_batch(count, lo, int(rec[-1]["n_max"]), seed=1704)

    def run(bs):
        return time_batch_table(sbr, mats, [(int(r["n_max"]), b) for r, b in zip(rec, bs)], precision, reps, warmup)

    def note(k, c, t):
        log("mixed batch, bucket n <= %d at b = %d: %.3f ms" % (rec[k]["n_max"], c, t))

    first = [int(r["band"]) for r in rec]
    bands, best, start, tried = coordinate_descent(first, candidates, run, note)
    log("mixed batch (%d matrices): per-bucket choice %s %.3f ms, refined %s %.3f ms"
        % (count, first, start, bands, best))
    for r, b, t in zip(rec, bands, tried):
        r["band"] = b
        r["mixed_ms"] = t
    del mats
    return {"count": count, "orders": [lo, int(rec[-1]["n_max"])], "ms_per_bucket_choice": round(start, 4),
            "ms": round(best, 4)}


def tune(precision="fp64", count: int = 1024, reps: int = 5, warmup: int = 2, path: str = DB,
         buckets=BUCKETS, candidates=CANDIDATES, log=print) -> dict:
    import paper_1604_03703_amd as sbr
    arch = device_arch()
    rec = []
    lo = 1
    for k, hi in enumerate(buckets):
        mats = scf_batch(count, max(lo, 3), hi, seed=1604 + k)
        ms = {}
        for b in candidates:
            ms[b] = time_batch(sbr, mats, b, precision, reps, warmup)
            log("bucket n <= %d, b = %d: %.3f ms (%d matrices)" % (hi, b, ms[b], count))
        best = min(ms, key=ms.get)
        rec.append({"n_min": lo, "n_max": hi, "band": best, "count": count,
                    "ms": {str(b): round(t, 4) for b, t in ms.items()}})
        lo = hi + 1
        del mats
    mixed = refine_mixed(sbr, rec, precision, 4 * count, reps, warmup, candidates, log=log)
    db = _load_db(path)
    db.setdefault(arch, {})["fp64" if precision in ("fp64", 0) else "fp32_mfma"] = {
        "buckets": rec, "candidates": list(candidates), "reps": reps, "mixed": mixed,
        "input": "SCF-like: sorted diagonal U[-20, 5], off-diagonal N(0, 0.1^2) exp(-|i-j|/20)",
    }
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
        f.write("\n")
    return db


# ---- band-to-band stage sequence of the single-matrix path ----------------

STAGE_DB = os.path.join(_PKG, "tuning", "stages.json")
# every (b, h) with a kernel: halvings, b -> b/k on the wide-band MFMA chase
# (h >= 8) and the direct b -> 1 stages
STAGE_PAIRS = ((128, 64), (128, 32), (128, 16), (64, 32), (64, 16), (64, 8), (32, 16), (32, 8), (16, 8),
               (8, 4), (4, 2), (2, 1), (4, 1), (8, 1), (16, 1))
TRI_VARIANTS = 3


def time_stage(sbr, n: int, b: int, h: int, reps: int = 2, warmup: int = 1, variant: int = 0,
               precision="fp64") -> float:
    """Median ms of one band stage b -> h on a seeded random band of order n
    (band restored from a device copy before every launch)."""
    g = torch.Generator(device="cuda").manual_seed(1604 + b)
    ld = 2 * b + 1
    src = torch.zeros((n, ld), dtype=torch.float64, device="cuda")
    src[:, : b + 1] = torch.randn((n, b + 1), dtype=torch.float64, device="cuda", generator=g)
    for d in range(1, b + 1):
        src[n - d:, d] = 0.0
    plan = sbr.Plan(0)
    plan.set_tridiag_band(0, variant)
    bd = torch.empty_like(src)
    ts = []
    for it in range(warmup + reps):
        bd.copy_(src)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        sbr.band_reduce(bd, b, h, plan, precision=precision)
        e1.record()
        torch.cuda.synchronize()
        if plan.status() != 0:
            raise RuntimeError("band stage %d -> %d reported a stalled wait" % (b, h))
        if it >= warmup:
            ts.append(e0.elapsed_time(e1))
    plan.close()
    ts.sort()
    return ts[len(ts) // 2]


def best_sequence(ms: dict, b0: int):
    """Fastest b0 -> ... -> 1 over the measured stages ms[(b, h)] (a shortest
    path on the powers of two); (widths after each stage, total ms)."""
    best = {1: (0.0, [])}
    b = 2
    while b <= b0:
        cands = [(ms[(b, h)] + best[h][0], [h] + best[h][1]) for (bb, h) in ms if bb == b and h in best]
        if cands:
            best[b] = min(cands, key=lambda c: c[0])
        b *= 2
    if b0 not in best:
        return None, None
    return best[b0][1], best[b0][0]


def tune_stages(ns=(8192, 16384, 32768), reps: int = 2, warmup: int = 1, precision="fp64", path: str = STAGE_DB,
                log=print) -> dict:
    import paper_1604_03703_amd as sbr
    arch = device_arch()
    prec = "fp64" if precision in ("fp64", 0) else "fp32_mfma"
    db = _load_db(path)
    rec = db.setdefault(arch, {}).setdefault(prec, {})
    for n in ns:
        ms, variant = {}, {}
        for b, h in STAGE_PAIRS:
            if b >= n:
                continue
            if h == 1 and b > 2:
                per = [time_stage(sbr, n, b, h, reps, warmup, v, precision) for v in range(TRI_VARIANTS)]
                variant[b] = min(range(TRI_VARIANTS), key=lambda v: per[v])
                ms[(b, h)] = per[variant[b]]
                log("n = %d: %d -> 1: %s ms (launch shapes 0..%d)" % (n, b, ["%.2f" % x for x in per],
                                                                      TRI_VARIANTS - 1))
            else:
                ms[(b, h)] = time_stage(sbr, n, b, h, reps, warmup, 0, precision)
                log("n = %d: %d -> %d: %.2f ms" % (n, b, h, ms[(b, h)]))
        seqs = {}
        for b0 in (16, 32, 64, 128):
            widths, total = best_sequence(ms, b0)
            if widths:
                direct = [b for b, h in zip([b0] + widths, widths) if h == 1 and b > 2]
                seqs[str(b0)] = {"widths": widths, "ms": round(total, 3),
                                 "tri_variant": variant.get(direct[0], 0) if direct else 0}
                log("n = %d, b0 = %d: %s (%.1f ms)" % (n, b0, " -> ".join(str(x) for x in [b0] + widths), total))
        rec[str(n)] = {"ms": {"%d->%d" % k: round(v, 3) for k, v in ms.items()},
                       "tri_variant": {str(k): v for k, v in variant.items()}, "sequences": seqs,
                       "reps": reps}
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
        f.write("\n")
    return db


def stage_sequence(n: int, b0: int, precision="fp64", arch: str | None = None, path: str = STAGE_DB):
    """(widths, launch shape of the direct stage) tuned for the stored order
    nearest to n (by ratio) and this b0; ([], 0) when there is none."""
    import math
    prec = "fp64" if precision in ("fp64", 0) else "fp32_mfma"
    if arch is None:
        if not torch.cuda.is_available():
            return [], 0
        arch = device_arch()
    rec = _load_db(path).get(arch, {}).get(prec) or {}
    best = None
    for key, r in rec.items():
        if str(b0) not in r.get("sequences", {}):
            continue
        d = abs(math.log(max(n, 2) / int(key)))
        if best is None or d < best[0]:
            best = (d, r["sequences"][str(b0)])
    if best is None:
        return [], 0
    return list(best[1]["widths"]), int(best[1]["tri_variant"])


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--count", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--db", default=None)
    ap.add_argument("--stages", action="store_true", help="tune the band-stage sequence of the single-matrix path")
    ap.add_argument("--n", type=int, nargs="*", default=[8192, 16384, 32768])
    args = ap.parse_args()
    if args.stages:
        path = args.db or STAGE_DB
        tune_stages(args.n, reps=min(args.reps, 3), warmup=1, precision=args.precision, path=path)
        print(json.dumps({"arch": device_arch(),
                          "sequences": {n: stage_sequence(n, 128, args.precision, path=path) for n in args.n}}))
        return
    path = args.db or DB
    tune(args.precision, args.count, args.reps, args.warmup, path)
    print(json.dumps({"arch": device_arch(), "table": batch_table(args.precision, path=path)}))


if __name__ == "__main__":
    main()
