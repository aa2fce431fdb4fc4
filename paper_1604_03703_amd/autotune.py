"""Autotuner of the batched form: the band width per matrix-size bucket.

The batched solver (`sbr_syev_eigvals_batched` with b0 = 0) reduces each
matrix to a band of width b in {4, 8, 16} before the halvings and the
bisection; which b is fastest depends on the order n (a wider band halves the
number of panels of the full-to-band step but adds a halving stage).  For
every size bucket this module times the captured batched launch on a batch of
synthetic matrices of that bucket (SCF-like: sorted diagonal in [-20, 5],
off-diagonal N(0, 0.1^2) exp(-|i-j|/20), symmetrised) with each candidate b,
and stores the winner per bucket in tuning/batched.json, keyed by the device
architecture and the precision form:

    {"gfx950": {"fp64": {"buckets": [{"n_max": 48, "band": 8, "ms": {...}}, ...]}}}

`batch_table()` reads it back as the (n_max, band) list that
`Plan.set_batch_bands` hands to the library; `eigvalsh_batched(b0=0)` applies
it to the plans it creates.  Run on the target GPU:

    python -m paper_1604_03703_amd.autotune [--count 1024] [--reps 5]
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
    db = _load_db(path)
    db.setdefault(arch, {})["fp64" if precision in ("fp64", 0) else "fp32_mfma"] = {
        "buckets": rec, "candidates": list(candidates), "reps": reps,
        "input": "SCF-like: sorted diagonal U[-20, 5], off-diagonal N(0, 0.1^2) exp(-|i-j|/20)",
    }
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
        f.write("\n")
    return db


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--count", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--db", default=DB)
    args = ap.parse_args()
    tune(args.precision, args.count, args.reps, args.warmup, args.db)
    print(json.dumps({"arch": device_arch(), "table": batch_table(args.precision, path=args.db)}))


if __name__ == "__main__":
    main()
