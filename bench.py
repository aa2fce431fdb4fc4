"""Benchmark of the SBR symmetric eigensolver on one MI355X.

One step = one whole solve of the hot path on one synthetic input already in
HBM: full-to-band (b0), band halvings b0 -> 1, Sturm bisection of all n
eigenvalues.  The input is restored from a pristine device copy before every
step (the solve overwrites it); that copy is outside the timed region, every
timed step is bracketed by device synchronisations.

Default workload: n = 32768, (G + G^T)/2 Gaussian, b0 = 128, FP64 form, then
the same input in the FP32-MFMA form, then the batched form (4096 SCF-like
matrices of orders 32 .. 512, one step = one call over the whole batch).  The
headline `value` is the full-to-band rate (4/3 n^3 flops over the
full-to-band time) of the FP64 form.

Prints ONE JSON line (rank 0).  `--gpus N` with N > 1 is refused: this
benchmark measures one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("full-to-band TFLOP/s (4/3·n³) + s/solve at n=32768 FP64 vs FP32; batch solves/s")
PEAK_FP64_MFMA = 78.6     # TFLOP/s, MI355X dense FP64 matrix
PEAK_FP32_MFMA = 157.3    # TFLOP/s, MI355X dense FP32 matrix
PEAK_HBM = 8000.0         # GB/s


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def band_stage_bytes(n: int, b: int, h: int | None = None) -> float:
    """Algorithmic bytes of one band stage b -> h (FP64; h = b/2 a halving):
    every chase reads and writes the entries it touches once (QR block b x h,
    left block b x (b - h), lower half of the diagonal block, below block),
    summed over all chases."""
    import numpy as np
    h = b // 2 if h is None else h
    total = 0
    for i in range(1, (n - 2) // h + 1):
        o = i * h + b * np.arange(0, (n - 2 - i * h) // b + 1, dtype=np.int64)
        nr = np.minimum(n - o, b)
        nbr = np.maximum(0, np.minimum(n, o + 2 * b) - (o + b))
        ent = nr * h + nr * (nr + 1) // 2 + nbr * b
        ent[1:] += nr[1:] * (b - h)      # left block for j > 1
        total += int(ent.sum())
    return 16.0 * total   # 8 B read + 8 B written per entry


def f2b_update_flops(n: int, b: int):
    """Per-panel algorithmic flops of the two dominant kernels: SYMM
    W = A22 Y (2 m^2 b) and the bulk lower-triangle SYR2K launch.  The trailing
    update of a panel with a next panel is split: the next panel's b columns
    first (not counted here), then the remaining m' = m - b rows and columns,
    2 b m' (m' + 1) flops; the last panel's update is one launch over m."""
    symm, syr2k = [], []
    k = 0
    while True:
        m = n - (k + 1) * b
        if m < b:
            break
        symm.append(2.0 * m * m * b)
        mr = m - b if m - b >= b else m
        syr2k.append(2.0 * b * mr * (mr + 1))
        k += 1
    return symm, syr2k


def measured_traffic(kernel_src: str):
    """HBM bytes per launch of the bulk SYR2K from the committed counter
    profile, or None when the kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "syr2k_lower_kernel_n32768_b128_traffic.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    rec = None
    for line in text.splitlines():
        if line.startswith("TRAFFIC "):
            rec = json.loads(line[len("TRAFFIC "):])
    if rec is None:
        return None
    src = open(os.path.join(ROOT, "paper_1604_03703_amd", "csrc", kernel_src), "rb").read()
    if hashlib.sha256(src).hexdigest() != rec.get("src_sha256"):
        return None
    return rec["bytes_per_launch"]


def run_form(sbr, torch, A0, n, b0, precision, steps, warmup, plan):
    A = torch.empty_like(A0)
    w = torch.empty(n, dtype=torch.float64, device=A0.device)
    stream = torch.cuda.current_stream()
    times, tims, wtims = [], [], []
    for it in range(warmup + steps):
        A.copy_(A0)
        torch.cuda.synchronize()
        # warmup steps record every event pair (the SYMM / SYR2K breakdown);
        # timed steps only the phase totals and the bulk SYR2K launches (the
        # roofline kernel): events around the SYMM sit on the critical path
        plan.set_timing(1 if it < warmup else 2)
        t0 = time.perf_counter()
        rc = sbr.lib().sbr_syev_eigvals_ex(plan.handle, n, sbr._dev_f64(A, "A"), n, b0, sbr._prec(precision),
                                           sbr._stream(stream), sbr._dev_f64(w, "w"))
        sbr._check(rc, "sbr_syev_eigvals_ex")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tm = plan.timing()
        log("%s step %d: %.1f ms (f2b %.1f, band %.1f, bisect %.1f) stages %s" % (
            precision, it, (t1 - t0) * 1e3, tm["ms_f2b"], tm["ms_band"], tm["ms_bisect"],
            ["%.1f" % x for x in tm["ms_stage"]]))
        st = plan.status()
        if st != 0:
            raise RuntimeError("the plan reported status bits %d (1: a band stage stalled, 2: non-finite)" % st)
        if it >= warmup:
            times.append(t1 - t0)
            tims.append(tm)
        else:
            wtims.append(tm)
    return times, tims, w, (wtims or tims)


def run_batch(sbr, torch, si, count, steps, warmup):
    """Batched form: `count` SCF-like matrices, n ~ U{32..512}; one step =
    one replay of the captured batched launch over all of them (inputs
    restored from pristine device copies outside the timed region)."""
    import numpy as np
    log("generating the batch of %d SCF-like matrices" % count)
    mats = si.batch_workload(count=count)
    dev0 = [torch.from_numpy(M).cuda() for M in mats]
    dev = [torch.empty_like(d) for d in dev0]
    ws = [torch.empty(d.shape[0], dtype=torch.float64, device=d.device) for d in dev0]
    out = {"count": count, "n_range": [int(min(M.shape[0] for M in mats)), int(max(M.shape[0] for M in mats))]}
    wsave = {}
    for prec in ("fp64", "fp32_mfma"):
        plan = sbr.Plan(512, count, prec)
        # band per size bucket: the form's own tuning table, else the FP64 one
        table = plan.use_tuned_batch_bands(prec) or plan.use_tuned_batch_bands("fp64")
        out.setdefault("tuned_bands", {})[prec] = [list(x) for x in table]
        # arguments marshalled once, as an SCF loop that refills the same
        # buffers would; each step is one call (one replay of the captured
        # launch), timed on the host clock around the call and a sync
        call = sbr.BatchedSolve(dev, precision=prec, plan=plan, out=ws)
        times = []
        for it in range(max(1, warmup) + steps):
            for d, d0 in zip(dev, dev0):
                d.copy_(d0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            call.run()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            log("batch %s step %d: %.2f ms" % (prec, it, (t1 - t0) * 1e3))
            if it >= max(1, warmup):
                times.append(t1 - t0)
        tm = mean(times)
        out[prec] = {"ms": round(tm * 1e3, 3), "solves_per_s": round(count / tm, 1)}
        wsave[prec] = [w.cpu().numpy() for w in ws[:256]]
        del call
        plan.close()
    # FP32-MFMA form against the FP64 form, matrix by matrix (first 256)
    errs = [float(np.max(np.abs(a - b)) / max(1e-300, float(np.max(np.abs(b)))))
            for a, b in zip(wsave["fp32_mfma"], wsave["fp64"])]
    out["fp32_mfma"]["err_vs_fp64_max_rel"] = max(errs)
    out["fp32_speedup"] = round(out["fp64"]["ms"] / out["fp32_mfma"]["ms"], 3)
    # the plain FP64 solver called once per matrix (one plan, the same stream)
    # on the first `plain` matrices: what the batched launch replaces
    plain = min(count, 512)
    plan = sbr.Plan(512, 0, "fp64")
    for d, d0 in zip(dev[:plain], dev0[:plain]):
        d.copy_(d0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for d, w in zip(dev[:plain], ws[:plain]):
        w.copy_(sbr.eigvalsh(d, precision="fp64", plan=plan, overwrite=True))
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    plan.close()
    out["plain_fp64_loop"] = {"count": plain, "solves_per_s": round(plain / tp, 1)}
    out["batched_speedup_vs_plain"] = round(out["fp64"]["solves_per_s"] / (plain / tp), 2)
    # every matrix's eigenvalues (batched FP64 form) sum to its trace (cheap
    # check at full size)
    tr = max(abs(float(w.sum()) - float(np.trace(M))) / max(1.0, float(np.abs(M).max()) * M.shape[0])
             for w, M in zip(wsave["fp64"][:64], mats[:64]))
    out["trace_check_rel"] = tr
    # roofline of the batch: sum over phases of max(flops / peak, bytes / BW)
    # with the method's own work: full-to-band 4/3 n^3 flops per matrix on
    # the FP64 MFMA peak, the halvings' band traffic (32 n^2 bytes per
    # stage) on HBM, and the bisection's n^2 I Sturm steps of 12 FP64 lane
    # operations (a reciprocal, its refinement, the recurrence) on the FP64
    # vector rate (78.6 TFLOP/s = 39.3 T lane-op/s)
    ns = [M.shape[0] for M in mats]
    t_f2b = sum(4.0 / 3.0 * m ** 3 for m in ns) / (PEAK_FP64_MFMA * 1e12)
    t_band = sum(32.0 * m * m * max(1, int(math.log2(max(2, min(16, m))))) for m in ns) / (PEAK_HBM * 1e9)
    t_bis = sum(m * m * 56 * 12 for m in ns) / 39.3e12
    t_roof = t_f2b + t_band + t_bis
    out["roofline"] = {"t_roof_ms": round(t_roof * 1e3, 3), "f2b_ms": round(t_f2b * 1e3, 3),
                       "band_ms": round(t_band * 1e3, 3), "bisect_ms": round(t_bis * 1e3, 3),
                       "frac": round(t_roof / (out["fp64"]["ms"] * 1e-3), 4)}
    return out


def mean(xs):
    return sum(xs) / max(1, len(xs))


def time_band_stage(sbr, torch, n, b, h, direct, variant, steps, warmup):
    """One band stage alone: a seeded random symmetric band of width b (lower
    band storage, ld 2b + 1) reduced to width h (sbr_band_reduce; h = b/2 by
    default) or, with direct, taken straight to the tridiagonal
    (sbr_band_to_tridiag, launch shape variant); the band is restored from a
    device copy before every launch (outside the timed region)."""
    h = 1 if direct else (h or b // 2)
    g = torch.Generator(device="cuda").manual_seed(1604 + b)
    ld = 2 * b + 1
    src = torch.zeros((n, ld), dtype=torch.float64, device="cuda")
    src[:, : b + 1] = torch.randn((n, b + 1), dtype=torch.float64, device="cuda", generator=g)
    for d in range(1, b + 1):
        src[n - d:, d] = 0.0
    plan = sbr.Plan(0)
    plan.set_tridiag_band(0, variant)
    bd = torch.empty_like(src)
    ms = []
    for it in range(warmup + steps):
        bd.copy_(src)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        if direct:
            sbr.band_to_tridiag(bd, b, plan)
        else:
            sbr.band_reduce(bd, b, h, plan)
        e1.record()
        torch.cuda.synchronize()
        if plan.status() != 0:
            raise RuntimeError("band stage reported a stalled wait")
        if it >= warmup:
            ms.append(e0.elapsed_time(e1))
    by = band_stage_bytes(n, b, h)
    out = {"n": n, "b": b, "stage": "%d->%d" % (b, h),
           "variant": variant if direct else None, "ms": [round(x, 3) for x in ms]}
    out["alg_GB"] = round(by / 1e9, 3)
    out["GBps"] = round(by / (mean(ms) * 1e-3) / 1e9, 1)
    plan.close()
    return out


def golden_eigenvalues(A_host, n):
    """The oracle's eigenvalues of this exact input, stored by
    tests/golden/make_oracle_golden.py (None when there is no file for n or
    the matrix bytes differ from the ones the values were computed on)."""
    import hashlib
    import numpy as np
    gdir = os.path.join(ROOT, "tests", "golden")
    try:
        meta = json.load(open(os.path.join(gdir, "oracle_golden.json")))
    except OSError:
        return None
    rec = meta.get("n%d" % n)
    if rec is None:
        return None
    h = hashlib.sha256()
    rows = max(1, (1 << 24) // n)
    for r0 in range(0, n, rows):
        h.update(np.ascontiguousarray(A_host[r0:r0 + rows]).tobytes())
    if h.hexdigest() != rec["matrix_sha256"]:
        log("golden eigenvalues are for another matrix (hash differs): not used")
        return None
    return np.load(os.path.join(gdir, rec["file"]))


def err_vs(w, ref):
    import numpy as np
    d = np.abs(w - ref)
    nrm = float(np.max(np.abs(ref)))
    return {"max_rel": float(d.max() / nrm), "rms_rel": float(math.sqrt(float(np.mean(d * d))) / nrm)}


def cpu_baseline(A_host, n_sample: int):
    import oracle
    oracle.build()
    S = A_host[:n_sample, :n_sample].copy()
    t0 = time.perf_counter()
    d, e = oracle.tridiagonalize(S)
    t1 = time.perf_counter()
    oracle.tridiag_eigvals(d, e)
    t2 = time.perf_counter()
    tflops = (4.0 / 3.0) * n_sample ** 3 / (t1 - t0) / 1e12
    return {
        "value": tflops,
        "unit": "TFLOP/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": ("Householder tridiagonalisation (4/3 n^3 flops) of the leading %dx%d block of the "
                   "same input; %.2f s, plus %.2f s of bisection for its %d eigenvalues; host %s"
                   % (n_sample, n_sample, t1 - t0, t2 - t1, n_sample, platform.processor() or platform.machine())),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--b0", type=int, default=128)
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--batch-only", action="store_true",
                    help="only run the batched form and print its results (profiling)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run three device-to-device copies of MIB MiB (counter calibration) and exit")
    ap.add_argument("--band-stage", type=int, default=0, metavar="B",
                    help="only time one band stage of width B on a seeded random band of order --n "
                         "(to width --to, a halving by default, or with --direct straight to tridiagonal) and exit")
    ap.add_argument("--to", type=int, default=0, metavar="H", help="with --band-stage: the width to reduce to")
    ap.add_argument("--direct", action="store_true", help="with --band-stage: the direct B -> 1 stage")
    ap.add_argument("--variant", type=int, default=0, help="with --band-stage --direct: launch shape")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the eigensolver here runs on a single device "
              "(no sharding, no collectives); run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_probe > 0:
        nbytes = args.copy_probe << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": nbytes, "copies": 3}), flush=True)
        return

    import sbr_inputs as si
    import paper_1604_03703_amd as sbr

    if args.band_stage:
        print(json.dumps(time_band_stage(sbr, torch, args.n, args.band_stage, args.to, args.direct, args.variant,
                                         args.steps, args.warmup)), flush=True)
        return

    if args.batch_only:
        print(json.dumps({"batch": run_batch(sbr, torch, si, args.batch_count, args.steps, args.warmup)}), flush=True)
        return

    n, b0 = args.n, args.b0
    cfg = si.CFG_LARGE if n == 32768 else si.CFG_MEDIUM
    log("generating n=%d Gaussian input (seeded)" % n)
    t0 = time.perf_counter()
    A_host = si.gaussian_symmetric(n, si.make_rng(cfg, 0))
    log("generated in %.1f s" % (time.perf_counter() - t0))
    dev = torch.device("cuda:0")
    A0 = torch.from_numpy(A_host).to(dev)
    trace = float(np.trace(A_host))
    fro2 = float(np.sum(A_host * A_host))

    plan = sbr.Plan(n, 0, "fp64")
    # band-stage sequence: the autotuner's table for this device when there
    # is one (tuning/stages.json), else the library's built-in choice
    stage_src = "tuned" if plan.use_tuned_stages(n, b0, "fp64") else "built-in"
    widths = plan.band_stages(n, b0)
    times, tims, w, btims = run_form(sbr, torch, A0, n, b0, "fp64", args.steps, args.warmup, plan)
    wh = w.cpu().numpy()
    # properties that hold at any size: sum of eigenvalues = trace, sum of squares = ||A||_F^2
    tr_err = abs(wh.sum() - trace) / math.sqrt(fro2)
    fr_err = abs(float(np.sum(wh * wh)) - fro2) / fro2
    f2b_ms = mean([t["ms_f2b"] for t in tims])
    band_ms = mean([t["ms_band"] for t in tims])
    bis_ms = mean([t["ms_bisect"] for t in tims])
    ms_per_step = 1e3 * mean(times)
    f2b_flops = (4.0 / 3.0) * n ** 3
    value = f2b_flops / (f2b_ms * 1e-3) / 1e12

    # dominant kernel roofline: whichever of SYMM / SYR2K took longer in total
    # (the per-kernel breakdown comes from the warmup steps, which record every
    # event pair; the timed steps record the bulk SYR2K pairs only)
    symm_f, syr2k_f = f2b_update_flops(n, b0)
    syr2k_ms = mean([t["ms_syr2k"] for t in btims])
    symm_ms = mean([t["ms_symm"] for t in btims])
    if syr2k_ms >= symm_ms:
        # the bulk launches on 128 x 128 tiles (`syr2k_lower_kernel<double, 128, ...>`,
        # the first ones: the last, small trailing matrices run on 64 x 64 tiles)
        nbig = int(tims[-1]["syr2k_big_launches"])
        kname = "syr2k_lower_kernel<double, 128, 2, 4> (bulk trailing update)"
        kflops, klaunch = sum(syr2k_f[:nbig]), nbig
        kms = mean([t["ms_syr2k_big"] for t in tims])
        traffic = measured_traffic("sbr_gemm.hip")
    else:
        kname, kflops, kms, klaunch = "symm_lower_kernel", sum(symm_f), symm_ms, len(symm_f)
        traffic = None
    achieved = kflops / (kms * 1e-3) / 1e12 if kms > 0 else 0.0
    stage_ms = [mean([t["ms_stage"][i] for t in tims]) for i in range(len(tims[0]["ms_stage"]))]
    stages = []
    b = b0
    band_bytes = 0.0
    for sms, h in zip(stage_ms, widths):
        by = band_stage_bytes(n, b, h)
        band_bytes += by
        gbps = by / (sms * 1e-3) / 1e9 if sms > 0 else None
        stages.append({"b": b, "h": h, "ms": round(sms, 3), "alg_GB": round(by / 1e9, 3),
                       "GBps": round(gbps, 1) if gbps else None,
                       "frac_hbm": round(gbps / PEAK_HBM, 4) if gbps else None})
        b = h

    result = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "symmetric eigenvalues, n=%d (G+G^T)/2 Gaussian, full-to-band b0=%d, "
                               "band stages %s, Sturm bisection (all n), FP64"
                               % (n, b0, "->".join(str(x) for x in [b0] + widths)),
                   "n": n, "b0": b0},
        "s_per_solve": round(ms_per_step / 1e3, 4),
        "phases_ms": {"f2b": round(f2b_ms, 3), "band": round(band_ms, 3), "bisect": round(bis_ms, 3)},
        "f2b_kernels_ms": {"symm": round(symm_ms, 3), "syr2k": round(syr2k_ms, 3),
                           "symm_TFLOPs": round(sum(symm_f) / (symm_ms * 1e-3) / 1e12, 2) if symm_ms > 0 else None,
                           "syr2k_TFLOPs": round(sum(syr2k_f) / (syr2k_ms * 1e-3) / 1e12, 2) if syr2k_ms > 0 else None,
                           "panel_and_other": round(mean([t["ms_f2b"] for t in btims]) - symm_ms - syr2k_ms, 3),
                           "measured_in": "warmup steps (every event pair recorded)"},
        "band_stages": stages,
        "band_stage_source": stage_src,
        "band_GBps_alg": round(band_bytes / (band_ms * 1e-3) / 1e9, 1) if band_ms > 0 else None,
        "checks": {"trace_rel": tr_err, "frobenius_rel": fr_err},
        "band_frac_hbm": round(band_bytes / (band_ms * 1e-3) / 1e9 / PEAK_HBM, 4) if band_ms > 0 else None,
        "roofline": {"bound": "mfma", "kernel": kname, "achieved": round(achieved, 3),
                     "peak": PEAK_FP64_MFMA, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_MFMA, 4),
                     "traffic": traffic, "launches": klaunch, "avg_launch_ms": round(kms / max(1, klaunch), 4)},
    }

    golden = golden_eigenvalues(A_host, n)
    if golden is not None:
        result["checks"]["fp64_vs_oracle"] = err_vs(wh, golden)
    # the FP64 plan's streams (side + CU-masked) go before the FP32 plan
    # creates its own: the process has four hardware queues
    plan.close()
    del plan

    if not args.no_fp32:
        plan32 = sbr.Plan(n, 0, "fp32_mfma")
        if not plan32.use_tuned_stages(n, b0, "fp32_mfma"):
            plan32.use_tuned_stages(n, b0, "fp64")
        t32, tim32, w32, wt32 = run_form(sbr, torch, A0, n, b0, "fp32_mfma", args.steps, args.warmup, plan32)
        f2b32 = mean([t["ms_f2b"] for t in tim32])
        d = np.abs(w32.cpu().numpy() - wh)
        norm2 = float(np.max(np.abs(wh)))
        result["fp32_mfma"] = {
            "f2b_TFLOPs": round(f2b_flops / (f2b32 * 1e-3) / 1e12, 4),
            "s_per_solve": round(mean(t32) , 4),
            "phases_ms": {"f2b": round(f2b32, 3), "band": round(mean([t["ms_band"] for t in tim32]), 3),
                          "bisect": round(mean([t["ms_bisect"] for t in tim32]), 3)},
            "err_vs_fp64_max_rel": float(d.max() / norm2),
            "err_vs_fp64_rms_rel": float(math.sqrt(float(np.mean(d * d))) / norm2),
            "speedup_f2b": round(f2b_ms / f2b32, 3) if f2b32 > 0 else None,
            "speedup_solve": round(mean(times) / mean(t32), 3),
            "speedup_band": round(band_ms / mean([t["ms_band"] for t in tim32]), 3),
            "band_stage_widths": plan32.band_stages(n, b0),
            "band_stage_ms": [round(mean([t["ms_stage"][i] for t in tim32]), 3)
                              for i in range(len(tim32[0]["ms_stage"]))],
        }
        # the FP32 trailing-update kernels against the FP32 MFMA peak (same
        # bookkeeping as the FP64 roofline: warmup steps give the SYMM /
        # SYR2K split, the timed steps the bulk SYR2K launches)
        symm32 = mean([t["ms_symm"] for t in wt32])
        syr2k32 = mean([t["ms_syr2k"] for t in wt32])
        nbig32 = int(tim32[-1]["syr2k_big_launches"])
        kms32 = mean([t["ms_syr2k_big"] for t in tim32])
        ach32 = sum(syr2k_f[:nbig32]) / (kms32 * 1e-3) / 1e12 if kms32 > 0 else 0.0
        result["fp32_mfma"]["f2b_kernels_ms"] = {
            "symm": round(symm32, 3), "syr2k": round(syr2k32, 3),
            "symm_TFLOPs": round(sum(symm_f) / (symm32 * 1e-3) / 1e12, 2) if symm32 > 0 else None,
            "syr2k_TFLOPs": round(sum(syr2k_f) / (syr2k32 * 1e-3) / 1e12, 2) if syr2k32 > 0 else None,
            "panel_and_other": round(mean([t["ms_f2b"] for t in wt32]) - symm32 - syr2k32, 3)}
        result["fp32_mfma"]["roofline"] = {
            "bound": "mfma", "kernel": "syr2k_lower_kernel<float, 128, 2, 4, 2, float, true, float> (bulk trailing update, "
                                       "FP32 storage and operands)",
            "achieved": round(ach32, 3), "peak": PEAK_FP32_MFMA, "unit": "TFLOP/s",
            "frac": round(ach32 / PEAK_FP32_MFMA, 4), "traffic": None, "launches": nbig32,
            "avg_launch_ms": round(kms32 / max(1, nbig32), 4)}
        if golden is not None:
            result["fp32_mfma"]["err_vs_oracle"] = err_vs(w32.cpu().numpy(), golden)
        plan32.close()
        del plan32

    if not args.no_batch:
        result["batch"] = run_batch(sbr, torch, si, args.batch_count, args.steps, args.warmup)

    if not args.no_cpu:
        log("timing the CPU oracle on a %d sample" % args.cpu_sample)
        result["cpu_baseline"] = cpu_baseline(A_host, min(args.cpu_sample, n))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
