"""Benchmark of the FDAS correlation step on one MI355X.

A step is one call of the hot path (segment load, forward FFT, per-template
product + inverse FFT, overlap discard, |.|^2 store) over the whole input of
the workload. The default workload is the paper-scale plain-FP32 one (2^21
bins, z in [-100, 100] step 2 -> 101 templates of width 256, segment FFT
2048) producing the 101 x 2^21 FP32 power plane (847 MB). Inputs are resident
in device memory before the timed region; the plan (templates, bank) is
built once outside it and its time is reported separately. The same run also
times the FP16 matrix-core form on the same input ("compare").

Other workloads (--workload): fp32-small, mixed-paper, batch-fp32 (512 series
of uneven length, per-series zmax, one graph-captured launch per wave),
batch-mixed-wide (256 series, z in [-200, 200], m 512, run in waves that fit
device memory).

Prints ONE JSON line. `value` is z-r plane points per second; `roofline`
prices the dominant kernel's algorithmic bytes per launch (4 B per plane
point written + 8 B per input bin read) against the 8 TB/s HBM peak, with
the kernel time measured by HIP events on the stream the kernel runs on;
`cpu_baseline` times the FP64 oracle on a bounded sample of the same input.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=200,
                    help="untimed steps first (the GPU clock needs tens of ms of load "
                         "to reach its steady state)")
    ap.add_argument("--workload", default="fp32-paper")
    ap.add_argument("--variant", default=None, help="force a compiled kernel variant")
    ap.add_argument("--zpb", type=int, default=None, help="templates per work unit")
    ap.add_argument("--precision", default=None, help="override the workload precision")
    ap.add_argument("--seg-len", type=int, default=None)
    ap.add_argument("--split", action="store_true",
                    help="mixed precisions: hi + lo split products (FDAS_FLAG_SPLIT)")
    ap.add_argument("--interbin", action="store_true",
                    help="also the half-bin rows (FDAS_FLAG_INTERBIN): 2 nz rows per plane")
    ap.add_argument("--candidates", type=float, default=None, metavar="THR",
                    help="single series: detection epilogue (points with power >= THR "
                         "listed) instead of writing the plane")
    ap.add_argument("--nseries", type=int, default=None, help="batched: first N series only")
    ap.add_argument("--wave-gb", type=float, default=100.0,
                    help="batched: device memory budget for the planes of one wave")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-bins", type=int, default=1 << 20)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (for "
                         "scaling HBM byte counters) and exit")
    return ap.parse_args()


def traffic_from_profiles(kernel: str, workload: str):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on this exact kernel variant, workload and kernel source (else None)."""
    from paper_1711_10855_amd.profile_summary import source_hash
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rows = json.load(f)
    except (OSError, ValueError):
        return None
    h = source_hash()
    for row in rows:
        if (row.get("kernel") == kernel and row.get("workload") == workload
                and row.get("source_hash") == h):
            return row.get("bytes_per_launch")
    return None


def cpu_baseline(a, zmax, dz, m, nz, sample_bins: int, checks=()):
    """The FP64 oracle (unchanged) on the first `sample_bins` bins, all rows.

    `checks`: (name, plane, first_row, row_step, bar) with `plane` the GPU
    result's first `sample_bins` columns (rows first_row, first_row +
    row_step, ... of the oracle's rows); each gets max |P - P_ref| / max P_ref
    over the columns that do not depend on bins beyond the sample."""
    import numpy as np

    import oracle
    sample = np.ascontiguousarray(a[:sample_bins])
    t0 = time.perf_counter()
    p = oracle.plane_direct(sample, zmax, dz, m)
    dt = time.perf_counter() - t0
    pts = p.shape[0] * p.shape[1]
    base = {"value": pts / dt, "unit": "points/s", "cores": 1, "kind": "oracle",
            "sample": f"{nz} rows x first {sample_bins} bins of the input spectrum "
                      f"({pts} points, {dt:.1f} s, single process NumPy FP64 direct sum)"}
    errors = {}
    ncol = sample_bins - m // 2
    for name, plane, r0, step, bar in checks:
        rows = plane.shape[0] // step
        ref = p[r0:r0 + rows, :ncol]
        got = plane[::step][:rows, :ncol].astype(np.float64)
        err = float(np.max(np.abs(got - ref)) / np.max(ref))
        errors[name] = {"max_abs_err_over_max_ref": err, "bar": bar, "pass": err <= bar,
                        "points": int(ref.size),
                        "sample": f"{rows} rows x first {ncol} bins, against the oracle above"}
    return base, errors


def _time(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(steps):
        fn()
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(stop) / steps, wall


def run_single(a_dev, zmax, dz, m, seg_len, prec, steps, warmup, flags=0, cand_thr=None,
               keep_cols=0):
    """Time fdas_convolve (or the candidate epilogue) on one resident
    spectrum; returns a result dict (with the plane's first `keep_cols`
    columns, copied to the host after the timing, as "check")."""
    import torch

    from paper_1711_10855_amd import fdas
    plan = fdas.Plan(zmax, dz, m, seg_len, prec, flags, device=0)
    info = plan.info
    nz, nbins = info.nz, a_dev.numel()
    stream = torch.cuda.current_stream(a_dev.device)
    ncand = None
    if cand_thr is None:
        out = torch.empty((nz, nbins), dtype=torch.float32, device=a_dev.device)
        ms, wall = _time(lambda: plan.convolve(a_dev, out=out), steps, warmup, stream)
        check = out[:, :keep_cols].cpu().numpy() if keep_cols else None
        del out
    else:
        buf = plan.candidates(a_dev, cand_thr, capacity=1 << 20)
        ms, wall = _time(lambda: plan.candidates(a_dev, cand_thr, buf=buf), steps, warmup, stream)
        ncand = int(buf[1].cpu()[0])
        check = None
    info = plan.get_info()  # templates per unit as the timed launches chose them
    plan.close()
    points = nz * nbins
    bytes_launch = (4.0 * points if cand_thr is None else 16.0 * ncand) + 8.0 * nbins
    return {"points": points, "nz": nz, "nbins": nbins, "ms": ms, "wall": wall,
            "value": points / (ms * 1e-3), "bytes_launch": bytes_launch,
            "achieved": bytes_launch / (ms * 1e-3) / 1e9, "info": info, "ncand": ncand,
            "check": check}


def run_batch(name, prec, seg_len, nseries, steps, warmup, wave_bytes, flags=0, keep_cols=0):
    """Time fdas_convolve_batch over a batched workload, in waves that fit;
    afterwards the wave holding the longest series runs once more and that
    series' first `keep_cols` plane columns come back as "check"."""
    import numpy as np
    import torch

    from paper_1711_10855_amd import fdas, synth
    w = synth.WORKLOADS[name]
    t0 = time.perf_counter()
    specs, spectra = synth.batch_inputs(name, nseries)
    gen_s = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    spec_dev = [torch.from_numpy(a).to(dev) for a in spectra]
    plan = fdas.Plan(w.zmax, w.dz, w.m, seg_len, prec, flags, device=0)
    info = plan.info
    per = 2 if flags & fdas.FLAG_INTERBIN else 1
    rows = [per * (int(round(2 * sp.zmax / w.dz)) + 1) for sp in specs]
    # plane rows padded to 256-byte multiples (ld >= nbins), so that every row
    # starts on a cache-line boundary
    lds = [(sp.nbins + 63) // 64 * 64 for sp in specs]
    sizes = [r * ld * 4 for r, ld in zip(rows, lds)]
    # waves: consecutive series whose planes fit the budget
    waves, cur, acc = [], [], 0
    for i, b in enumerate(sizes):
        if cur and acc + b > wave_bytes:
            waves.append(cur)
            cur, acc = [], 0
        cur.append(i)
        acc += b
    if cur:
        waves.append(cur)
    buf = torch.empty(max(sum(sizes[i] for i in wv) for wv in waves) // 4,
                      dtype=torch.float32, device=dev)
    calls = []
    for wv in waves:
        outs, off = [], 0
        for i in wv:
            plane = buf[off:off + rows[i] * lds[i]].view(rows[i], lds[i])
            outs.append(plane[:, :specs[i].nbins])
            off += rows[i] * lds[i]
        calls.append(([spec_dev[i] for i in wv], [specs[i].zmax for i in wv], outs))

    def step():
        for sp, zm, outs in calls:
            plan.convolve_batch(sp, zm, outs)

    stream = torch.cuda.current_stream(dev)
    ms, wall = _time(step, steps, warmup, stream)
    i0 = int(np.argmax([sp.nbins for sp in specs]))
    check = None
    if keep_cols:
        for k, wv in enumerate(waves):
            if i0 in wv:
                sp, zm, outs = calls[k]
                plan.convolve_batch(sp, zm, outs)
                check = outs[wv.index(i0)][:, :keep_cols].cpu().numpy()
    plan.close()
    points = int(sum(r * sp.nbins for r, sp in zip(rows, specs)))
    nbins_total = int(sum(sp.nbins for sp in specs))
    bytes_launch = 4.0 * points + 8.0 * nbins_total
    a0 = spectra[i0]
    return {"points": points, "nseries": len(specs), "waves": len(waves), "ms": ms,
            "wall": wall, "value": points / (ms * 1e-3), "bytes_launch": bytes_launch,
            "achieved": bytes_launch / (ms * 1e-3) / 1e9, "info": info, "gen_s": gen_s,
            "sample_spectrum": a0, "zmax": w.zmax, "dz": w.dz, "m": w.m, "check": check,
            "check_first_row": int(round((w.zmax - specs[i0].zmax) / w.dz))}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.variant:
        os.environ["FDAS_VARIANT"] = args.variant
    if args.zpb:
        os.environ["FDAS_ZPB"] = str(args.zpb)

    import torch

    from paper_1711_10855_amd import fdas, synth

    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n, "launches": 3}))
        return

    fdas.load()
    torch.cuda.set_device(0)
    w = synth.WORKLOADS[args.workload]
    prec = args.precision or w.precision
    if args.split and prec == "fp32":
        print(json.dumps({"error": "--split applies to the mixed precisions only"}))
        sys.exit(2)
    flags = (fdas.FLAG_SPLIT if args.split else 0) | (fdas.FLAG_INTERBIN if args.interbin else 0)
    compare = None
    keep = 0 if args.no_cpu_baseline else args.cpu_sample_bins
    bar = 1e-4 if prec == "fp32" else 1e-3
    if w.nseries == 1:
        seg_len = args.seg_len or (4096 if prec != "fp32" else w.seg_len)
        src = "fp32-paper" if args.workload == "mixed-paper" else args.workload
        a, _ = synth.single_series(src)
        a_dev = torch.from_numpy(a).to("cuda:0")
        r = run_single(a_dev, w.zmax, w.dz, w.m, seg_len, prec, args.steps, args.warmup, flags,
                       args.candidates, keep_cols=min(keep, a.size))
        step = 2 if args.interbin else 1  # integer-bin rows only
        checks = [] if r["check"] is None else [(prec, r["check"], 0, step, bar)]
        if not args.no_compare and prec == "fp32" and not args.variant and w.m < 4096:
            c = run_single(a_dev, w.zmax, w.dz, w.m, 4096, "fp16", args.steps, args.warmup,
                           flags & fdas.FLAG_INTERBIN, args.candidates,
                           keep_cols=min(keep, a.size))
            compare = {"fp16_mfma": {
                "value": c["value"], "ms_per_step": c["ms"], "seg_len": 4096,
                "kernel": c["info"].kernel, "frac": c["achieved"] / HBM_PEAK_GBS,
                "speedup_vs_fp32": c["value"] / r["value"],
                "error_bar": "max|P-P_ref| <= 1e-3 max P_ref"}}
            if c["check"] is not None:
                checks.append(("fp16_mfma", c["check"], 0, step, 1e-3))
        cpu_in = (a, w.zmax, w.dz, w.m, r["nz"] // step)
        cfg = {"workload": args.workload, "nbins": r["nbins"], "nz": r["nz"]}
    else:
        seg_len = args.seg_len or (4096 if prec != "fp32" else w.seg_len)
        r = run_batch(args.workload, prec, seg_len, args.nseries, args.steps, args.warmup,
                      int(args.wave_gb * 1e9), flags, keep_cols=keep)
        step = 2 if args.interbin else 1
        checks = [] if r["check"] is None else [
            (f"{prec} (longest series)", r["check"], r["check_first_row"], step, bar)]
        cpu_in = (r["sample_spectrum"], r["zmax"], r["dz"], r["m"], r["info"].nz // step)
        cfg = {"workload": args.workload, "nseries": r["nseries"], "waves": r["waves"],
               "input_gen_s": round(r["gen_s"], 1)}
    info = r["info"]
    cfg.update({"m": info.m, "seg_len": info.seg_len, "zmax": w.zmax, "dz": w.dz,
                "precision": prec, "kernel": info.kernel,
                "templates_per_block": info.templates_per_block,
                "plan_ms": round(info.plan_ms, 3), "wall_s_timed": round(r["wall"], 4)})
    traffic = traffic_from_profiles(info.kernel, args.workload)
    cfg["arithmetic"] = ("plain FP32" if prec == "fp32"
                         else f"{prec} storage, MFMA DFT stages, FP32 accumulation"
                         + (", hi+lo split products" if args.split else ""))
    if args.interbin:
        cfg["rows"] = "2 nz: integer and half-bin (r + 1/2) responses"
    if args.candidates is not None:
        cfg["epilogue"] = (f"threshold: points with power >= {args.candidates} listed, "
                           f"no plane written ({r.get('ncand')} found)")
    line = {
        "metric": "z\u2013r plane points/s, batched mixed-precision vs plain FP32; "
                  "% of HBM roofline",
        "value": r["value"],
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == "fp32" else f"{prec}{'x3' if args.split else ''}+f32acc",
        "data": "synthetic",
        "config": cfg,
        "roofline": {"bound": "hbm", "achieved": r["achieved"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": r["achieved"] / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_point": r["bytes_launch"] / r["points"]},
        "cpu_baseline": None,
    }
    if compare:
        line["compare"] = compare
    if not args.no_cpu_baseline:
        a0, zmax, dz, m, nz = cpu_in
        base, errors = cpu_baseline(a0, zmax, dz, m, nz, min(args.cpu_sample_bins, a0.size),
                                    checks)
        line["cpu_baseline"] = base
        if errors:
            line["error_vs_oracle"] = errors
    print(json.dumps(line))


if __name__ == "__main__":
    main()
