"""Benchmark of the FDAS correlation step on one MI355X.

A step is one call of the hot path (segment load, forward FFT, per-template
product + inverse FFT, overlap discard, |.|^2 store) over the whole input of
the workload: by default the paper-scale plain-FP32 workload (2^21 bins,
z in [-100, 100] step 2 -> 101 templates of width 256, segment FFT 2048),
producing the 101 x 2^21 FP32 power plane (847 MB). Inputs are resident in
device memory before the timed region; the plan (templates, bank) is built
once outside it and its time is reported separately.

Prints ONE JSON line. `value` is z-r plane points per second; `roofline`
prices the dominant kernel's algorithmic bytes per launch
(4 B per plane point written + 8 B per input bin read) against the 8 TB/s
HBM peak, with the kernel duration measured by HIP events on the stream the
kernel runs on; `cpu_baseline` times the FP64 oracle on a bounded sample.
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
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="fp32-paper")
    ap.add_argument("--variant", default=None, help="force a compiled kernel variant")
    ap.add_argument("--zpb", type=int, default=None, help="templates per work unit")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-bins", type=int, default=1 << 20)
    ap.add_argument("--seg-len", type=int, default=None)
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


def cpu_baseline(a, w, sample_bins: int):
    """The FP64 oracle (unchanged) on the first `sample_bins` bins, all rows."""
    import numpy as np

    import oracle
    sample = np.ascontiguousarray(a[:sample_bins])
    t0 = time.perf_counter()
    p = oracle.plane_direct(sample, w.zmax, w.dz, w.m)
    dt = time.perf_counter() - t0
    pts = p.shape[0] * p.shape[1]
    return {"value": pts / dt, "unit": "points/s", "cores": 1, "kind": "oracle",
            "sample": f"{w.nz} rows x first {sample_bins} bins of the same spectrum "
                      f"({pts} points, {dt:.1f} s, single process NumPy FP64 direct sum)"}


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

    import numpy as np
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

    w = synth.WORKLOADS[args.workload]
    if w.nseries != 1:
        raise SystemExit(f"workload {args.workload} is batched; single-series workloads only here")
    prec = w.precision
    seg_len = args.seg_len or (4096 if prec != "fp32" else w.seg_len)
    fdas.load()
    a, _ = synth.single_series("fp32-paper" if args.workload == "mixed-paper" else args.workload)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    spec = torch.from_numpy(a).to(dev)
    plan = fdas.Plan(w.zmax, w.dz, w.m, seg_len, prec, device=0)
    info = plan.info
    nz, nbins = info.nz, spec.numel()
    out = torch.empty((nz, nbins), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)

    for _ in range(args.warmup):
        plan.convolve(spec, out=out)
    torch.cuda.synchronize(dev)

    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(args.steps):
        plan.convolve(spec, out=out)
    stop.record(stream)
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    ms_total = start.elapsed_time(stop)
    ms_step = ms_total / args.steps

    points = nz * nbins
    value = points / (ms_step * 1e-3)
    bytes_launch = 4.0 * points + 8.0 * nbins
    achieved = bytes_launch / (ms_step * 1e-3) / 1e9
    traffic = traffic_from_profiles(info.kernel, args.workload)

    line = {
        "metric": f"z-r plane points/s ({'plain FP32' if prec == 'fp32' else prec + ' MFMA'}, "
                  f"paper-scale workload); % of HBM roofline",
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == "fp32" else f"{prec}+f32acc",
        "data": "synthetic",
        "config": {"workload": args.workload, "nbins": nbins, "nz": nz, "m": info.m,
                   "seg_len": info.seg_len, "zmax": w.zmax, "dz": w.dz,
                   "kernel": info.kernel, "templates_per_block": info.templates_per_block,
                   "plan_ms": round(info.plan_ms, 3), "wall_s_timed": round(wall, 4)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_point": bytes_launch / points},
        "cpu_baseline": None,
    }
    plan.close()
    del out
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(a, w, min(args.cpu_sample_bins, nbins))
    print(json.dumps(line))


if __name__ == "__main__":
    main()
