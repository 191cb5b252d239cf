"""Summarise rocprofv3 CSV output of the benchmark into profiles/.

Reads the kernel-trace statistics and the counter-collection CSVs written by
`rocprofv3 --output-format csv` runs of bench.py, and writes a short
markdown summary plus one row of profiles/traffic.json (HBM bytes per launch
of the hot kernel, FETCH_SIZE and WRITE_SIZE scaled by what the same counters
read for a plain device copy of known size).

Usage:
  python -m paper_1711_10855_amd.profile_summary --dir <rocprofv3 output dir> \
      --workload fp32-paper --kernel-match ols_ --name <summary-name> \
      --command "<the rocprofv3 commands that produced the CSVs>"
"""

from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
# Sources each hot kernel is built from: a traffic row stays current only
# while the sources of its own kernel are unchanged.
FP32_SOURCES = ["csrc/ols_fp32.hip", "csrc/fft_radix.hpp", "csrc/fft_block.hpp",
                "csrc/layout.hpp", "csrc/ols_variants.hpp"]
MIXED_SOURCES = ["csrc/ols_mixed.hip", "csrc/fft_radix.hpp", "csrc/ols_variants.hpp", "csrc/cand4.hpp"]
MIXED2048_SOURCES = ["csrc/ols_mixed2048.hip", "csrc/fft_radix.hpp", "csrc/ols_variants.hpp",
                     "csrc/cand4.hpp"]


def kernel_sources(kernel: str) -> list[str]:
    """Source files of a hot-kernel variant, by its name (fp32_* variants are
    the FP32 kernels, *_L2048_mfma_* the 2048-point matrix-core kernel, the
    others the 4096-point matrix-core kernels)."""
    if kernel.startswith("fp32_"):
        return FP32_SOURCES
    return MIXED2048_SOURCES if "_L2048_mfma" in kernel else MIXED_SOURCES


def source_hash(kernel: str) -> str:
    """Hash of the sources of the named kernel variant."""
    h = hashlib.sha256()
    for rel in kernel_sources(kernel):
        p = os.path.join(HERE, rel)
        if os.path.exists(p):
            h.update(rel.encode())
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def _counters(path, match):
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(path)):
        agg[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    out = {}
    for k, d in agg.items():
        if match in k:
            out[k] = {c: sum(v) / len(v) for c, v in d.items()}
    return out


def _one(pattern):
    files = glob.glob(pattern)
    return files[0] if files else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dir", required=True, help="directory holding the rocprofv3 CSV runs")
    ap.add_argument("--workload", required=True)
    ap.add_argument("--kernel-match", default="ols_")
    ap.add_argument("--name", required=True)
    ap.add_argument("--command", required=True)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--variant", required=True, help="kernel variant name the bench ran")
    ap.add_argument("--timed-last", type=int, default=0,
                    help="also report the mean over the last N dispatches of the hot "
                         "kernel (the bench's timed steps, after its warm-up)")
    ap.add_argument("--bytes-per-launch", type=float, default=None,
                    help="algorithmic bytes per launch, for the ratio")
    a = ap.parse_args()
    d = a.dir
    lines = [f"# {a.name}", "", "Command(s):", "", "```", a.command, "```", ""]

    stats = _one(os.path.join(d, "prof_kt", "*kernel_stats.csv"))
    kname = None
    avg_ns = None
    if stats:
        lines += ["## Kernel trace (--kernel-trace --stats)", "",
                  "| kernel | calls | avg us | min us | max us | % time |", "|---|---|---|---|---|---|"]
        for r in csv.DictReader(open(stats)):
            nm = r["Name"]
            short = nm.split("(")[0][:110]
            lines.append(f"| `{short}` | {r['Calls']} | {float(r['AverageNs'])/1e3:.1f} | "
                         f"{float(r['MinNs'])/1e3:.1f} | {float(r['MaxNs'])/1e3:.1f} | "
                         f"{float(r['Percentage']):.1f} |")
            if a.kernel_match in nm and kname is None:
                kname = nm
                avg_ns = float(r["AverageNs"])
        lines.append("")

    merged = {}
    for sub in sorted(glob.glob(os.path.join(d, "prof_sq*"))):
        sq = _one(os.path.join(sub, "*counter_collection.csv"))
        if sq:
            for k, c in _counters(sq, a.kernel_match).items():
                merged.setdefault(k, {}).update(c)
    if merged:
        lines += ["## SQ counters (per dispatch, mean)", ""]
        for k, c in merged.items():
            lines.append(f"`{k.split('(')[0][:110]}`")
            lines.append("")
            for name, v in sorted(c.items()):
                lines.append(f"- {name}: {v:.6g}")
            if "SQ_INSTS_VALU" in c and "SQ_WAVES" in c:
                lines.append(f"- VALU instructions per wave: {c['SQ_INSTS_VALU']/c['SQ_WAVES']:.0f}")
            if "SQ_LDS_BANK_CONFLICT" in c and "SQ_LDS_IDX_ACTIVE" in c and c["SQ_LDS_IDX_ACTIVE"] > 0:
                lines.append(f"- LDS bank-conflict cycles / LDS active cycles: "
                             f"{c['SQ_LDS_BANK_CONFLICT']/c['SQ_LDS_IDX_ACTIVE']:.3f}")
            if "SQ_WAVE_CYCLES" in c and c["SQ_WAVE_CYCLES"] > 0:
                for w in ("SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_ANY"):
                    if w in c:
                        lines.append(f"- {w} / SQ_WAVE_CYCLES: {c[w]/c['SQ_WAVE_CYCLES']:.3f}")
            lines.append("")

    def counter(sub, cname, match):
        p = _one(os.path.join(d, sub, "*counter_collection.csv"))
        if not p:
            return None
        vals = [v.get(cname) for v in _counters(p, match).values() if cname in v]
        return max(vals) if vals else None

    fetch = counter("prof_fetch", "FETCH_SIZE", a.kernel_match)
    write = counter("prof_write", "WRITE_SIZE", a.kernel_match)
    cfetch = counter("prof_cfetch", "FETCH_SIZE", "copyBuffer")
    cwrite = counter("prof_cwrite", "WRITE_SIZE", "copyBuffer")
    row = None
    if fetch is not None and write is not None and cfetch and cwrite:
        copy_kib = a.copy_mib * 1024.0
        ffac = copy_kib / cfetch
        wfac = copy_kib / cwrite
        tb = (fetch * ffac + write * wfac) * 1024.0
        lines += ["## HBM traffic (--pmc FETCH_SIZE, then --pmc WRITE_SIZE; KiB per dispatch)", "",
                  f"- hot kernel FETCH_SIZE {fetch:.1f} KiB, WRITE_SIZE {write:.1f} KiB",
                  f"- plain copy of {a.copy_mib} MiB reads FETCH_SIZE {cfetch:.1f} KiB and "
                  f"WRITE_SIZE {cwrite:.1f} KiB -> scale factors {ffac:.3f} (fetch), {wfac:.3f} (write)",
                  f"- scaled HBM traffic per launch: {tb/1e6:.2f} MB "
                  f"(read {fetch*ffac*1024/1e6:.2f} MB, write {write*wfac*1024/1e6:.2f} MB)"]
        if a.bytes_per_launch:
            lines.append(f"- algorithmic bytes per launch {a.bytes_per_launch/1e6:.2f} MB -> "
                         f"traffic / algorithmic = {tb/a.bytes_per_launch:.3f}")
        lines.append("")
        row = {"kernel": a.variant, "workload": a.workload, "bytes_per_launch": tb,
               "source_hash": source_hash(a.variant), "profile": a.name}
    if avg_ns:
        lines.append(f"Average duration of the hot kernel under the profiler: {avg_ns/1e3:.1f} us")
    tr = _one(os.path.join(d, "prof_kt", "*kernel_trace.csv"))
    if a.timed_last and tr:
        with open(tr) as f:
            durs = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
                    for r in csv.DictReader(f) if a.kernel_match in r["Kernel_Name"]]
        durs.sort()
        last = [x for _, x in durs[-a.timed_last:]]
        if last:
            lines.append(f"Mean over the last {len(last)} dispatches (the timed steps after the "
                         f"warm-up): {sum(last) / len(last) / 1e3:.1f} us")
    out_md = os.path.join(ROOT, "profiles", a.name + ".md")
    os.makedirs(os.path.dirname(out_md), exist_ok=True)
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    if row is not None:
        tj = os.path.join(ROOT, "profiles", "traffic.json")
        rows = []
        if os.path.exists(tj):
            rows = [r for r in json.load(open(tj))
                    if r.get("profile") != a.name
                    and (r.get("kernel"), r.get("workload")) != (a.variant, a.workload)]
        row["kernel_symbol"] = kname.split("(")[0] if kname else None
        rows.append(row)
        with open(tj, "w") as f:
            json.dump(rows, f, indent=1)
    print(out_md)


if __name__ == "__main__":
    main()
