"""Turn rocprofv3 outputs of the benchmark into the committed summaries.

Inputs (directories written by rocprofv3 -d ... --output-format csv):
  --trace DIR...     --kernel-trace --stats runs of bench.py
  --fetch DIR...     --pmc FETCH_SIZE runs of bench.py
  --write DIR...     --pmc WRITE_SIZE runs of bench.py
                     (one directory per profiled command, in the order of
                     --command; float64 and float32 runs give separate rows)
  --copy-fetch DIR   --pmc FETCH_SIZE run of pmc_copy.py
  --copy-write DIR   --pmc WRITE_SIZE run of pmc_copy.py
Outputs: profiles/pmc_stage_preheat256.json (read by bench.py for
roofline.traffic) and a text summary (markdown) with the commands.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
VARIANTS = {
    ("false", "false", "false", "false", "true"): "kick",
    ("false", "false", "true", "false", "true"): "kick_red",
    ("true", "false", "false", "true", "true"): "drift_kick",
    ("true", "false", "true", "true", "true"): "drift_kick_red",
    ("false", "true", "false", "true", "true"): "kick_drift",
    ("false", "false", "true", "false", "false"): "energy",
}
COPY_BYTES = 1 << 30


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in ("stage_rows.hpp", "stage_scalar.hpp", "common.hpp"):
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def variant_key(name: str):
    m = re.search(r"scalar_(stage|rows)<(.*?)>", name)
    if not m:
        return None
    args = [a.strip() for a in m.group(2).split(",")]
    prec = "f32" if args[0] == "float" else "f64"
    v = VARIANTS.get(tuple(args[4:9]))   # <T, NF, XS or TX, TY, five flags[, prefetch depth]>
    return f"{v}_{prec}" if v else None


def csv_in(d, suffix):
    files = glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return files[0]


def counters(d, counter):
    rows = list(csv.DictReader(open(csv_in(d, "counter_collection.csv"))))
    agg = defaultdict(list)
    for r in rows:
        if r["Counter_Name"] == counter:
            agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return agg


def copy_factor(d, counter):
    agg = counters(d, counter)
    vals = [v for k, vs in agg.items() if "copyBuffer" in k or "copy" in k.lower() for v in vs]
    vals = [v for v in vals if v > 0.25 * COPY_BYTES / 1024]
    kib = sum(vals) / len(vals)
    expect_kib = COPY_BYTES / 1024        # 1 GiB read and 1 GiB written per copy
    return expect_kib / kib, kib


def all_kernels(trace_dir, command, out_dir):
    """Per-kernel stats table of a --kernel-trace --stats run of the whole
    benchmark (every workload's kernels)."""
    stats = list(csv.DictReader(open(csv_in(trace_dir, "kernel_stats.csv"))))
    lines = ["# all kernels of the default benchmark run", "",
             f"Command: `rocprofv3 --kernel-trace --stats -d <dir> -o all --output-format csv -- {command}`", "",
             "| kernel | calls | average us | min us | max us | total ms | % |", "|---|---|---|---|---|---|---|"]
    for r in stats:
        lines.append(f"| {r['Name'][:100]} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f} |")
    with open(os.path.join(out_dir, "kernels_bench_default.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True, nargs="+")
    ap.add_argument("--fetch", required=True, nargs="+")
    ap.add_argument("--write", required=True, nargs="+")
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--command", required=True, nargs="+", help="the bench commands that were profiled")
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    ap.add_argument("--all-trace", help="--kernel-trace --stats run of the whole default benchmark")
    ap.add_argument("--all-command", default="python3 bench.py --no-cpu-baseline")
    ap.add_argument("--note", default="", help="provenance line for the summary (which runs, which machines)")
    a = ap.parse_args()
    if a.all_trace:
        all_kernels(a.all_trace, a.all_command, a.out)

    ff, fk = copy_factor(a.copy_fetch, "FETCH_SIZE")
    wf, wk = copy_factor(a.copy_write, "WRITE_SIZE")
    per = defaultdict(dict)
    for counter, dirs, fac in (("FETCH_SIZE", a.fetch, ff), ("WRITE_SIZE", a.write, wf)):
        for d in dirs:
            for name, vals in counters(d, counter).items():
                k = variant_key(name)
                if k:
                    per[k][counter] = sum(vals) / len(vals)
                    per[k][counter + "_scaled_bytes"] = fac * per[k][counter] * 1024
                    per[k]["launches"] = len(vals)
                    per[k]["kernel_name"] = name
    stats = []
    dur = defaultdict(list)
    for d in a.trace:
        stats += list(csv.DictReader(open(csv_in(d, "kernel_stats.csv"))))
        for r in csv.DictReader(open(csv_in(d, "kernel_trace.csv"))):
            k = variant_key(r["Kernel_Name"])
            if k:
                dur[k].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    stats.sort(key=lambda r: -float(r["TotalDurationNs"]))
    kernels = {}
    for k, d in per.items():
        kernels[k] = {
            "launches": d.get("launches"),
            "fetch_kib": d.get("FETCH_SIZE"),
            "write_kib": d.get("WRITE_SIZE"),
            "hbm_bytes_per_launch": d.get("FETCH_SIZE_scaled_bytes", 0.0) + d.get("WRITE_SIZE_scaled_bytes", 0.0),
            "mean_us_trace": sum(dur[k]) / len(dur[k]) if dur.get(k) else None,
            "kernel_name": d.get("kernel_name"),
        }
    out = {"kernel_hash": kernel_hash(), "command": " ; ".join(a.command),
           "fetch_factor": ff, "write_factor": wf, "copy_fetch_kib": fk, "copy_write_kib": wk,
           "copy_bytes": COPY_BYTES, "kernels": kernels}
    os.makedirs(a.out, exist_ok=True)
    with open(os.path.join(a.out, "pmc_stage_preheat256.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    lines = ["# scalar stage kernel, preheat-256^3-VV4-self workload", "",
             "Profiled commands: " + ", ".join(f"`{c}`" for c in a.command), "",
             "rocprofv3 runs (each its own pass, for each command):", ""]
    for c in a.command:
        lines += [f"- `rocprofv3 --kernel-trace --stats -d <dir> -o trace --output-format csv -- {c}`",
                  f"- `rocprofv3 --pmc FETCH_SIZE -d <dir> -o fetch --output-format csv -- {c}`",
                  f"- `rocprofv3 --pmc WRITE_SIZE -d <dir> -o write --output-format csv -- {c}`"]
    lines += [
             "- the same two counter runs on `python3 paper_2102_01031_amd/pmc_copy.py` (1 GiB device copy)",
             "", f"Kernel source hash: `{out['kernel_hash']}`", ""] + ([a.note, ""] if a.note else []) + [
             
             f"Copy calibration: FETCH_SIZE reads {fk:.0f} KiB per 1 GiB copy -> factor {ff:.4f}; "
             f"WRITE_SIZE {wk:.0f} KiB -> factor {wf:.4f}.", "",
             "## kernel stats (rocprofv3 --stats)", "",
             "| kernel | calls | average ns | min ns | max ns | total ns | % |", "|---|---|---|---|---|---|---|"]
    for r in stats[:12]:
        lines.append(f"| {r['Name'][:90]} | {r['Calls']} | {float(r['AverageNs']):.0f} | {r['MinNs']} | "
                     f"{r['MaxNs']} | {r['TotalDurationNs']} | {float(r['Percentage']):.2f} |")
    lines += ["", "## per variant (trace mean, counters per dispatch)", "",
              "| variant | launches | mean us (trace) | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes / launch (scaled) |",
              "|---|---|---|---|---|---|"]
    for k, v in sorted(kernels.items()):
        mu = f"{v['mean_us_trace']:.1f}" if v["mean_us_trace"] else "-"
        lines.append(f"| {k} | {v['launches']} | {mu} | {v['fetch_kib'] or 0:.0f} | {v['write_kib'] or 0:.0f} | "
                     f"{v['hbm_bytes_per_launch'] / 1e6:.1f} MB |")
    with open(os.path.join(a.out, "stage_preheat256.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
