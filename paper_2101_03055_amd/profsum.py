"""Summaries of rocprofv3 output for the committed profile notes.

    python -m paper_2101_03055_amd.profsum --name NAME --command "CMD" \\
        --stats DIR/run_kernel_stats.csv [--kernel SUBSTR --bytes-per-launch B] \\
        [--fetch F.csv --write W.csv --copy-fetch CF.csv --copy-write CW.csv --copy-bytes N]

writes profiles/NAME.md (kernel table, counters, calibration, the command)
and, with counters, profiles/NAME.traffic.json: bytes per launch of the
matching kernels measured by FETCH_SIZE / WRITE_SIZE (KiB per dispatch),
each scaled by what the same counter reads for a plain device copy of known
size, tagged with a hash of the kernel sources so that a benchmark can tell
whether the numbers still describe the code it runs.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
KERNEL_SOURCES = ["csrc/lb_device.h", "csrc/lb_kernels.hip", "csrc/lb_internal.h", "csrc/lb_batch.hip", "csrc/lb_cde.hip"]


def source_hash(files=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short(name: str) -> str:
    return name.replace("void ", "").split("(")[0]


def kernel_stats(path):
    rows = []
    for r in csv.DictReader(open(path)):
        rows.append({"kernel": short(r["Name"]), "calls": int(r["Calls"]), "avg_us": float(r["AverageNs"]) / 1e3,
                     "min_us": float(r["MinNs"]) / 1e3, "max_us": float(r["MaxNs"]) / 1e3,
                     "pct": float(r["Percentage"])})
    return rows


def counter_means(path):
    acc = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        acc[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--name", required=True)
    ap.add_argument("--command", required=True)
    ap.add_argument("--stats", required=True)
    ap.add_argument("--kernel", default="k_step")
    ap.add_argument("--bytes-per-launch", type=float, default=None)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--copy-bytes", type=float, default=float(1 << 30))
    ap.add_argument("--copy-kernel", default="__amd_rocclr_copyBuffer")
    ap.add_argument("--note", default="")
    ap.add_argument("--sources", default=None,
                    help="comma-separated kernel sources (under the package) hashed into the traffic record")
    args = ap.parse_args()

    stats = kernel_stats(args.stats)
    lines = [f"# {args.name}", "", f"Command: `{args.command}`", ""]
    if args.note:
        lines += [args.note, ""]
    lines += ["| kernel | calls | avg us | min us | max us | % time |", "|---|---|---|---|---|---|"]
    for r in stats[:12]:
        lines.append(f"| `{r['kernel']}` | {r['calls']} | {r['avg_us']:.2f} | {r['min_us']:.2f} | {r['max_us']:.2f} "
                     f"| {r['pct']:.1f} |")
    sel = [r for r in stats if args.kernel in r["kernel"]]
    if sel:
        calls = sum(r["calls"] for r in sel)
        avg = sum(r["avg_us"] * r["calls"] for r in sel) / calls
        lines += ["", f"Mean duration over the `{args.kernel}` launches: {avg:.3f} us ({calls} launches)."]
        if args.bytes_per_launch:
            lines.append(f"Algorithmic bytes per launch {args.bytes_per_launch:.0f} -> "
                         f"{args.bytes_per_launch / avg / 1e3:.1f} GB/s.")
    out_json = None
    if args.fetch and args.write and args.copy_fetch and args.copy_write:
        f, w = counter_means(args.fetch), counter_means(args.write)
        cf, cw = counter_means(args.copy_fetch)[args.copy_kernel], counter_means(args.copy_write)[args.copy_kernel]
        kib = args.copy_bytes / 1024.0
        ff, fw = kib / cf, kib / cw
        ks = [k for k in f if args.kernel in k]
        lines += ["", "HBM-side counters (KiB per dispatch, mean), calibrated by a plain device copy of "
                  f"{args.copy_bytes / 2**30:.2f} GiB: FETCH_SIZE reads {cf:.0f} KiB (factor {ff:.3f}), "
                  f"WRITE_SIZE {cw:.0f} KiB (factor {fw:.3f}).", "",
                  "| kernel | FETCH_SIZE | WRITE_SIZE | calibrated bytes |", "|---|---|---|---|"]
        per = []
        for k in ks:
            b = (f[k] * ff + w[k] * fw) * 1024.0
            per.append(b)
            lines.append(f"| `{k}` | {f[k]:.1f} | {w[k]:.1f} | {b:.0f} |")
        if per:
            mean = sum(per) / len(per)
            lines.append("")
            lines.append(f"Mean calibrated traffic per `{args.kernel}` launch: {mean:.0f} B" +
                         (f" ({mean / args.bytes_per_launch:.3f} x algorithmic)." if args.bytes_per_launch else "."))
            out_json = {"kernel": args.kernel, "traffic_bytes_per_launch": mean, "fetch_factor": ff,
                        "write_factor": fw,
                        "source_hash": source_hash(args.sources.split(",")) if args.sources else source_hash(),
                        "command": args.command}
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", args.name + ".md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    if out_json:
        with open(os.path.join(ROOT, "profiles", args.name + ".traffic.json"), "w") as fh:
            json.dump(out_json, fh, indent=1)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
