"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_1803_09876_amd.rocprof_summary kernels <csv dir> <out.md> <title> <command> [rows]
        kernel statistics of a `rocprofv3 --kernel-trace --stats --output-format csv` run
        (the run_kernel_stats.csv table) as a short markdown table (the first 12 kernels by
        total time, or [rows]).

    python -m paper_1803_09876_amd.rocprof_summary traffic <fetch csv dir> <write csv dir> <kernel substring>
                                                         <key> <out.json> <out.md> <command>
        HBM bytes per dispatch of the kernel from a FETCH_SIZE pass and a WRITE_SIZE pass
        (`rocprofv3 --pmc ... --output-format csv`), each scaled by what the same counter read
        for the largest device-to-device copy in the run (a plain copy of known size: the
        benchmark's --copy-probe, 512 MiB read and 512 MiB written).

    python -m paper_1803_09876_amd.rocprof_summary counters <csv dir> <kernel substring> <out.md> <title> <command>
        every counter of a `rocprofv3 --pmc ... --output-format csv` run averaged over the
        kernel's dispatches (the L2 hit rate, and the ratio SQ_WAVE_CYCLES / SQ_BUSY_CYCLES, are
        derived when those counters are among them).

Reads only the CSV files rocprofv3 writes; nothing here runs on the GPU.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys

COPY_BYTES = 512 << 20
HERE = os.path.dirname(os.path.abspath(__file__))


def _one(pattern: str) -> str:
    files = sorted(glob.glob(pattern, recursive=True))
    if not files:
        raise SystemExit(f"no file matches {pattern}")
    return files[0]


def kernels(csv_dir: str, out: str, title: str, command: str, top: int = 12) -> None:
    path = _one(os.path.join(csv_dir, "**", "*kernel_stats.csv"))
    with open(path) as f:
        rows = list(csv.DictReader(f))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    with open(out, "w") as f:
        f.write(f"# {title}\n\nCommand (on the MI355X, from /tmp with TMPDIR=/tmp):\n\n```\n{command}\n```\n\n")
        f.write("rocprofv3 kernel statistics (durations in microseconds):\n\n"
                "| kernel | calls | total us | average us | min us | max us | % |\n|---|---|---|---|---|---|---|\n")
        for r in rows[:top]:
            name = r["Name"].replace("(anonymous namespace)::", "")
            name = name.split("(")[0] if "jsw::" in name else (name[:70] + "..." if len(name) > 70 else name)
            f.write(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e3:.1f} | "
                    f"{float(r['AverageNs']) / 1e3:.3f} | {float(r['MinNs']) / 1e3:.3f} | "
                    f"{float(r['MaxNs']) / 1e3:.3f} | {float(r['Percentage']):.2f} |\n")
    print(open(out).read())


def _per_dispatch(csv_dir: str, counter: str):
    path = _one(os.path.join(csv_dir, "**", "*counter_collection.csv"))
    out = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                out.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return out


def _scaled(csv_dir: str, counter: str, kernel: str):
    rows = _per_dispatch(csv_dir, counter)
    copies = [v for n, v in rows if "copyBuffer" in n]
    if not copies:
        raise SystemExit(f"{counter}: no copy dispatch to calibrate against")
    factor = (COPY_BYTES / 1024.0) / max(copies)
    vals = [v for n, v in rows if kernel in n]
    if not vals:
        raise SystemExit(f"{counter}: no dispatch of {kernel}")
    return sum(vals) / len(vals), factor, len(vals)


def traffic(fetch_dir, write_dir, kernel, key, out_json, out_md, command) -> None:
    f_kib, f_fac, nf = _scaled(fetch_dir, "FETCH_SIZE", kernel)
    w_kib, w_fac, nw = _scaled(write_dir, "WRITE_SIZE", kernel)
    read_b = f_kib * f_fac * 1024.0
    write_b = w_kib * w_fac * 1024.0
    with open(os.path.join(HERE, "csrc", "sweep.hip"), "rb") as fh:
        src_hash = hashlib.sha256(fh.read()).hexdigest()[:16]
    data = {}
    if os.path.exists(out_json):
        with open(out_json) as fh:
            data = json.load(fh)
    data[key] = {"kernel": kernel, "source_hash": src_hash, "dispatches": [nf, nw],
                 "fetch_kib_per_dispatch": f_kib, "write_kib_per_dispatch": w_kib,
                 "fetch_scale": f_fac, "write_scale": w_fac,
                 "hbm_read_bytes_per_launch": read_b, "hbm_write_bytes_per_launch": write_b,
                 "hbm_bytes_per_launch": read_b + write_b}
    with open(out_json, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    with open(out_md, "w") as fh:
        fh.write(f"# HBM traffic of `{kernel}` ({key})\n\nCommands (on the MI355X, from /tmp with TMPDIR=/tmp):\n\n"
                 f"```\n{command}\n```\n\n"
                 f"| counter | KiB per dispatch (raw) | scale (copy of 512 MiB) | bytes per launch |\n|---|---|---|---|\n"
                 f"| FETCH_SIZE | {f_kib:.1f} | {f_fac:.4f} | {read_b:.4e} |\n"
                 f"| WRITE_SIZE | {w_kib:.1f} | {w_fac:.4f} | {write_b:.4e} |\n\n"
                 f"Total HBM bytes per launch: {read_b + write_b:.4e} (dispatches averaged: {nf} / {nw}; "
                 f"sweep source hash {src_hash}).\n")
    print(open(out_md).read())


def counters(csv_dir, kernel, out, title, command) -> None:
    path = _one(os.path.join(csv_dir, "**", "*counter_collection.csv"))
    vals = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            if kernel in r["Kernel_Name"]:
                vals.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    if not vals:
        raise SystemExit(f"no dispatch of {kernel}")
    avg = {k: sum(v) / len(v) for k, v in vals.items()}
    with open(out, "w") as f:
        f.write(f"# {title}\n\nCommand (on the MI355X, from /tmp with TMPDIR=/tmp):\n\n```\n{command}\n```\n\n")
        f.write(f"Counters of `{kernel}`, averaged over its dispatches:\n\n| counter | per dispatch | dispatches |\n"
                "|---|---|---|\n")
        for k in sorted(avg):
            f.write(f"| {k} | {avg[k]:.6g} | {len(vals[k])} |\n")
        if "TCC_HIT_sum" in avg and "TCC_MISS_sum" in avg:
            h, m = avg["TCC_HIT_sum"], avg["TCC_MISS_sum"]
            f.write(f"\nL2 hit rate: {h / max(1.0, h + m):.3f} ({h + m:.4g} L2 requests per dispatch).\n")
        if "SQ_WAVE_CYCLES" in avg and "SQ_BUSY_CYCLES" in avg and avg["SQ_BUSY_CYCLES"] > 0:
            f.write(f"\nSQ_WAVE_CYCLES / SQ_BUSY_CYCLES (wavefront-cycles per busy cycle of the counting "
                    f"sequencers, as summed by rocprofv3): {avg['SQ_WAVE_CYCLES'] / avg['SQ_BUSY_CYCLES']:.1f}.\n")
        if "SQ_WAVES" in avg:
            f.write(f"\nWavefronts launched per dispatch (SQ_WAVES): {avg['SQ_WAVES']:.0f}.\n")
    print(open(out).read())


def main(argv):
    if len(argv) >= 5 and argv[0] == "kernels":
        kernels(*argv[1:5], *([int(argv[5])] if len(argv) > 5 else []))
    elif len(argv) >= 8 and argv[0] == "traffic":
        traffic(*argv[1:8])
    elif len(argv) >= 6 and argv[0] == "counters":
        counters(*argv[1:6])
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
