"""Summaries of rocprofv3 output for the profiles/ directory.

    python -m paper_2305_18025_amd.profiling stats <kernel_stats.csv> <out.md> "<command>" ["<note>"]
    python -m paper_2305_18025_amd.profiling traffic <fetch_counter.csv> <write_counter.csv> \
        <kernel substring> <batch> <copy bytes> <out.json> <out.md> "<command>"

    python -m paper_2305_18025_amd.profiling sq <counter_collection.csv> <kernel substring> \
        <terms per launch> <out.md> "<command>"

`stats` turns a --kernel-trace --stats CSV into a short markdown table.
`sq` averages SQ/GRBM counters per dispatch of the named kernel and derives
VALU instructions per term (SQ_INSTS_VALU, wave instructions of 64 lanes,
times 64 over the launch's terms) and the VALU-active share of the waves'
cycles (SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES).
`traffic` reads two --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per
dispatch), takes the mean per dispatch of the named kernel, and scales each by
what the same counter reads for the calibration copy kernel (a copy of
`copy bytes` bytes reads and writes exactly that many bytes); the result is
HBM bytes per launch.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# the sources the fused exchange launch is compiled from
EXCHANGE_SOURCES = ("common.h", "exchange.h", "exchange_inst.hip", "kernels.hip", "internal.h")


def device_sources_sha1():
    """SHA-1 over the exchange launch's device sources: a counter summary is
    valid for the bench only while this is unchanged."""
    h = hashlib.sha1()
    for f in EXCHANGE_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2305_18025_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def kernel_stats(csv_path):
    rows = list(csv.DictReader(open(csv_path)))
    out = []
    for r in rows:
        out.append(dict(name=r["Name"], calls=int(r["Calls"]), total_ns=float(r["TotalDurationNs"]),
                        avg_ns=float(r["AverageNs"]), min_ns=float(r["MinNs"]), max_ns=float(r["MaxNs"]),
                        pct=float(r["Percentage"])))
    return out


def stats_markdown(csv_path, out_md, command, note=""):
    ks = kernel_stats(csv_path)
    lines = ["# rocprofv3 kernel statistics", "", "Command:", "", "```", command, "```", "",
             "| kernel | calls | avg (us) | min (us) | max (us) | share |", "|---|---|---|---|---|---|"]
    for k in ks:
        lines.append("| `%s` | %d | %.1f | %.1f | %.1f | %.1f%% |" % (
            k["name"], k["calls"], k["avg_ns"] / 1e3, k["min_ns"] / 1e3, k["max_ns"] / 1e3, k["pct"]))
    if note:
        lines += ["", note]
    open(out_md, "w").write("\n".join(lines) + "\n")
    return ks


def _per_dispatch(csv_path, counter, substr):
    vals = {}
    for r in csv.DictReader(open(csv_path)):
        if r["Counter_Name"] != counter or substr not in r["Kernel_Name"]:
            continue
        vals.setdefault(r["Dispatch_Id"], 0.0)
        vals[r["Dispatch_Id"]] += float(r["Counter_Value"])
    return list(vals.values())


def traffic(fetch_csv, write_csv, substr, batch, copy_bytes, out_json, out_md, command):
    fk = _per_dispatch(fetch_csv, "FETCH_SIZE", substr)
    wk = _per_dispatch(write_csv, "WRITE_SIZE", substr)
    fc = _per_dispatch(fetch_csv, "FETCH_SIZE", "copy")
    wc = _per_dispatch(write_csv, "WRITE_SIZE", "copy")
    # the calibration copy is the largest copy dispatch
    fcal = max(fc) * 1024.0 / copy_bytes
    wcal = max(wc) * 1024.0 / copy_bytes
    fetch = sum(fk) / len(fk) * 1024.0 / fcal
    write = sum(wk) / len(wk) * 1024.0 / wcal
    rec = {"kernel": substr, "batch": int(batch), "dispatches": [len(fk), len(wk)],
           "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
           "hbm_bytes_per_launch": fetch + write,
           "calibration": {"copy_bytes": int(copy_bytes), "fetch_counter_per_byte": fcal,
                           "write_counter_per_byte": wcal},
           "device_sources_sha1": device_sources_sha1(),
           "command": command}
    json.dump(rec, open(out_json, "w"), indent=1)
    lines = ["# HBM traffic of the fused exchange launch", "", "Commands (one counter per run):", "", "```",
             command, "```", "",
             "| quantity | value |", "|---|---|",
             "| kernel | `%s` |" % substr,
             "| batch (systems per launch) | %d |" % batch,
             "| FETCH_SIZE per launch, scaled | %.3f MB |" % (fetch / 1e6),
             "| WRITE_SIZE per launch, scaled | %.3f MB |" % (write / 1e6),
             "| calibration: FETCH_SIZE KiB per copied KiB | %.4f |" % fcal,
             "| calibration: WRITE_SIZE KiB per copied KiB | %.4f |" % wcal,
             ""]
    open(out_md, "w").write("\n".join(lines) + "\n")
    return rec


def sq_summary(csv_path, substr, terms, out_md, command):
    """Mean per dispatch of every counter in a --pmc CSV for the named
    kernel, and the derived issue figures."""
    per = {}
    for r in csv.DictReader(open(csv_path)):
        if substr not in r["Kernel_Name"]:
            continue
        per.setdefault(r["Counter_Name"], {}).setdefault(r["Dispatch_Id"], 0.0)
        per[r["Counter_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
    mean = {k: sum(v.values()) / len(v) for k, v in per.items()}
    n = {k: len(v) for k, v in per.items()}
    lines = ["# SQ counters of `%s`" % substr, "", "Command:", "", "```", command, "```", "",
             "| counter | mean per dispatch | dispatches |", "|---|---|---|"]
    for k in sorted(mean):
        lines.append("| %s | %.6g | %d |" % (k, mean[k], n[k]))
    lines.append("")
    if "SQ_INSTS_VALU" in mean and terms > 0:
        lines.append("VALU instructions per term: SQ_INSTS_VALU x 64 / %d terms = %.2f" %
                     (terms, mean["SQ_INSTS_VALU"] * 64.0 / terms))
    if "SQ_ACTIVE_INST_VALU" in mean and "SQ_WAVE_CYCLES" in mean:
        lines.append("")
        lines.append("VALU-active share of wave cycles: SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES = %.3f" %
                     (mean["SQ_ACTIVE_INST_VALU"] / mean["SQ_WAVE_CYCLES"]))
    if "SQ_INSTS_VALU" in mean and "GRBM_GUI_ACTIVE" in mean:
        # GRBM_GUI_ACTIVE sums the 8 XCDs' busy cycles; 1024 SIMDs in all
        simd_cycles = 1024.0 * mean["GRBM_GUI_ACTIVE"] / 8.0
        lines.append("")
        lines.append("VALU wave instructions per SIMD cycle: SQ_INSTS_VALU / (1024 SIMDs x GRBM_GUI_ACTIVE / 8 "
                     "XCDs) = %.3f (a SIMD completes one FP64 wave instruction per 4 cycles: 0.25)" %
                     (mean["SQ_INSTS_VALU"] / simd_cycles))
    lines.append("")
    lines.append("Device sources SHA-1: %s" % device_sources_sha1())
    open(out_md, "w").write("\n".join(lines) + "\n")
    return mean


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats_markdown(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5] if len(sys.argv) > 5 else "")
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]), int(sys.argv[6]), sys.argv[7], sys.argv[8],
                sys.argv[9])
    elif sys.argv[1] == "sq":
        sq_summary(sys.argv[2], sys.argv[3], int(sys.argv[4]), sys.argv[5], sys.argv[6])
    else:
        raise SystemExit(__doc__)
