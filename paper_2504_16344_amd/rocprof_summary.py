"""Summaries of rocprofv3 output for profiles/: kernel-trace statistics and
calibrated HBM byte counters (FETCH_SIZE, WRITE_SIZE).

The byte counters are calibrated on a plain device copy of known size that
runs in the same profiled command: scale = bytes moved / counter reading.

Matrix-core utilisation of the multi-right-hand-side products comes from
the SQ counters: SQ_VALU_MFMA_BUSY_CYCLES (busy cycles summed over all
SIMDs) over the SIMD-cycles of the dispatch (1024 SIMDs times the
per-XCD GRBM_GUI_ACTIVE cycles, GRBM_GUI_ACTIVE being summed over the 8
XCDs); the same counters give the shader clock during the dispatch.

Usage:
  python -m paper_2504_16344_amd.rocprof_summary trace STATS_CSV OUT_MD TITLE CMD
  python -m paper_2504_16344_amd.rocprof_summary counters FETCH_CSV WRITE_CSV OUT_MD OUT_JSON \
         COPY_BYTES CMD_FETCH CMD_WRITE
  python -m paper_2504_16344_amd.rocprof_summary mfma SQ_CSV FETCH_CSV WRITE_CSV OUT_MD \
         COPY_BYTES TITLE CMD_SQ CMD_FETCH CMD_WRITE
"""
from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import re
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
# Sources of the single-right-hand-side product kernels the counters cover.
PRODUCT_SOURCES = (os.path.join(PKG, "csrc", "gemv.hip"),
                   os.path.join(PKG, "csrc", "product_units.h"))
COPY_KERNEL = "__amd_rocclr_copyBuffer"
SIMDS = 1024   # 256 compute units x 4 SIMDs
XCDS = 8


def source_digest(paths=PRODUCT_SOURCES) -> str:
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def short_name(name: str) -> str:
    n = name.replace("(p2o::Fmt16)0", "FP16").replace("(p2o::Fmt16)1", "BF16")
    n = n.replace("void ", "").replace("p2o::(anonymous namespace)::", "")
    n = n.replace("(anonymous namespace)::", "")
    if n.startswith("__"):
        return n
    depth, out = 0, []
    for ch in n:  # drop the argument list, keep template arguments
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out).strip()


def family(kname: str):
    """(precision tier, op) of a block-product kernel name, else None."""
    op = "F" if kname.startswith("gemv_rows") else "FADJ" if kname.startswith("gemv_cols") else None
    if op is None:
        return None
    if "_f64_" in kname:
        return ("fp64", op)
    if "FP16, true" in kname:
        return ("mixed_fp16", op)
    if "BF16, true" in kname:
        return ("mixed_bf16", op)
    if "BF16, false" in kname:
        return ("fast_bf16", op)
    return None


def trace_md(stats_csv: str, out_md: str, title: str, cmd: str) -> None:
    rows = list(csv.DictReader(open(stats_csv)))
    lines = [f"# {title}", "", "Command (from /tmp with TMPDIR=/tmp; R = repository root):", "",
             "```", cmd, "```", "",
             "| kernel | calls | avg us | min us | max us | total % |", "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} "
                     f"| {float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} "
                     f"| {float(r['Percentage']):.2f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")


def counters(fetch_csv: str, write_csv: str, out_md: str, out_json: str, copy_bytes: float,
             cmds: list[str]) -> dict:
    vals = collections.defaultdict(list)
    for path in (fetch_csv, write_csv):
        for r in csv.DictReader(open(path)):
            vals[(short_name(r["Kernel_Name"]), r["Counter_Name"])].append(float(r["Counter_Value"]))
    known_kb = copy_bytes / 1024.0
    fetch_scale = known_kb / max(vals[(COPY_KERNEL, "FETCH_SIZE")])
    write_scale = known_kb / max(vals[(COPY_KERNEL, "WRITE_SIZE")])
    names = sorted({k for k, _ in vals}, key=lambda k: -max(vals.get((k, "FETCH_SIZE"), [0])))
    kernels = {}
    for k in names:
        f = vals.get((k, "FETCH_SIZE"), [0.0])
        w = vals.get((k, "WRITE_SIZE"), [0.0])
        kernels[k] = {"dispatches": len(f),
                      "read_bytes": sum(f) / len(f) * fetch_scale * 1024,
                      "write_bytes": sum(w) / len(w) * write_scale * 1024}
    fams = {}
    for k, v in kernels.items():
        fam = family(k)
        if fam is None:
            continue
        key = f"{fam[0]}/{fam[1]}"
        if key not in fams or v["dispatches"] > kernels[fams[key]]["dispatches"]:
            fams[key] = k
    out = {"source": [os.path.relpath(p, os.path.dirname(PKG)) for p in PRODUCT_SOURCES],
           "source_sha256": source_digest(),
           "fetch_scale": fetch_scale, "write_scale": write_scale, "commands": cmds,
           "kernels": kernels, "by_family": fams}
    json.dump(out, open(out_json, "w"), indent=1)
    lines = ["# HBM byte counters (FETCH_SIZE, WRITE_SIZE)", "",
             "Two separate counter runs, commands (from /tmp with TMPDIR=/tmp; R = repository root):",
             "", "```", *cmds, "```", "",
             f"Calibration: the plain device copy of {copy_bytes / 1e9:.0f} GB in the same command "
             f"(`{COPY_KERNEL}`, largest dispatch) gives FETCH_SIZE x {fetch_scale:.4f} and "
             f"WRITE_SIZE x {write_scale:.4f} = bytes actually moved; the figures below are scaled.",
             "", f"Product-kernel source digest: `{out['source_sha256'][:16]}`", "",
             "| kernel | dispatches | read GB / dispatch | write GB / dispatch |", "|---|---|---|---|"]
    for k, v in kernels.items():
        lines.append(f"| `{k}` | {v['dispatches']} | {v['read_bytes'] / 1e9:.3f} | "
                     f"{v['write_bytes'] / 1e9:.3f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")
    return out


def mfma(sq_csv: str, fetch_csv: str, write_csv: str, out_md: str, copy_bytes: float,
         title: str, cmds: list[str]) -> None:
    """Per matrix-core product kernel: dispatches, duration, MFMA
    instructions, MFMA busy fraction, shader clock, calibrated HBM bytes."""
    vals = collections.defaultdict(list)
    dur = collections.defaultdict(list)
    for path in (sq_csv, fetch_csv, write_csv):
        for r in csv.DictReader(open(path)):
            k = short_name(r["Kernel_Name"])
            vals[(k, r["Counter_Name"])].append(float(r["Counter_Value"]))
            if path == sq_csv and r["Counter_Name"] == "GRBM_GUI_ACTIVE":
                dur[k].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9)
    known_kb = copy_bytes / 1024.0
    fetch_scale = known_kb / max(vals[(COPY_KERNEL, "FETCH_SIZE")])
    write_scale = known_kb / max(vals[(COPY_KERNEL, "WRITE_SIZE")])
    mean = lambda v: sum(v) / len(v)
    lines = [f"# {title}", "",
             "Three counter runs, commands (from /tmp with TMPDIR=/tmp; R = repository root):", "",
             "```", *cmds, "```", "",
             "MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (1024 SIMDs x GRBM_GUI_ACTIVE / 8 XCDs); "
             "clock = (GRBM_GUI_ACTIVE / 8) / dispatch time. "
             f"HBM bytes: FETCH_SIZE x {fetch_scale:.4f}, WRITE_SIZE x {write_scale:.4f} "
             f"(calibrated on the plain {copy_bytes / 1e9:.0f} GB device copy, `{COPY_KERNEL}`).",
             "",
             "| kernel | dispatches | avg ms | MFMA instr | MFMA busy | clock GHz | read GB | write GB |",
             "|---|---|---|---|---|---|---|---|"]
    names = sorted({k for (k, c) in vals if c == "SQ_INSTS_MFMA" and max(vals[(k, c)]) > 0},
                   key=lambda k: -mean(dur[k]) if dur[k] else 0)
    for k in names:
        t = mean(dur[k]) if dur[k] else float("nan")
        busy = mean(vals[(k, "SQ_VALU_MFMA_BUSY_CYCLES")])
        gui = mean(vals[(k, "GRBM_GUI_ACTIVE")]) / XCDS
        rd = mean(vals.get((k, "FETCH_SIZE"), [0.0])) * fetch_scale * 1024
        wr = mean(vals.get((k, "WRITE_SIZE"), [0.0])) * write_scale * 1024
        lines.append(f"| `{k}` | {len(dur[k])} | {t * 1e3:.3f} | "
                     f"{mean(vals[(k, 'SQ_INSTS_MFMA')]):.4g} | {busy / (SIMDS * gui):.3f} | "
                     f"{gui / t / 1e9:.2f} | {rd / 1e9:.3f} | {wr / 1e9:.3f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    a = sys.argv[1:]
    if a[0] == "trace":
        trace_md(a[1], a[2], a[3], a[4])
    elif a[0] == "counters":
        counters(a[1], a[2], a[3], a[4], float(a[5]), a[6:])
    elif a[0] == "mfma":
        mfma(a[1], a[2], a[3], a[4], float(a[5]), a[6], a[7:])
    else:
        raise SystemExit(__doc__)
