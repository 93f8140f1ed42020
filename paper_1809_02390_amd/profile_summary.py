"""Summaries of rocprofv3 output for one library kernel.

Kernel trace (``--kernel-trace --stats``): per-kernel call count and average
duration from ``<prefix>_kernel_stats.csv``.

Counters (``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE`` runs of
``profile_driver``): HBM bytes per launch of the chosen kernel, each counter
scaled by what it reads for the runtime's copy kernel of known size in the
same run (FETCH_SIZE and WRITE_SIZE are in KiB per dispatch; the copy of
M MiB reads and writes M MiB).  Writes a JSON file that ``bench.py`` reads
as the ``traffic`` of its roofline, keyed by a hash of the kernel sources so
that a stale measurement is not reported.

Instruction counters (one ``--pmc SQ_WAVES SQ_INSTS_VALU SQ_ACTIVE_INST_VALU
... GRBM_GUI_ACTIVE`` run of ``profile_driver``): vector instructions per
lattice update (SQ_INSTS_VALU counts wave instructions; times 64 lanes over
the lattice updates of a launch, its nodes times --updates-per-node) and
the share of SIMD cycles with a vector instruction issued (SQ_ACTIVE_INST_VALU, in quad cycles, times 4 over
256 CUs x 4 SIMDs x GRBM_GUI_ACTIVE / 8, the GRBM count being summed over
the eight XCDs).  Written to a JSON file that ``bench.py`` reads for the
vector-ALU roofline of the kernels bound by it.

Usage:
    python -m paper_1809_02390_amd.profile_summary counters --fetch DIR --write DIR \
        --kernel step_kernel --storage-tag F32 --n-nodes 16777216 --copy-mib 1024 --out FILE
    python -m paper_1809_02390_amd.profile_summary valu --sq DIR --kernel step_kernel \
        --storage-tag F32 --n-nodes 16777216 --out FILE
    python -m paper_1809_02390_amd.profile_summary trace --stats FILE
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))


def kernel_source_hash():
    """Hash of the kernel sources with comments and whitespace removed, so
    that a profile stays current across edits that change no code."""
    h = hashlib.sha256()
    for f in ("lbm_kernels.hip", "lbm_cell.h"):
        with open(os.path.join(PKG, "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def _rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    with open(files[0]) as fh:
        return list(csv.DictReader(fh))


def _mean(rows, counter, match):
    v = [float(r["Counter_Value"]) for r in rows if r["Counter_Name"].startswith(counter) and match(r["Kernel_Name"])]
    if not v:
        raise ValueError(f"no {counter} rows for the kernel")
    return sum(v) / len(v), len(v)


def _copy_mean(rows, counter):
    """Mean counter of the largest copy dispatches: the calibration copies
    (the driver makes them larger than any other copy of the run, which the
    runtime does with the same kernel)."""
    v = [float(r["Counter_Value"]) for r in rows
         if "copyBuffer" in r["Kernel_Name"] and r["Counter_Name"].startswith(counter)]
    if not v:
        raise ValueError("no copy dispatches in the run")
    top = [x for x in v if x >= 0.99 * max(v)]
    return sum(top) / len(top)


def counters(a):
    is_kernel = lambda k: a.kernel in k and (a.storage_tag is None or a.storage_tag in k)
    fr, wr = _rows(a.fetch), _rows(a.write)
    fetch_k, nf = _mean(fr, "FETCH_SIZE", is_kernel)
    write_k, nw = _mean(wr, "WRITE_SIZE", is_kernel)
    copy_f = _copy_mean(fr, "FETCH_SIZE")
    copy_w = _copy_mean(wr, "WRITE_SIZE")
    copy_kib = a.copy_mib * 1024.0
    ff, fw = copy_kib / copy_f, copy_kib / copy_w
    bytes_launch = (fetch_k * ff + write_k * fw) * 1024.0
    doc = {
        "kernel": a.kernel + (f"<{a.storage_tag}>" if a.storage_tag else ""),
        "kernel_sha": kernel_source_hash(), "n_nodes": a.n_nodes,
        "fetch_kib_raw": fetch_k, "write_kib_raw": write_k, "dispatches": [nf, nw],
        "copy_fetch_kib_raw": copy_f, "copy_write_kib_raw": copy_w,
        "fetch_factor": ff, "write_factor": fw,
        "updates_per_node": a.updates_per_node,
        "bytes_per_launch": bytes_launch, "bytes_per_lu": bytes_launch / (a.n_nodes * a.updates_per_node),
        "algorithmic_bytes_per_lu": a.algorithmic,
        "commands": a.command,
    }
    with open(a.out, "w") as fh:
        json.dump(doc, fh, indent=1)
    print(json.dumps(doc, indent=1))


def valu(a):
    is_kernel = lambda k: a.kernel in k and (a.storage_tag is None or a.storage_tag in k)
    per = {}
    for r in _rows(a.sq):
        if is_kernel(r["Kernel_Name"]):
            d = per.setdefault(r["Dispatch_Id"], {})
            d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    per = [d for d in per.values() if d.get("SQ_WAVES", 0.0) > 0]
    if not per:
        raise ValueError("no SQ rows for the kernel")
    m = {k: sum(d[k] for d in per) / len(per) for k in per[0]}
    doc = {
        "kernel": a.kernel + (f"<{a.storage_tag}>" if a.storage_tag else ""),
        "kernel_sha": kernel_source_hash(), "n_nodes": a.n_nodes, "dispatches": len(per),
        "waves": m["SQ_WAVES"], "valu_instr_per_wave": m["SQ_INSTS_VALU"] / m["SQ_WAVES"],
        "updates_per_node": a.updates_per_node,
        "valu_lane_instr_per_lu": m["SQ_INSTS_VALU"] * 64.0 / (a.n_nodes * a.updates_per_node),
        "valu_busy": m["SQ_ACTIVE_INST_VALU"] * 4.0 / (256 * 4 * m["GRBM_GUI_ACTIVE"] / 8.0),
        "commands": a.command,
    }
    with open(a.out, "w") as fh:
        json.dump(doc, fh, indent=1)
    print(json.dumps(doc, indent=1))


def short_name(name):
    """Kernel name without argument list and namespaces."""
    s = name[5:] if name.startswith("void ") else name
    for ns in ("lbm::(anonymous namespace)::", "at::native::"):
        s = s.replace(ns, "")
    return s.split("(")[0]


def trace(a):
    """Per-kernel table of the --stats file, then the same per (kernel, grid)
    from the dispatch trace: one kernel launched on several lattice sizes has
    one row per size."""
    with open(a.stats) as fh:
        rows = list(csv.DictReader(fh))
    print("| kernel | calls | total (us) | average (us) | share |")
    print("|---|---|---|---|---|")
    for r in rows:
        print(f"| {short_name(r['Name'])[:100]} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e3:.1f} | "
              f"{float(r['AverageNs']) / 1e3:.3f} | {float(r['Percentage']):.2f} % |")
    if not a.dispatches:
        return
    with open(a.dispatches) as fh:
        disp = list(csv.DictReader(fh))
    groups = {}
    for r in disp:
        key = (short_name(r["Kernel_Name"]), int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]))
        groups.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    print()
    print("| kernel | work-items | calls | average (us) | min (us) |")
    print("|---|---|---|---|---|")
    for (k, g), v in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        if sum(v) >= a.min_total_us:
            print(f"| {k[:100]} | {g} | {len(v)} | {sum(v) / len(v):.3f} | {min(v):.3f} |")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("counters")
    c.add_argument("--fetch", required=True)
    c.add_argument("--write", required=True)
    c.add_argument("--kernel", required=True)
    c.add_argument("--storage-tag", default=None)
    c.add_argument("--n-nodes", type=int, required=True)
    c.add_argument("--copy-mib", type=float, default=1024)
    c.add_argument("--algorithmic", type=float, default=None)
    c.add_argument("--updates-per-node", type=int, default=1, help="lattice updates per node per launch")
    c.add_argument("--out", required=True)
    c.add_argument("--command", action="append", default=[], help="the rocprofv3 command lines (recorded)")
    v = sub.add_parser("valu")
    v.add_argument("--sq", required=True)
    v.add_argument("--kernel", required=True)
    v.add_argument("--storage-tag", default=None)
    v.add_argument("--n-nodes", type=int, required=True)
    v.add_argument("--updates-per-node", type=int, default=1, help="lattice updates per node per launch")
    v.add_argument("--out", required=True)
    v.add_argument("--command", action="append", default=[], help="the rocprofv3 command line (recorded)")
    t = sub.add_parser("trace")
    t.add_argument("--stats", required=True)
    t.add_argument("--dispatches", default=None, help="the kernel_trace.csv of the same run")
    t.add_argument("--min-total-us", type=float, default=100.0)
    a = ap.parse_args()
    {"counters": counters, "valu": valu, "trace": trace}[a.cmd](a)


if __name__ == "__main__":
    main()
