"""Kernel timings and HBM traffic of the decoder from rocprofv3 runs.

Helpers for the profiler runs whose summaries sit in ``profiles/``:

``python -m paper_2606_04268_amd.profiling copycal``
    A plain device copy of 1 GiB (three times), run under
    ``rocprofv3 --pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE`` to calibrate the
    counters: the copy reads and writes exactly 1 GiB, so
    ``1 GiB / counter`` is the factor that turns each counter into bytes.

``python -m paper_2606_04268_amd.profiling trace ...``
    A Markdown summary of a ``rocprofv3 --kernel-trace --stats`` run.

``python -m paper_2606_04268_amd.profiling summarize ...``
    Reads the counter CSVs of a decode run and of the copy run and writes a
    Markdown summary: per decode, the scaled HBM bytes fetched and written by
    each kernel group (setup, parse, levels) beside its algorithmic bytes.
    The summary ends with one machine-readable line (an HTML comment holding
    JSON) that ``bench.py`` reads to fill ``roofline.traffic``, together with
    the SHA-256 of the kernel source it was measured on, so that a changed
    kernel reports no stale traffic.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(HERE, "csrc", "aceapex.hip")
GIB_KIB = 1 << 20  # counters are reported in KiB

EDGE = 12  # level launches of a deep stream listed one by one at each end
GRID_BANDS = (1 << 20, 1 << 18, 1 << 16, 1 << 14, 0)  # grid-size bands of the other level launches
GROUP_OF = {"k_map": "setup", "k_setup": "setup", "k_count": "parse", "k_otiles": "parse", "k_oapply": "parse",
            "k_parse": "parse", "k_level": "levels", "k_tail": "levels"}


def source_sha256() -> str:
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def copycal():
    import torch

    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    b = torch.empty(n, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied 3 x 1 GiB", flush=True)


def _rows(d: str):
    path = d if d.endswith(".csv") else os.path.join(d, "run_counter_collection.csv")
    with open(path) as f:
        return list(csv.DictReader(f))


def _short(name: str) -> str:
    m = re.search(r"::(k_\w+)[(<]", name)
    return m.group(1) if m else name.split("(")[0][:60]


def _label(name: str) -> str:
    """The kernel's name with its template arguments (k_level<false, 1u>)."""
    m = re.search(r"::(k_\w+(?:<[^>]*>)?)\(", name)
    return m.group(1) if m else _short(name)


def calibration(d: str, counter: str) -> float:
    """Bytes per counter unit: 1 GiB over what the counter read for the copy
    dispatches of 1 GiB (the largest dispatches of the copy run)."""
    vals = [float(r["Counter_Value"]) for r in _rows(d) if r["Counter_Name"] == counter
            and "copyBuffer" in r["Kernel_Name"]]
    if not vals:
        raise SystemExit(f"no copy dispatch with {counter} in {d}")
    v = max(vals)
    return GIB_KIB / v * 1024.0


def per_decode(d: str, counter: str):
    """Mean counter value (KiB) per decode for each kernel group; a decode
    starts at each k_setup dispatch (preceded by k_map in a batch)."""
    decodes = []
    cur = None
    for r in sorted(_rows(d), key=lambda r: int(r["Dispatch_Id"])):
        if r["Counter_Name"] != counter:
            continue
        k = _short(r["Kernel_Name"])
        g = GROUP_OF.get(k)
        if g is None:
            continue
        if k == "k_setup" and (cur is None or cur.get("_parsed")):
            cur = {"setup": 0.0, "parse": 0.0, "levels": 0.0, "dispatches": 0}
            decodes.append(cur)
        if cur is None:
            continue
        cur[g] += float(r["Counter_Value"])
        cur["dispatches"] += 1
        if k == "k_parse":
            cur["_parsed"] = True
    if not decodes:
        raise SystemExit(f"no decode found in {d}")
    out = {g: sum(x[g] for x in decodes) / len(decodes) for g in ("setup", "parse", "levels")}
    out["decodes"] = len(decodes)
    out["dispatches_per_decode"] = decodes[-1]["dispatches"]
    return out


def summarize(args):
    import sys

    sys.path.insert(0, os.path.dirname(HERE))
    ff = calibration(args.cal_fetch, "FETCH_SIZE")
    fw = calibration(args.cal_write, "WRITE_SIZE")
    fetch = per_decode(args.fetch, "FETCH_SIZE")
    write = per_decode(args.write, "WRITE_SIZE")
    alg = json.loads(args.algorithmic) if args.algorithmic else {}
    groups = {}
    for g in ("setup", "parse", "levels"):
        fb = fetch[g] * ff
        wb = write[g] * fw
        groups[g] = {"fetch_bytes": round(fb), "write_bytes": round(wb), "traffic_bytes": round(fb + wb)}
        if g in alg:
            groups[g]["algorithmic_bytes"] = alg[g]
            groups[g]["traffic_over_algorithmic"] = round((fb + wb) / alg[g], 3) if alg[g] else None
    lines = [f"# HBM traffic per decode: {args.title}", ""]
    lines += [f"Workload: {args.workload}", ""]
    lines += ["Counters (KiB per dispatch) are scaled by what the same counter reads for a plain",
              f"1 GiB device copy: FETCH_SIZE x {ff / 1024:.3f} KiB-to-KiB, WRITE_SIZE x {fw / 1024:.3f}.",
              f"Decodes in the run: {fetch['decodes']}; kernel dispatches per decode: "
              f"{fetch['dispatches_per_decode']}.", ""]
    lines += ["Commands (from the repository root):", "", "```"]
    lines += args.command
    lines += ["```", ""]
    lines += ["| Kernel group | Fetched (MB) | Written (MB) | Traffic (MB) | Algorithmic (MB) | Traffic / algorithmic |",
              "|---|---|---|---|---|---|"]
    for g, v in groups.items():
        a = v.get("algorithmic_bytes")
        lines.append(f"| {g} | {v['fetch_bytes'] / 1e6:.1f} | {v['write_bytes'] / 1e6:.1f} | "
                     f"{v['traffic_bytes'] / 1e6:.1f} | {a / 1e6:.1f} | {v.get('traffic_over_algorithmic')} |"
                     if a is not None else
                     f"| {g} | {v['fetch_bytes'] / 1e6:.1f} | {v['write_bytes'] / 1e6:.1f} | "
                     f"{v['traffic_bytes'] / 1e6:.1f} | - | - |")
    rec = {"workload": args.key, "source_sha256": source_sha256(), "groups": groups}
    lines += ["", f"<!-- traffic: {json.dumps(rec, sort_keys=True)} -->", ""]
    with open(args.out, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


def trace(args):
    """Markdown summary of a rocprofv3 --kernel-trace --stats run: per-kernel
    statistics, and the kernels of the last decode one by one."""
    with open(os.path.join(args.dir, "run_kernel_stats.csv")) as f:
        stats = list(csv.DictReader(f))
    with open(os.path.join(args.dir, "run_kernel_trace.csv")) as f:
        rows = sorted(csv.DictReader(f), key=lambda r: int(r["Start_Timestamp"]))
    lines = [f"# {args.title}", "", f"Workload: {args.workload}", "",
             "Command (from the repository root):", "", "```"] + args.command + ["```", "",
             "## Per-kernel statistics over the run", "",
             "| Kernel | Calls | Average (us) | Min (us) | Max (us) | Share of GPU time |", "|---|---|---|---|---|---|"]
    for r in stats:
        lines.append(f"| {_label(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f}% |")
    starts = [i for i, r in enumerate(rows) if _short(r["Kernel_Name"]) == "k_setup"]
    if starts:
        i0 = starts[-1]
        seq = []
        for r in rows[i0:]:
            k = _short(r["Kernel_Name"])
            if k not in GROUP_OF and k != "k_seal":
                break
            seq.append(r)
        t0 = int(seq[0]["Start_Timestamp"])
        lines += ["", "## The last decode, kernel by kernel", "",
                  "Start times are relative to `k_setup`; gaps between kernels include the profiler's own.",
                  f"With more than {2 * EDGE} level launches, the first and last {EDGE} are listed one by one and",
                  "the others in bands of grid size (work-items per launch).", "",
                  "| Kernel | Grid (work-items) | Start (us) | Duration (us) |", "|---|---|---|---|"]
        levels = [i for i, r in enumerate(seq) if _short(r["Kernel_Name"]) == "k_level"]
        banded = set(levels[EDGE:-EDGE]) if len(levels) > 2 * EDGE else set()
        bands = {}
        lvl = 0
        for i, r in enumerate(seq):
            k = _short(r["Kernel_Name"])
            a, b = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
            label = _label(r["Kernel_Name"])
            if k == "k_level":
                if i in banded:
                    g = int(r["Grid_Size_X"])
                    key = (label, next(lo for lo in GRID_BANDS if g >= lo))
                    bands.setdefault(key, []).append((lvl, b - a))
                    if i == max(banded):
                        for (bl, lo), v in sorted(bands.items(), key=lambda kv: kv[1][0][0]):
                            tot = sum(d for _, d in v)
                            lines.append(f"| {bl}, {len(v)} launches between launch {v[0][0]} and {v[-1][0]} | "
                                         f">= {lo} | | {tot / 1e3:.1f} in all, {tot / len(v) / 1e3:.1f} each |")
                    lvl += 1
                    continue
                label = f"{label} (launch {lvl})"
                lvl += 1
            lines.append(f"| {label} | {r['Grid_Size_X']} | {(a - t0) / 1e3:.1f} | {(b - a) / 1e3:.1f} |")
        grp = {}
        for r in seq:
            g = GROUP_OF.get(_short(r["Kernel_Name"]))
            if g:
                grp[g] = grp.get(g, 0) + int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        lines += ["", "Kernel time of the last decode by group: " +
                  ", ".join(f"{g} {v / 1e3:.1f} us" for g, v in grp.items()) + "."]
        total = (int(seq[-1]["End_Timestamp"]) - t0) / 1e3
        lines += ["", f"First kernel start to last kernel end: {total:.1f} us."]
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def occupancy(args):
    """Registers, scratch, LDS and the compiler's occupancy (waves per SIMD,
    from the launch bounds, registers and LDS) of every kernel, from the
    device compile's kernel-resource-usage remarks."""
    import subprocess
    import tempfile

    root = os.path.dirname(HERE)
    rows = []
    for src in ("aceapex.hip", "tans.hip"):
        with tempfile.TemporaryDirectory() as tmp:
            cmd = [os.environ.get("HIPCC", "/opt/rocm/bin/hipcc"), "--offload-arch=gfx950", "-O3", "-std=c++17",
                   "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I" + os.path.join(root, "include"),
                   "--offload-device-only", "-c", "-Rpass-analysis=kernel-resource-usage",
                   os.path.join(HERE, "csrc", src), "-o", os.path.join(tmp, "dev.o")]
            r = subprocess.run(cmd, capture_output=True, text=True, check=True)
        cur = None
        for line in r.stderr.splitlines():
            m = re.search(r"remark: (?:\S+: )?([A-Za-z ]+(?:\[[^]]+\])?): (\S+) \[-Rpass", line)
            if not m:
                continue
            key, val = m.group(1).strip(), m.group(2)
            if key == "Function Name":
                cur = {"kernel": _demangle(val), "source": src}
                rows.append(cur)
            elif cur is not None:
                cur[key] = val
    lines = ["# Kernel resources and occupancy (gfx950)", "",
             "From the device compile's resource remarks; occupancy is the compiler's waves per SIMD",
             "(of 8) allowed by the launch bounds, registers and LDS of one workgroup.", "",
             "Command (from the repository root):", "", "```",
             "python -m paper_2606_04268_amd.profiling occupancy --out profiles/occupancy_kernels.md", "```", "",
             "| Kernel | Source | VGPRs | SGPRs | Scratch (B/lane) | LDS (B/workgroup) | Occupancy (waves/SIMD) |",
             "|---|---|---|---|---|---|---|"]
    for c in rows:
        if c["kernel"].startswith("__"):
            continue
        lines.append(f"| {c['kernel']} | {c['source']} | {c.get('VGPRs', '?')} | {c.get('TotalSGPRs', '?')} | "
                     f"{c.get('ScratchSize [bytes/lane]', '?')} | {c.get('LDS Size [bytes/block]', '?')} | "
                     f"{c.get('Occupancy [waves/SIMD]', '?')} |")
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _demangle(name: str) -> str:
    import subprocess

    try:
        out = subprocess.run(["c++filt", name], capture_output=True, text=True, check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return name
    return out.replace("(anonymous namespace)::", "")


def load_traffic(path: str):
    """The traffic record of a summary, or None when it is absent or was
    measured on another version of the kernel source."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        m = re.search(r"<!-- traffic: (\{.*\}) -->", f.read())
    if not m:
        return None
    rec = json.loads(m.group(1))
    return rec if rec.get("source_sha256") == source_sha256() else None


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    sub.add_parser("copycal")
    s = sub.add_parser("summarize")
    s.add_argument("--fetch", required=True)
    s.add_argument("--write", required=True)
    s.add_argument("--cal-fetch", required=True)
    s.add_argument("--cal-write", required=True)
    s.add_argument("--algorithmic", default="", help="JSON {group: algorithmic bytes per decode}")
    s.add_argument("--title", required=True)
    s.add_argument("--workload", required=True)
    s.add_argument("--key", required=True)
    s.add_argument("--command", action="append", default=[])
    s.add_argument("--out", required=True)
    o = sub.add_parser("occupancy")
    o.add_argument("--out", required=True)
    t = sub.add_parser("trace")
    t.add_argument("--dir", required=True)
    t.add_argument("--title", required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--command", action="append", default=[])
    t.add_argument("--out", required=True)
    args = ap.parse_args()
    if args.cmd == "copycal":
        copycal()
    elif args.cmd == "trace":
        trace(args)
    elif args.cmd == "occupancy":
        occupancy(args)
    else:
        summarize(args)


if __name__ == "__main__":
    main()
