"""Summarises rocprofv3 CSV output of the benchmark into short text files.

Usage (after the runs described in each summary's header):

    python -m paper_2405_12520_amd.profile_summary \\
        --trace <dir>/run_kernel_stats.csv \\
        --fetch <dir>/run_counter_collection.csv --write <dir>/run_counter_collection.csv \\
        --copy-bytes 268435456 --vehicles 2000000 --out profiles/<name>

Writes ``<name>.md`` (per-kernel durations, HBM byte counters per launch,
calibrated by a plain copy of known size measured in the same runs) and
``profiles/traffic.json`` (bytes per launch of each kernel, keyed by a hash of
the kernel sources so that stale numbers are not reported).
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def kernel_sources_sha() -> str:
    h = hashlib.sha256()
    for f in ("moss_kernels.hip", "moss_internal.h", "moss_mlp.h"):
        with open(os.path.join(ROOT, "paper_2405_12520_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short(name: str) -> str:
    name = name.split("(")[0]
    if name.startswith("void "):
        name = name[5:]
    return name.replace("moss::", "")


def counter_means(path, counter, kernel_filter=None):
    """Mean counter value (KiB per dispatch) per kernel, skipping the first
    dispatch of each moss kernel (the one after creation)."""
    vals = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        vals[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    out = {}
    for k, v in vals.items():
        if k.startswith("k_") and len(v) > 2:
            v = v[2:]
        out[k] = sum(v) / len(v)
    return out


def copy_probe_kib(path, counter, copy_bytes):
    """Counter reading of the largest copy/elementwise kernel whose dispatch
    moved exactly copy_bytes (the probe)."""
    best = None
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        n = r["Kernel_Name"]
        if "copyBuffer" in n or "elementwise" in n or "copy" in n.lower():
            v = float(r["Counter_Value"])
            if best is None or v > best:
                best = v
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-bytes", type=int, default=268435456)
    ap.add_argument("--vehicles", type=int, default=2_000_000)
    ap.add_argument("--out", required=True)
    ap.add_argument("--title", default="city snapshot, 2M vehicles")
    ap.add_argument("--command", default="")
    ap.add_argument("--sq", help="counter CSV of a pass over SQ_WAVES, SQ_WAVE_CYCLES, "
                                 "SQ_BUSY_CYCLES, SQ_WAIT_INST_ANY, SQ_INSTS_VALU, "
                                 "SQ_INSTS_LDS, SQ_INSTS_SALU, SQ_ACTIVE_INST_VALU")
    ap.add_argument("--sq-command", default="")
    ap.add_argument("--waits", help="counter CSV of a pass over SQ_WAVES, SQ_WAIT_ANY, "
                                    "SQ_ACTIVE_INST_ANY, SQ_INSTS_VMEM_RD, SQ_INSTS_VMEM_WR "
                                    "(needs --sq for the wave cycles)")
    ap.add_argument("--waits-command", default="")
    ap.add_argument("--note", default="", help="closing paragraph")
    ap.add_argument("--no-traffic-json", action="store_true",
                    help="keep traffic.json as it is (a workload other than the benchmark's)")
    args = ap.parse_args()

    rows = list(csv.DictReader(open(args.trace)))
    # the same durations without each step kernel's first two dispatches (the
    # steps right after creation), from the per-dispatch trace beside the stats
    steady = {}
    trace_csv = os.path.join(os.path.dirname(args.trace),
                             os.path.basename(args.trace).replace("kernel_stats", "kernel_trace"))
    if trace_csv != args.trace and os.path.exists(trace_csv):
        per = collections.defaultdict(list)
        for r in csv.DictReader(open(trace_csv)):
            per[short(r["Kernel_Name"])].append(
                (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1000.0)
        steady = {k: sum(v[2:]) / len(v[2:]) for k, v in per.items()
                  if k.startswith("k_") and len(v) > 2}
    lines = [f"# rocprofv3 summary: {args.title}", ""]
    if args.command:
        lines += ["Commands (from the repository root):", "", "```", args.command, "```", ""]
    lines += ["## Kernel durations (rocprofv3 --kernel-trace --stats)", "",
              "The last column leaves out each step kernel's first two dispatches (the steps "
              "right after creation), as the byte and instruction counters below do.", "",
              "| kernel | calls | avg us | min us | max us | share | avg us after 2 |",
              "|---|---|---|---|---|---|---|"]
    dur = {}
    for r in rows:
        k = short(r["Name"])
        dur[k] = float(r["AverageNs"]) / 1000.0
        st = f"{steady[k]:.2f}" if k in steady else "-"
        lines.append(f"| {k} | {r['Calls']} | {float(r['AverageNs'])/1e3:.2f} | "
                     f"{float(r['MinNs'])/1e3:.2f} | {float(r['MaxNs'])/1e3:.2f} | "
                     f"{float(r['Percentage']):.1f}% | {st} |")
    traffic = {}
    if args.fetch and args.write:
        f = counter_means(args.fetch, "FETCH_SIZE")
        w = counter_means(args.write, "WRITE_SIZE")
        pf = copy_probe_kib(args.fetch, "FETCH_SIZE", args.copy_bytes)
        pw = copy_probe_kib(args.write, "WRITE_SIZE", args.copy_bytes)
        true_kib = args.copy_bytes / 1024.0
        sf = true_kib / pf if pf else 1.0
        sw = true_kib / pw if pw else 1.0
        lines += ["", "## HBM bytes per launch (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE)", "",
                  f"Calibration: a device copy of {args.copy_bytes} bytes reads "
                  f"FETCH_SIZE = {pf:.0f} KiB and WRITE_SIZE = {pw:.0f} KiB; scale factors "
                  f"{sf:.3f} (fetch) and {sw:.3f} (write) are applied below.", "",
                  "| kernel | fetch MB | write MB | total MB | B per vehicle | GB/s at the steady duration |",
                  "|---|---|---|---|---|---|"]
        for k in sorted(set(f) & set(w)):
            if not k.startswith("k_"):
                continue
            fb = f[k] * 1024 * sf
            wb = w[k] * 1024 * sw
            tot = fb + wb
            traffic[k] = dict(bytes_per_launch=tot, fetch=fb, write=wb)
            dk = steady.get(k, dur.get(k, 0.0))
            gbs = tot / (dk * 1e-6) / 1e9 if dk else 0.0
            lines.append(f"| {k} | {fb/1e6:.1f} | {wb/1e6:.1f} | {tot/1e6:.1f} | "
                         f"{tot/args.vehicles:.1f} | {gbs:.0f} |")
        rec = dict(source_sha=kernel_sources_sha(), vehicles=args.vehicles,
                   calibration=dict(copy_bytes=args.copy_bytes, fetch_kib=pf, write_kib=pw),
                   kernels=traffic)
        if not args.no_traffic_json:
            with open(os.path.join(os.path.dirname(args.out) or ".", "traffic.json"), "w") as fh:
                json.dump(rec, fh, indent=1)
    if args.sq:
        names = ("SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS",
                 "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_VALU")
        per = {n: counter_means(args.sq, n) for n in names}
        lines += ["", "## Instruction counters per wave (rocprofv3 --pmc, one pass)", ""]
        if args.sq_command:
            lines += ["```", args.sq_command, "```", ""]
        lines += ["| kernel | waves | VALU | SALU | LDS | wave cycles | waiting on instructions |",
                  "|---|---|---|---|---|---|---|"]
        for k in sorted(per["SQ_WAVES"]):
            if not k.startswith("k_"):
                continue
            w = per["SQ_WAVES"][k] or 1.0
            g = lambda n: per[n].get(k, 0.0) / w
            lines.append(f"| {k} | {per['SQ_WAVES'][k]:.0f} | {g('SQ_INSTS_VALU'):.0f} | "
                         f"{g('SQ_INSTS_SALU'):.0f} | {g('SQ_INSTS_LDS'):.0f} | "
                         f"{g('SQ_WAVE_CYCLES'):.0f} | {g('SQ_WAIT_INST_ANY'):.0f} |")
    if args.waits and args.sq:
        names = ("SQ_WAVES", "SQ_WAIT_ANY", "SQ_ACTIVE_INST_ANY", "SQ_INSTS_VMEM_RD",
                 "SQ_INSTS_VMEM_WR")
        per = {n: counter_means(args.waits, n) for n in names}
        cyc = counter_means(args.sq, "SQ_WAVE_CYCLES")
        waves = counter_means(args.sq, "SQ_WAVES")
        lines += ["", "## Where the waves' time goes (second counter pass)", ""]
        if args.waits_command:
            lines += ["```", args.waits_command, "```", ""]
        lines += ["Per wave, in the units of the wave cycles above (their ratios are what "
                  "matter): cycles waiting on anything (memory, barriers, dependencies), cycles "
                  "issuing any instruction, and vector memory instructions.", "",
                  "| kernel | wave cycles | waiting | issuing | waiting share | issuing share "
                  "| VMEM reads | VMEM writes |", "|---|---|---|---|---|---|---|---|"]
        for k in sorted(per["SQ_WAVES"]):
            if not k.startswith("k_") or not waves.get(k):
                continue
            w = per["SQ_WAVES"][k] or 1.0
            wc = cyc.get(k, 0.0) / waves[k]
            g = lambda n: per[n].get(k, 0.0) / w
            wa, ac = g("SQ_WAIT_ANY"), g("SQ_ACTIVE_INST_ANY")
            lines.append(f"| {k} | {wc:.0f} | {wa:.0f} | {ac:.0f} | {wa / wc:.2f} | "
                         f"{ac / wc:.2f} | {g('SQ_INSTS_VMEM_RD'):.1f} | "
                         f"{g('SQ_INSTS_VMEM_WR'):.1f} |")
    if args.note:
        lines += ["", args.note]
    with open(args.out + ".md", "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
