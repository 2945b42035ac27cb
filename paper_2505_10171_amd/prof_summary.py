"""Summaries of rocprofv3 CSV output for the lbm kernels.

    python -m paper_2505_10171_amd.prof_summary stats KERNEL_STATS_CSV OUT --command "..."
    python -m paper_2505_10171_amd.prof_summary counters --fetch CSV --write CSV \
        --kernel k_fused --probe-bytes BYTES OUT --command "..." --command "..."

``stats`` condenses a ``--kernel-trace --stats`` kernel_stats CSV into a short
table (calls, average and total duration, share of GPU time per kernel).

``sq`` condenses one ``--pmc`` run of SQ counters into per-thread instruction
counts of each kernel (a thread is one lane of a wave: INSTS / WAVES) and the
time the vector-ALU instructions alone take to issue (4 cycles per wave64
instruction on each of the 1,024 SIMDs at 2.4 GHz).

``counters`` turns two ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs into HBM
bytes per launch of each kernel named (``--kernel`` regex, repeatable).  Both runs must contain one plain device copy of
known size (the largest ``__amd_rocclr_copyBuffer`` dispatch): each counter is
scaled by (copy bytes / what the same counter reads for that copy), which
calibrates the counter's unit and coverage on this chip.  The summary records a
hash of the kernel sources so that consumers can tell when it is stale.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os
import re
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(HERE, "csrc", "lbm_fluid.hip"),
                  os.path.join(HERE, "csrc", "lbm_device.h"),
                  os.path.join(HERE, "csrc", "lbm_api.hip")]


def kernel_sources_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    m = re.match(r"(?:void )?([\w:]+(?:<[^()]*>)?)\(", name)
    return m.group(1) if m else name[:60]


def stats(path, out, commands):
    rows = list(csv.DictReader(open(path)))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# kernel time summary (rocprofv3 --kernel-trace --stats)", ""]
    for c in commands:
        lines.append(f"command: {c}")
    lines += ["", f"{'kernel':60s} {'calls':>7s} {'avg_us':>10s} {'total_ms':>10s} {'share':>7s}"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        lines.append(f"{short_name(r['Name']):60s} {int(r['Calls']):7d} "
                     f"{float(r['AverageNs']) / 1e3:10.2f} {float(r['TotalDurationNs']) / 1e6:10.3f} "
                     f"{100 * float(r['TotalDurationNs']) / total:6.2f}%")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _per_kernel(path, counter):
    vals, probe = {}, []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        v = float(r["Counter_Value"])
        name = r["Kernel_Name"]
        if "copyBuffer" in name:
            probe.append(v)
        else:
            vals.setdefault(short_name(name), []).append(v)
    return vals, probe


def counters(fetch, write, kernels, probe_bytes, out, commands):
    """HBM bytes per launch of each kernel matching one of the regexes in
    `kernels`, from a FETCH_SIZE run and a WRITE_SIZE run."""
    lines = ["# HBM traffic per launch from rocprofv3 counters", ""]
    for c in commands:
        lines.append(f"command: {c}")
    lines.append("")
    result = {}
    for label, path, ctr in (("fetch", fetch, "FETCH_SIZE"), ("write", write, "WRITE_SIZE")):
        vals, probe = _per_kernel(path, ctr)
        if not probe:
            raise SystemExit(f"{path}: no copy probe dispatch")
        pk = max(probe)  # KiB reported for the probe copy
        scale = probe_bytes / (pk * 1024.0)
        lines.append(f"{ctr}: copy probe {probe_bytes:.0f} B reads as {pk:.1f} KiB -> scale {scale:.4f}")
        for kern in kernels:
            ks = [k for k in vals if re.search(kern, k)]
            if not ks:
                raise SystemExit(f"{path}: no dispatch of {kern}")
            k = ks[0]
            kib = statistics.mean(vals[k])
            result.setdefault(k, {})[label] = kib * 1024.0 * scale
            lines.append(f"  {k}: {len(vals[k])} dispatches, mean {kib:.1f} KiB -> "
                         f"{result[k][label]:.4e} B per launch")
    lines.append("")
    for k, r in result.items():
        lines.append(f"bytes_per_launch[{k}]: fetch {r['fetch']:.6e} write {r['write']:.6e} "
                     f"total {r['fetch'] + r['write']:.6e}")
    lines.append(f"kernel_source_sha256_16: {kernel_sources_hash()}")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


SIMDS, CLOCK_HZ, VALU_CYCLES = 1024, 2.4e9, 4


def sq(path, out, commands):
    """Per-kernel means of every SQ counter in one --pmc run, with per-thread
    instruction counts and the vector-ALU issue time."""
    per = {}
    for r in csv.DictReader(open(path)):
        name = short_name(r["Kernel_Name"])
        per.setdefault(name, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    lines = ["# SQ counters per launch (rocprofv3 --pmc)", ""]
    for c in commands:
        lines.append(f"command: {c}")
    lines.append("")
    for name, ctr in per.items():
        m = {k: statistics.mean(v) for k, v in ctr.items()}
        lines.append(f"{name}: {len(next(iter(ctr.values())))} dispatches")
        for k in sorted(m):
            lines.append(f"  {k:24s} {m[k]:.4e}")
        waves = m.get("SQ_WAVES", 0.0)
        if waves:
            for k in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS"):
                if k in m:
                    lines.append(f"  {k.lower()}_per_thread  {m[k] / waves:.1f}")
        if "SQ_INSTS_VALU" in m:
            t = m["SQ_INSTS_VALU"] * VALU_CYCLES / (SIMDS * CLOCK_HZ)
            lines.append(f"  valu_issue_us            {t * 1e6:.1f}")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def read_counters(path):
    """{kernel: total HBM bytes per launch} and the source hash of a summary
    written by `counters`."""
    txt = open(path).read()
    out = {}
    for m in re.finditer(r"bytes_per_launch\[(.+?)\]: fetch \S+ write \S+ total (\S+)", txt):
        out[m.group(1)] = float(m.group(2))
    h = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    return out, (h.group(1) if h else None)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("out")
    a.add_argument("--command", action="append", default=[])
    b = sub.add_parser("counters")
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--kernel", action="append", default=[])
    b.add_argument("--probe-bytes", type=float, required=True)
    b.add_argument("out")
    b.add_argument("--command", action="append", default=[])
    c = sub.add_parser("sq")
    c.add_argument("csv")
    c.add_argument("out")
    c.add_argument("--command", action="append", default=[])
    args = ap.parse_args()
    if args.cmd == "sq":
        sq(args.csv, args.out, args.command)
    elif args.cmd == "stats":
        stats(args.csv, args.out, args.command)
    else:
        counters(args.fetch, args.write, args.kernel or ["k_fused"], args.probe_bytes, args.out,
                 args.command)


if __name__ == "__main__":
    main()
