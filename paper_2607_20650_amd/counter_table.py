"""Per-kernel hardware counters in one table (cache hit rate, instruction mix),
from rocprofv3 --pmc databases of profile_run, one database per variant.

    rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum SQ_WAVES SQ_INSTS_VALU SQ_INSTS_LDS \\
        SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_INSTS_SALU -d <dir> -o run -- \\
        python3 -m paper_2607_20650_amd.profile_run --scheme ... --steps 4
    python -m paper_2607_20650_amd.counter_table --out profiles/counters.md \\
        --entry "label|<dir>/run_results.db|kernel fragment|nodes per launch" ...

Every counter is the median over the variant's dispatches of the kernel (for
"a+b" fragments, the mean of both kernels' medians).  SQ_INSTS_* count
wavefront instructions; they are given per 64 updated nodes (the counter
divided by nodes / 64), which is per wavefront wherever a wavefront updates
64 nodes, and stays comparable where one updates more (a z-marching kernel's
wavefront covers 64 nodes of several planes).
"""
from __future__ import annotations

import argparse
import os
import sqlite3
import statistics

COUNTERS = ["TCC_HIT_sum", "TCC_MISS_sum", "SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS",
            "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR"]


def medians(db: str, needle: str) -> dict:
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, counter_name, value from counters_collection").fetchall()
    con.close()
    per = {}
    for name, ctr, v in rows:
        if needle in name:
            per.setdefault(name, {}).setdefault(ctr, []).append(float(v))
    if not per:
        raise SystemExit(f"no kernel matching {needle!r} in {db}")
    out = {}
    for ctr in COUNTERS:
        vals = [statistics.median(d[ctr]) for d in per.values() if ctr in d]
        if vals:
            out[ctr] = sum(vals) / len(vals)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--entry", action="append", required=True,
                    help="label|database|kernel fragment ('a+b' averages two kernels)|nodes per launch")
    ap.add_argument("--command", default="")
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    lines = ["# Hardware counters per update kernel (rocprofv3 --pmc)", ""]
    if args.command:
        lines += ["Commands:", "", "```", args.command.strip(), "```", ""]
    lines += ["L2 hit rate = TCC_HIT / (TCC_HIT + TCC_MISS); instructions are wavefront instructions per 64 "
              "updated nodes (nodes per wavefront in the third column).", "",
              "| variant | L2 hit | waves | nodes / wave | VALU | SALU | LDS | VMEM loads | VMEM stores |",
              "|---|---|---|---|---|---|---|---|---|"]
    for e in args.entry:
        label, db, needle, nodes = e.split("|")
        parts = [medians(db, n) for n in needle.split("+")]
        c = {k: sum(p.get(k, 0.0) for p in parts) / len(parts) for k in COUNTERS}
        hit = c["TCC_HIT_sum"] / max(1.0, c["TCC_HIT_sum"] + c["TCC_MISS_sum"])
        u = int(nodes) / 64  # units of 64 updated nodes
        per_wave = int(nodes) / max(1.0, c["SQ_WAVES"])
        lines.append(f"| {label} | {hit:.1%} | {c['SQ_WAVES']:.0f} | {per_wave:.0f} | "
                     f"{c['SQ_INSTS_VALU'] / u:.0f} | {c['SQ_INSTS_SALU'] / u:.0f} | {c['SQ_INSTS_LDS'] / u:.1f} | "
                     f"{c['SQ_INSTS_VMEM_RD'] / u:.1f} | {c['SQ_INSTS_VMEM_WR'] / u:.1f} |")
    os.makedirs(os.path.dirname(args.out) or ".", exist_ok=True)
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
