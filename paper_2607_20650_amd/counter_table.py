"""Per-kernel hardware counters in one table (cache hit rate, instruction mix),
from rocprofv3 --pmc databases of profile_run, one database per variant.

    rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum SQ_WAVES SQ_INSTS_VALU SQ_INSTS_LDS \\
        SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_INSTS_SALU -d <dir> -o run -- \\
        python3 -m paper_2607_20650_amd.profile_run --scheme ... --steps 4
    python -m paper_2607_20650_amd.counter_table --out profiles/counters.md \\
        --entry "label|<dir>/run_results.db|kernel fragment|nodes per launch" ...

Every counter is the median over the variant's dispatches of the kernel (for
"a+b" fragments, the mean of both kernels' medians).  SQ_INSTS_* count
wavefront instructions, so dividing by SQ_WAVES gives instructions per
wavefront; one wavefront updates 64 nodes in every kernel here (staged and
batched kernels too).
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
    lines += ["L2 hit rate = TCC_HIT / (TCC_HIT + TCC_MISS); instructions are per wavefront (64 nodes).", "",
              "| variant | L2 hit | waves | VALU / wave | SALU / wave | LDS / wave | VMEM loads / wave | "
              "VMEM stores / wave |", "|---|---|---|---|---|---|---|---|"]
    for e in args.entry:
        label, db, needle, nodes = e.split("|")
        parts = [medians(db, n) for n in needle.split("+")]
        c = {k: sum(p.get(k, 0.0) for p in parts) / len(parts) for k in COUNTERS}
        hit = c["TCC_HIT_sum"] / max(1.0, c["TCC_HIT_sum"] + c["TCC_MISS_sum"])
        w = max(1.0, c["SQ_WAVES"])
        lines.append(f"| {label} | {hit:.1%} | {c['SQ_WAVES']:.0f} (nodes/64: {int(nodes) / 64:.0f}) | "
                     f"{c['SQ_INSTS_VALU'] / w:.0f} | {c['SQ_INSTS_SALU'] / w:.0f} | {c['SQ_INSTS_LDS'] / w:.1f} | "
                     f"{c['SQ_INSTS_VMEM_RD'] / w:.1f} | {c['SQ_INSTS_VMEM_WR'] / w:.1f} |")
    os.makedirs(os.path.dirname(args.out) or ".", exist_ok=True)
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
