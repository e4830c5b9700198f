"""Summarise rocprofv3 output databases into the short text reports kept
under profiles/, and record calibrated HBM traffic per update-kernel launch.

    python -m paper_2607_20650_amd.profile_summary \\
        --trace <trace dir>/run_results.db \\
        --fetch <fetch dir>/run_results.db --write <write dir>/run_results.db \\
        --kernel k_npol --variant bundle/fp32 --workload karman-4096x1024 \\
        --command "<the rocprofv3 commands>" --out profiles/k_npol_bundle_fp32_karman4096x1024.md

FETCH_SIZE / WRITE_SIZE (KiB per dispatch) are scaled by what the same counter
reads for the copy probe of known size in the same run (k_probe_copy moves
probe_bytes each way).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sqlite3
import statistics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def csrc_digest() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2607_20650_amd", "csrc")
    for name in sorted(os.listdir(d)):
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def kernel_stats(db):
    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    con.close()
    return rows


def busy_fraction(db, needle):
    """Fraction of the span from the first to the last dispatch of kernels
    matching `needle` during which at least one of them runs (the union of
    their intervals), plus the span in seconds and the dispatch count."""
    con = sqlite3.connect(db)
    rows = con.execute("select start, end from kernels where name like ? order by start",
                       (f"%{needle}%",)).fetchall()
    con.close()
    if not rows:
        raise SystemExit(f"no kernel matching {needle!r}")
    busy, cur_s, cur_e = 0, rows[0][0], rows[0][1]
    for st, en in rows[1:]:
        if st > cur_e:
            busy += cur_e - cur_s
            cur_s, cur_e = st, en
        else:
            cur_e = max(cur_e, en)
    busy += cur_e - cur_s
    span = max(en for _, en in rows) - rows[0][0]  # to the latest end, not the last start's
    return busy / span, span * 1e-9, len(rows)


def counter_values(db, counter):
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, value from counters_collection where counter_name = ?",
                       (counter,)).fetchall()
    con.close()
    out = {}
    for name, v in rows:
        out.setdefault(name, []).append(float(v))
    return out


def pick(d, needle):
    keys = [k for k in d if needle in k]
    if not keys:
        raise SystemExit(f"no kernel matching {needle!r}: {list(d)[:10]}")
    return keys[0]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--kernel", required=True, help="kernel name fragment, e.g. k_npol")
    ap.add_argument("--template", default="", help="template argument fragment, e.g. '<1, float>'")
    ap.add_argument("--variant", required=True, help="layout/precision, e.g. bundle/fp32")
    ap.add_argument("--workload", required=True)
    ap.add_argument("--nodes", type=int, default=4096 * 1024, help="nodes per launch (0: launches differ, no bandwidth)")
    ap.add_argument("--bytes-per-node", type=int, default=72)
    ap.add_argument("--probe-bytes", type=int, default=1 << 30)
    ap.add_argument("--command", default="")
    ap.add_argument("--out", required=True)
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "pmc_traffic.json"))
    ap.add_argument("--busy", action="store_true",
                    help="report the kernel-busy fraction of the kernel's dispatch span (serving runs)")
    args = ap.parse_args()

    # "k_a+k_b": kernels that alternate launch by launch (the AA scheme's even
    # and odd updates); durations and traffic are averaged over both
    needles = [k + (args.template or "") for k in args.kernel.split("+")]
    # a trailing '<' in the name fragment only keeps 'k3_pull<' from matching
    # 'k3_pull_aos'; labels and the traffic key go without it
    label = "+".join(k.rstrip("<") for k in args.kernel.split("+"))
    needle = needles[0]
    stats = kernel_stats(args.trace)
    lines = [f"# rocprofv3 summary: {label} ({args.variant}) on {args.workload}", ""]
    if args.command:
        lines += ["Commands:", "", "```", args.command.strip(), "```", ""]
    lines += ["## Kernel trace (--kernel-trace --stats)", "", "| kernel | calls | total us | avg us | % |",
              "|---|---|---|---|---|"]
    found = {}
    for name, calls, tot, avg, pct in stats[:12]:
        lines.append(f"| `{name[:90]}` | {calls} | {tot:.1f} | {avg:.2f} | {pct:.1f} |")
        for nd in needles:
            if nd not in found and nd in name:
                found[nd] = (float(tot), int(calls))
    avg_us = None
    if len(found) == len(needles):
        avg_us = sum(t for t, _ in found.values()) / sum(c for _, c in found.values())
    if args.busy:
        frac, span, count = busy_fraction(args.trace, needle)
        lines += ["", f"Kernel-busy fraction: {needle} runs during {frac:.1%} of the {span:.2f} s from its first "
                      f"to its last dispatch ({count} dispatches; the rest is host work between bundles and "
                      f"waits for arrivals)."]
    algo = args.bytes_per_node * args.nodes
    if algo:
        lines += ["", f"Algorithmic bytes per launch: {args.bytes_per_node} B x {args.nodes} nodes = {algo} B."]
    if avg_us and algo:
        lines.append(f"Average launch duration ({' and '.join(n.rstrip('<') for n in needles)}) {avg_us:.2f} us -> "
                     f"{algo / (avg_us * 1e-6) / 1e9:.1f} GB/s "
                     f"algorithmic ({algo / (avg_us * 1e-6) / 8e12:.1%} of 8 TB/s).")
    entry = None
    if args.fetch and args.write:
        f = counter_values(args.fetch, "FETCH_SIZE")
        w = counter_values(args.write, "WRITE_SIZE")
        pf, pw = pick(f, "k_probe_copy"), pick(w, "k_probe_copy")
        probe_kib = args.probe_bytes / 1024.0
        cal_f = probe_kib / statistics.median(f[pf])
        cal_w = probe_kib / statistics.median(w[pw])
        kfs = [pick(f, nd) for nd in needles]
        kws = [pick(w, nd) for nd in needles]
        raw_f = statistics.mean(statistics.median(f[k]) for k in kfs)
        raw_w = statistics.mean(statistics.median(w[k]) for k in kws)
        kf, kw = " + ".join(kfs), " + ".join(kws)
        fetch_b = raw_f * 1024.0 * cal_f
        write_b = raw_w * 1024.0 * cal_w
        lines += ["", "## HBM traffic (--pmc FETCH_SIZE, then --pmc WRITE_SIZE; per dispatch)", "",
                  f"Calibration on k_probe_copy ({args.probe_bytes} B each way): FETCH_SIZE reads "
                  f"{statistics.median(f[pf]):.1f} KiB -> factor {cal_f:.3f}; WRITE_SIZE reads "
                  f"{statistics.median(w[pw]):.1f} KiB -> factor {cal_w:.3f}.", "",
                  "| kernel | FETCH_SIZE KiB (raw, median) | WRITE_SIZE KiB (raw, median) | fetched B (cal.) | "
                  "written B (cal.) | total / algorithmic |", "|---|---|---|---|---|---|",
                  f"| `{kf[:160]}` | {raw_f:.1f} | {raw_w:.1f} | "
                  f"{fetch_b:.4g} | {write_b:.4g} | {(fetch_b + write_b) / algo:.3f} |"]
        entry = {"csrc_digest": csrc_digest(), "bytes_per_launch": round(fetch_b + write_b),
                 "fetch_bytes": round(fetch_b), "write_bytes": round(write_b), "calibration_fetch": cal_f,
                 "calibration_write": cal_w, "algorithmic_bytes": algo, "workload": args.workload}
    lines += ["", f"HIP source digest: {csrc_digest()}"]
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    if entry:
        data = {}
        if os.path.exists(args.traffic_json):
            data = json.load(open(args.traffic_json))
        layout, prec = args.variant.split("/")
        data[f"{label}/{layout}/{prec}"] = entry
        with open(args.traffic_json, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
