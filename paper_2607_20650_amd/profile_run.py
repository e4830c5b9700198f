"""Short, profiler-friendly run of one update kernel (D2Q9, or the D3Q19
extension with --workload sphere-array-256) plus a copy kernel of known size
(the calibration reference for memory counters).

    rocprofv3 --kernel-trace --stats -d <dir> -- python -m paper_2607_20650_amd.profile_run
    rocprofv3 --pmc FETCH_SIZE -d <dir> -- python -m paper_2607_20650_amd.profile_run
    rocprofv3 --pmc WRITE_SIZE -d <dir> -- python -m paper_2607_20650_amd.profile_run

Updates are launched one by one (no graphs) so every dispatch is visible.
"""
from __future__ import annotations

import argparse
import sys


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--scheme", default="NPTL")
    ap.add_argument("--layout", default="stream")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--workload", default="karman", choices=["karman", "channel-16000x8000", "sphere-array-256"])
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--probe-bytes", type=int, default=1 << 30)
    args = ap.parse_args()

    import torch

    from paper_2607_20650_amd import lbm, workloads
    if args.workload == "sphere-array-256":  # the D3Q19 extension
        sc3 = workloads.sphere_array(n=256)
        print(f"profile_run: {sc3.name} {args.scheme}/{args.layout}/{args.precision} {args.steps} updates", flush=True)
        with lbm.Simulation3.from_scenario(sc3, scheme=args.scheme, layout=args.layout,
                                           precision=args.precision) as sim:
            for k in range(args.steps):
                sim.step(1)
            sim.sync()
            print("profile_run: updates done", flush=True)
        gbs = lbm.bandwidth_probe("copy", args.probe_bytes, reps=1)
        print(f"profile_run: copy probe {args.probe_bytes} bytes each way, {gbs:.0f} GB/s", flush=True)
        torch.cuda.synchronize()
        return 0
    if args.workload == "karman":
        sc = workloads.karman()
    else:
        sc = workloads.channel(nx=16000, ny=8000)
    print(f"profile_run: {args.workload} {sc.nx}x{sc.ny} {args.scheme}/{args.layout}/{args.precision} "
          f"{args.steps} updates", flush=True)
    with lbm.Simulation.from_scenario(sc, scheme=args.scheme, layout=args.layout, precision=args.precision,
                                      bundle=0) as sim:
        for k in range(args.steps):
            sim.step(1)
        sim.sync()
        st, d = sim.diag()
        print(f"profile_run: updates done, diag status {st}, mass {d[0]:.6f}", flush=True)
    gbs = lbm.bandwidth_probe("copy", args.probe_bytes, reps=1)
    print(f"profile_run: copy probe {args.probe_bytes} bytes each way, {gbs:.0f} GB/s", flush=True)
    torch.cuda.synchronize()
    return 0


if __name__ == "__main__":
    sys.exit(main())
