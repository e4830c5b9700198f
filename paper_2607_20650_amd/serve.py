"""Serving request loop: a Poisson stream of independent simulations.

Two ways to serve the same trace:
  * batched: the continuous-batching engine (lbm_server_*): requests that
    arrive while others run are admitted as slots and memory free up, and all
    resident requests advance together in one batched kernel per update;
  * sequential: one request at a time in arrival order, each as its own
    simulation (lbm_create / lbm_step with cached graphs / lbm_macros).

Latency of a request = time its result is on the host - its arrival time.
Aggregate MLUPS = sum(cells * steps) / makespan.

    python -m paper_2607_20650_amd.serve --requests 2000
    python -m paper_2607_20650_amd.serve --requests 2000 --closed   (saturation only)
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import lbm, workloads


def _pct(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if xs else float("nan")


def run_batched(reqs, rate_scale=1.0, budget=64 << 30, max_slots=512, bundle_steps=50, layout="stream",
                precision="fp32", realtime=True, log=None, keep_results=False):
    """Serve `reqs` (workloads.Request) with the batching engine.  Arrival times
    are multiplied by rate_scale (< 1: faster arrivals).  With realtime=False
    every request is available at t = 0 (closed batch, saturation)."""
    srv = lbm.Server(budget, max_slots=max_slots, bundle_steps=bundle_steps, layout=layout, precision=precision)
    order = sorted(reqs, key=lambda r: r.arrival)
    arrival = {}
    done = {}
    status = {}
    results = {}
    by_id = {}
    k = 0
    occupancy = []
    joined_running = 0
    t0 = time.perf_counter()
    while len(done) < len(order):
        now = time.perf_counter() - t0
        while k < len(order) and (not realtime or order[k].arrival * rate_scale <= now):
            r = order[k]
            sc = r.scenario()
            if srv.stats()["running"] > 0:
                joined_running += 1  # admitted into a batch that is already advancing
            rid = srv.submit_scenario(sc, steps=r.steps)
            by_id[rid] = r
            arrival[rid] = r.arrival * rate_scale if realtime else 0.0
            k += 1
        srv.run_bundle()
        for rid, st in srv.poll():
            st2, rho, u = srv.fetch(rid)
            done[rid] = time.perf_counter() - t0
            status[rid] = st2
            if keep_results:
                results[by_id[rid].rid] = (rho, u)
        s = srv.stats()
        occupancy.append((round(time.perf_counter() - t0, 4), s["running"], s["queued"]))
        if s["running"] == 0 and s["queued"] == 0 and k < len(order) and realtime:
            wait = order[k].arrival * rate_scale - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.05))
    makespan = max(done.values()) - (min(arrival.values()) if arrival else 0.0)
    lat = [done[i] - arrival[i] for i in done]
    lups = sum(r.cells * r.steps for r in order)
    stats = srv.stats()
    srv.close()
    out = {"requests": len(order), "p50_s": _pct(lat, 50), "p99_s": _pct(lat, 99), "mean_s": float(np.mean(lat)),
           "makespan_s": makespan, "aggregate_mlups": lups / makespan / 1e6,
           "failed": sum(1 for v in status.values() if v != lbm.OK), "bundles": stats["bundles"],
           "max_resident": max(o[1] for o in occupancy) if occupancy else 0,
           "submitted_while_running": joined_running,
           "occupancy_timeline": occupancy[:: max(1, len(occupancy) // 200)]}
    if keep_results:
        out["results"] = results
    if log:
        log(f"batched: {out['requests']} requests, p50 {out['p50_s']:.3f}s p99 {out['p99_s']:.3f}s, "
            f"{out['aggregate_mlups']:.0f} MLUPS aggregate, max resident {out['max_resident']}")
    return out


def run_sequential(reqs, rate_scale=1.0, layout="stream", precision="fp32", realtime=True, log=None,
                   bundle_steps=50):
    """Serve the same trace one request at a time (FIFO), each as its own
    simulation with its own cached graphs."""
    order = sorted(reqs, key=lambda r: r.arrival)
    lat = []
    status = []
    t0 = time.perf_counter()
    last_done = 0.0
    for r in order:
        arr = r.arrival * rate_scale if realtime else 0.0
        now = time.perf_counter() - t0
        if realtime and arr > now:
            time.sleep(arr - now)
        sc = r.scenario()
        with lbm.Simulation.from_scenario(sc, scheme="NPTL", layout=layout, precision=precision,
                                          bundle=bundle_steps) as sim:
            sim.step(r.steps)
            rho, u = sim.macros()
        status.append(0 if np.isfinite(u).all() else lbm.EUNSTABLE)
        last_done = time.perf_counter() - t0
        lat.append(last_done - arr)
    first = min(r.arrival for r in order) * rate_scale if realtime else 0.0
    makespan = last_done - first
    lups = sum(r.cells * r.steps for r in order)
    out = {"requests": len(order), "p50_s": _pct(lat, 50), "p99_s": _pct(lat, 99), "mean_s": float(np.mean(lat)),
           "makespan_s": makespan, "aggregate_mlups": lups / makespan / 1e6,
           "failed": sum(1 for v in status if v != 0)}
    if log:
        log(f"sequential: {out['requests']} requests, p50 {out['p50_s']:.3f}s p99 {out['p99_s']:.3f}s, "
            f"{out['aggregate_mlups']:.0f} MLUPS aggregate")
    return out


def serving_study(n=2000, seed=5, load=0.7, calib=None, log=None, run_seq=True, seq_stable=False):
    """Full study: saturation throughput on a closed batch, then the Poisson
    trace at arrival rate load * saturation / E[LUP per request], batched and
    sequential.  With seq_stable, both are also run at load * the sequential
    saturation rate, where one-at-a-time serving keeps up."""
    base = workloads.request_trace(n=n, seed=seed, rate_per_s=1.0)  # arrival gaps ~ Exp(1 s)
    mean_lup = float(np.mean([r.cells * r.steps for r in base]))
    calib_reqs = base[: (calib or min(n, 200))]
    sat = run_batched(calib_reqs, realtime=False, log=None)["aggregate_mlups"]
    lam = load * sat * 1e6 / mean_lup  # requests per second
    scale = 1.0 / lam  # base trace has rate 1/s
    if log:
        log(f"saturation {sat:.0f} MLUPS on {len(calib_reqs)} requests; E[LUP] {mean_lup:.3g}; "
            f"arrival rate {lam:.2f}/s ({load:.0%} of saturation)")
    b = run_batched(base, rate_scale=scale, log=log)
    out = {"trace": {"requests": n, "seed": seed, "mean_lup": mean_lup, "arrival_rate_per_s": lam,
                     "load_vs_saturation": load, "saturation_mlups": sat},
           "batched": {k: v for k, v in b.items() if k != "occupancy_timeline"},
           "occupancy_timeline": b["occupancy_timeline"]}
    if run_seq:
        out["sequential"] = run_sequential(base, rate_scale=scale, log=log)
    if seq_stable:
        sat_seq = run_sequential(calib_reqs, realtime=False)["aggregate_mlups"]
        lam2 = load * sat_seq * 1e6 / mean_lup
        if log:
            log(f"sequential saturation {sat_seq:.0f} MLUPS; second arrival rate {lam2:.2f}/s")
        out["seq_stable"] = {"arrival_rate_per_s": lam2, "sequential_saturation_mlups": sat_seq,
                             "batched": {k: v for k, v in run_batched(base, rate_scale=1.0 / lam2, log=log).items()
                                         if k != "occupancy_timeline"},
                             "sequential": run_sequential(base, rate_scale=1.0 / lam2, log=log)}
    return out


def _brief(r):
    keys = ("p50_s", "p99_s", "aggregate_mlups", "max_resident", "submitted_while_running", "failed")
    return {k: (round(r[k], 4) if isinstance(r[k], float) else r[k]) for k in keys if k in r}


def bench_summary(n=2000, log=None):
    """Serving measurement for bench.py: the seeded 2000-request trace at 70%
    of the batched saturation rate and at 70% of the sequential one (both
    saturation rates calibrated on the trace's first 200 requests as a closed
    batch)."""
    res = serving_study(n=n, log=log, calib=min(n, 200), seq_stable=True)
    out = {"requests": n, "arrival_rate_per_s": round(res["trace"]["arrival_rate_per_s"], 3),
           "batched": _brief(res["batched"]), "sequential": _brief(res.get("sequential", {})),
           "saturation_mlups": round(res["trace"]["saturation_mlups"], 1)}
    st = res["seq_stable"]
    out["at_sequential_load"] = {"arrival_rate_per_s": round(st["arrival_rate_per_s"], 3),
                                 "sequential_saturation_mlups": round(st["sequential_saturation_mlups"], 1),
                                 "batched": _brief(st["batched"]), "sequential": _brief(st["sequential"])}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--load", type=float, default=0.7)
    ap.add_argument("--no-sequential", action="store_true")
    ap.add_argument("--out", default=None)
    ap.add_argument("--closed", action="store_true",
                    help="only the saturation run: every request of the trace available at t = 0")
    args = ap.parse_args()

    def log(m):
        print(m, file=sys.stderr, flush=True)

    if args.closed:
        reqs = workloads.request_trace(n=args.requests, seed=args.seed, rate_per_s=1.0)
        res = {k: v for k, v in run_batched(reqs, realtime=False, log=log).items() if k != "occupancy_timeline"}
    else:
        res = serving_study(n=args.requests, seed=args.seed, load=args.load, log=log,
                            run_seq=not args.no_sequential)
    txt = json.dumps(res)
    if args.out:
        with open(args.out, "w") as f:
            f.write(txt)
    print(txt)


if __name__ == "__main__":
    main()
