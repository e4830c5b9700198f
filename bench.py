#!/usr/bin/env python3
"""Throughput benchmark of the D2Q9 BGK lattice update on one MI355X.

Workload: the Karman vortex street case, 4096 x 1024 nodes, circular cylinder
of diameter 128 centred at (1024, 512), equilibrium inlet u_x = 0.05 at x = 0,
zero-gradient outlet, solid walls top and bottom, tau for Re = 100 (0.692).
A "step" is one full lattice update of that grid (stream + collide + boundary
rules).  The headline value is the MLUPS of the fastest FP32 scheme x layout
variant over exactly --steps updates, inputs resident in HBM, bracketed by
device synchronisation and timed with HIP events on the library's stream.

Also reported on the same JSON line:
  * every scheme x layout x precision variant (median of repeated runs),
  * roofline of the dominant update kernel (algorithmic bytes per launch over
    the measured average launch duration, against the 8 TB/s HBM peak),
  * the FP64 CPU oracle timed on the host cores on a bounded sample,
  * an off-cache reference grid and the 2^31-node memory-limit grid,
  * batched-serving latency and throughput when the serving engine is built.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SCHEMES = ["LPTL", "NPTL", "PUSH", "NPOL", "NSOL", "AA"]
LAYOUTS = ["stream", "bundle", "collision"]
PRECISIONS = ["fp32", "fp16s", "fp16sr", "fp16c", "fp16csr"]
GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")
MALL_BYTES = 256 * 2 ** 20  # MI355X Infinity Cache


def load_golden(name):
    """Stored oracle field of a workload (tests/golden/oracle_<name>.npz,
    written by a script that calls only the oracle): values on a stratified
    node set given by a bit mask.  None when absent."""
    path = os.path.join(GOLDEN_DIR, f"oracle_{name}.npz")
    if not os.path.exists(path):
        return None
    z = np.load(path)
    g = {k: z[k] for k in z.files}
    ny, nx = int(g["ny"]), int(g["nx"])
    g["sel"] = np.unpackbits(g["sel_bits"], count=nx * ny).astype(bool).reshape(ny, nx)
    return g


def golden_error(u, g) -> float:
    """max |u - u_oracle| / u_max over the stored nodes."""
    sel = g["sel"]
    d = np.hypot(u[0][sel].astype(np.float64) - g["ux"], u[1][sel].astype(np.float64) - g["uy"])
    return float(d.max() / float(g["umax"]))


def accuracy(lbm, sc, scheme, layout, prec, g):
    """Velocity error after the stored step count and, for forced flows, the
    relative permeability error (nu <u_x> / g_x over all nodes)."""
    n = int(g["steps"])
    with lbm.Simulation.from_scenario(sc, scheme=scheme, layout=layout, precision=prec, bundle=50) as sim:
        sim.step(n)
        _, u = sim.macros()
    out = {"variant": f"{scheme}/{layout}/{prec}", "steps": n, "velocity_error": golden_error(u, g)}
    if "permeability" in g:
        k = (sc.tau - 0.5) / 3.0 * float(u[0].astype(np.float64).mean()) / sc.g[0]
        out["permeability_rel_error"] = abs(k - float(g["permeability"])) / abs(float(g["permeability"]))
    return out


def kernel_name(scheme, layout, precision, tile_x):
    """Update kernel the library launches for a variant on this workload (the
    dispatch rules of the HIP sources: one-wavefront-wide NPOL tiles take the
    lean kernel; 64-wide collision-layout tiles of the two-lattice pull, of AA
    and of the FP32 push take the LDS-staged kernels)."""
    staged = layout == "collision" and tile_x == 64
    if scheme == "NPOL":
        return "k_npol64" if tile_x == 64 else "k_npol"
    if scheme == "NSOL":
        return "k_nsol"
    if scheme == "AA":
        # alternate launches, same bytes each
        return "k_aa_even_aos+k_aa_odd_aos" if staged else "k_aa_even+k_aa_odd"
    if scheme == "NPTL" and staged:
        return "k_nptl_aos"
    if scheme == "PUSH" and staged and precision == "fp32":
        return "k_push_staged"
    return {"LPTL": "k_lptl", "NPTL": "k_nptl", "PUSH": "k_push"}[scheme]


def csrc_digest() -> str:
    """Hash of the HIP sources: a stored PMC traffic figure is valid only for it."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2607_20650_amd", "csrc")
    for name in sorted(os.listdir(d)):
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel_key: str):
    """HBM bytes per launch measured with rocprofv3 PMC counters (committed
    under profiles/), or None when absent or taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except Exception:
        return None
    ent = data.get(kernel_key)
    if not ent or ent.get("csrc_digest") != csrc_digest():
        return None
    return ent.get("bytes_per_launch")


def time_steps(sim, steps, torch):
    """Milliseconds for `steps` updates measured with HIP events on sim.stream."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    sim.step(steps)
    e1.record(sim.stream)
    e1.synchronize()
    return e0.elapsed_time(e1)


def sweep(sc, torch, lbm, steps, reps, schemes, layouts, precisions, log):
    out = {}
    for prec in precisions:
        for scheme in schemes:
            for layout in layouts:
                with lbm.Simulation.from_scenario(sc, scheme=scheme, layout=layout, precision=prec,
                                                  bundle=50) as sim:
                    sim.step(100)
                    sim.sync()
                    ms = [time_steps(sim, steps, torch) for _ in range(reps)]
                mlups = [sc.nx * sc.ny * steps / (m * 1e-3) / 1e6 for m in ms]
                key = f"{scheme}/{layout}/{prec}"
                out[key] = {"mlups_median": round(statistics.median(mlups), 1), "mlups_min": round(min(mlups), 1),
                            "mlups_max": round(max(mlups), 1)}
                log(f"sweep {key:24s} {out[key]['mlups_median']:10.1f} MLUPS")
    return out


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sc, target_s: float, log):
    """The FP64 oracle as it stands, on this host's cores, on a bounded sample
    of the same workload (the full grid for as many updates as fit in about
    target_s seconds), plus the same on one thread."""
    import oracle

    def timed(seconds):
        o = oracle.Oracle.from_scenario(sc)
        o.run(1)  # first touch of the arrays, thread start-up
        t = time.perf_counter()
        o.run(2)
        one = (time.perf_counter() - t) / 2
        steps = int(max(2, min(5000, seconds / max(one, 1e-6))))
        t = time.perf_counter()
        o.run(steps)
        dt = time.perf_counter() - t
        return steps, dt, sc.nx * sc.ny * steps / dt / 1e6

    threads = oracle.threads()
    steps, dt, mlups = timed(target_s)
    log(f"cpu oracle: {steps} updates of {sc.nx}x{sc.ny} in {dt:.2f}s -> {mlups:.1f} MLUPS on {threads} threads")
    oracle.set_threads(1)
    try:
        steps1, dt1, mlups1 = timed(target_s / 4)
    finally:
        oracle.set_threads(threads)
    log(f"cpu oracle, 1 thread: {steps1} updates in {dt1:.2f}s -> {mlups1:.1f} MLUPS")
    return {"value": round(mlups, 2), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{steps} updates of the full {sc.nx}x{sc.ny} Karman grid, FP64 two-lattice pull, "
                      f"{dt:.1f} s wall",
            "value_1core": round(mlups1, 2), "sample_1core": f"{steps1} updates, {dt1:.1f} s wall",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count()}


def memory_limit(torch, lbm, workloads, log, steps=50):
    """The memory-limit workload: a 65536 x 32768 (2^31-node) flat-plate
    channel, FP32, with the one-lattice in-place schemes in bundle and stream
    layouts (77.3 GB of populations), and the two-lattice pull on the
    46341 x 23170 grid of the same footprint for comparison."""
    out = {}
    runs = [((65536, 32768), [("AA", "stream"), ("AA", "bundle"), ("NPOL", "bundle"), ("NPOL", "stream")]),
            ((46341, 23170), [("NPTL", "stream")])]
    for (nx, ny), variants in runs:
        sc = workloads.plate(nx=nx, ny=ny)
        for scheme, layout in variants:
            with lbm.Simulation.from_scenario(sc, scheme=scheme, layout=layout, precision="fp32", bundle=50) as sim:
                sim.step(10)
                sim.sync()
                ms = time_steps(sim, steps, torch)
                dev_gb = sim.info()["device_bytes"] / 1e9
            mlups = nx * ny * steps / (ms * 1e-3) / 1e6
            gbs = mlups * 1e6 * 72 / 1e9
            out[f"plate-{nx}x{ny}/{scheme}/{layout}/fp32"] = {
                "mlups": round(mlups, 1), "algorithmic_gbs": round(gbs, 1), "frac_of_8tbs": round(gbs / HBM_PEAK_GBS, 4),
                "device_gb": round(dev_gb, 1), "steps": steps}
            log(f"memory limit {nx}x{ny} {scheme}/{layout}/fp32: {mlups:.0f} MLUPS, {gbs:.0f} GB/s, "
                f"{dev_gb:.1f} GB on the device")
        del sc
    return out


def hbm_reference(torch, lbm, workloads, log, headline, steps=100):
    """A grid far beyond the 256 MB Infinity Cache (16000 x 8000 channel,
    9.2 GB two-lattice FP32, 4.6 GB one-lattice): the headline variant and
    the best two- and one-lattice variants there show what HBM itself
    sustains.  Each kernel launch is one update, so the event time per update
    is the average launch duration."""
    sc = workloads.channel(nx=16000, ny=8000)
    out = {"workload": f"channel-{sc.nx}x{sc.ny}", "steps": steps, "variants": {}}
    runs = [("NPTL", "stream"), ("AA", "stream"), ("NPOL", "bundle")]
    if headline not in runs:
        runs.append(headline)
    for scheme, layout in runs:
        with lbm.Simulation.from_scenario(sc, scheme=scheme, layout=layout, precision="fp32", bundle=50) as sim:
            sim.step(20)
            sim.sync()
            ms = min(time_steps(sim, steps, torch) for _ in range(3))
            lat_gb = sim.info()["device_bytes"] / 1e9
        mlups = sc.nx * sc.ny * steps / (ms * 1e-3) / 1e6
        gbs = mlups * 1e6 * 72 / 1e9
        out["variants"][f"{scheme}/{layout}/fp32"] = {
            "mlups": round(mlups, 1), "algorithmic_gbs": round(gbs, 1), "frac_of_8tbs": round(gbs / HBM_PEAK_GBS, 4),
            "avg_launch_us": round(ms * 1e3 / steps, 2), "device_gb": round(lat_gb, 2)}
        log(f"hbm reference {sc.nx}x{sc.ny} {scheme}/{layout}/fp32: {mlups:.0f} MLUPS, {gbs:.0f} GB/s")
    return out


def porous_block(torch, lbm, workloads, karman_variants, log, steps=1000, reps=5):
    """The porous-medium workload (2048^2 periodic, random discs, solid
    fraction 0.30, body force): speed of the best FP32 and 16-bit variants
    (the paper's scenario sensitivity: compare with the same variants on the
    Karman case) and, per precision, velocity and permeability errors after
    20000 updates against the stored oracle field."""
    sc = workloads.porous()
    runs = [("NPTL", "stream", "fp32"), ("AA", "stream", "fp32"), ("NPOL", "bundle", "fp32"),
            ("NPTL", "stream", "fp16s"), ("NPTL", "stream", "fp16sr"), ("NPTL", "stream", "fp16c"),
            ("NPTL", "stream", "fp16csr"), ("AA", "stream", "fp16sr")]
    out = {"workload": "porous-2048x2048", "solid_fraction": round(sc.meta["solid_fraction"], 4), "variants": {},
           "accuracy": {}}
    fluid = float((sc.flags == 0).mean())
    for scheme, layout, prec in runs:
        with lbm.Simulation.from_scenario(sc, scheme=scheme, layout=layout, precision=prec, bundle=50) as sim:
            sim.step(100)
            sim.sync()
            ms = [time_steps(sim, steps, torch) for _ in range(reps)]
        mlups = statistics.median(sc.nx * sc.ny * steps / (m * 1e-3) / 1e6 for m in ms)
        key = f"{scheme}/{layout}/{prec}"
        ent = {"mlups_median": round(mlups, 1), "mlups_fluid": round(mlups * fluid, 1)}
        kv = karman_variants.get(key)
        if kv:
            ent["ratio_vs_karman"] = round(mlups / kv["mlups_median"], 4)
        out["variants"][key] = ent
        log(f"porous {key:24s} {mlups:10.1f} MLUPS")
    g = load_golden("porous_20000")
    if g is not None:
        for prec in PRECISIONS:
            cands = {k: v for k, v in out["variants"].items() if k.endswith("/" + prec)}
            k = max(cands, key=lambda k: cands[k]["mlups_median"])
            s_, l_, _ = k.split("/")
            out["accuracy"][prec] = accuracy(lbm, sc, s_, l_, prec, g)
            log(f"porous accuracy {k}: {out['accuracy'][prec]}")
    return out


def channel_block(lbm, workloads, log):
    """The 128 x 64 channel (2000 updates): velocity and permeability errors
    of every precision (NPTL/stream) against the stored oracle field."""
    sc = workloads.channel()
    g = load_golden("channel_2000")
    if g is None:
        return None
    out = {"workload": "channel-128x64", "accuracy": {}}
    for prec in PRECISIONS:
        out["accuracy"][prec] = accuracy(lbm, sc, "NPTL", "stream", prec, g)
        log(f"channel accuracy {prec}: {out['accuracy'][prec]}")
    return out


def d3q19_sweep(torch, lbm, workloads, log, steps=100, reps=5):
    """The D3Q19 extension on a periodic sphere array of 256^3 nodes (16.8M,
    beyond the Infinity Cache even for one 16-bit lattice): MLUPS of every
    scheme x layout in FP32 and of the blocked layout in the 16-bit formats,
    with the algorithmic HBM rate (19 loads + 19 stores per node)."""
    sc = workloads.sphere_array(n=256)
    nodes = int(np.prod(sc.flags.shape))
    out = {"workload": sc.name, "nodes": nodes, "solid_fraction": round(sc.meta["solid_fraction"], 4),
           "variants": {}}
    runs = [(s, l, "fp32") for s in ("NPTL", "AA") for l in ("stream", "collision", "blocked")]
    runs += [(s, "blocked", p) for s in ("NPTL", "AA") for p in ("fp16s", "fp16sr", "fp16c", "fp16csr")]
    for scheme, layout, prec in runs:
        with lbm.Simulation3.from_scenario(sc, scheme=scheme, layout=layout, precision=prec) as sim:
            sim.step(20)
            sim.sync()
            ms = [time_steps(sim, steps, torch) for _ in range(reps)]
        mlups = statistics.median(nodes * steps / (m * 1e-3) / 1e6 for m in ms)
        bpn = 2 * 19 * (4 if prec == "fp32" else 2)
        key = f"{scheme}/{layout}/{prec}"
        out["variants"][key] = {"mlups_median": round(mlups, 1), "gbs": round(mlups * 1e6 * bpn / 1e9, 1),
                                "hbm_frac": round(mlups * 1e6 * bpn / 1e9 / HBM_PEAK_GBS, 4)}
        log(f"d3q19 {key:24s} {mlups:10.1f} MLUPS  {mlups * 1e6 * bpn / 1e9:7.1f} GB/s")
    # memory limit: 1024^3 nodes (2^30) in place, 81.6 GB of FP32 populations
    big = workloads.sphere_array(n=1024, radius=160.0)
    nb = int(np.prod(big.flags.shape))
    with lbm.Simulation3.from_scenario(big, scheme="AA", layout="stream", precision="fp32") as sim:
        sim.step(2)
        sim.sync()
        ms = time_steps(sim, 20, torch)
    mlups = nb * 20 / (ms * 1e-3) / 1e6
    out["memory_limit"] = {"workload": big.name, "nodes": nb, "variant": "AA/stream/fp32", "mlups": round(mlups, 1),
                           "gbs": round(mlups * 1e6 * 152 / 1e9, 1), "lattice_gb": round(nb * 76 / 1e9, 1)}
    log(f"d3q19 memory limit {big.name} AA/stream/fp32: {mlups:.0f} MLUPS, {mlups * 152 / 1e3:.0f} GB/s")
    del big
    # roofline of the fastest FP32 variant: its dominant kernels are HBM bound
    best = max((k for k in out["variants"] if k.endswith("/fp32")), key=lambda k: out["variants"][k]["mlups_median"])
    scheme, layout, _ = best.split("/")
    kern = "k3_aa_even+k3_aa_odd" if scheme == "AA" else "k3_pull"
    v = out["variants"][best]
    out["roofline"] = {"bound": "hbm", "variant": best, "achieved": v["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": v["hbm_frac"], "bytes_per_node": 152,
                       "traffic": stored_traffic(f"{kern}/{layout}/fp32"), "kernel": f"{kern}/{layout}/fp32"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--sweep-steps", type=int, default=1000)
    ap.add_argument("--sweep-reps", type=int, default=5)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-memory-limit", action="store_true", help="skip the 2^31-node plate runs")
    ap.add_argument("--no-d3q19", action="store_true", help="skip the D3Q19 extension sweep")
    ap.add_argument("--scheme", default=None, help="headline variant scheme (default: fastest FP32)")
    ap.add_argument("--layout", default=None)
    ap.add_argument("--cpu-seconds", type=float, default=18.0)
    ap.add_argument("--quiet", action="store_true")
    args = ap.parse_args()

    def log(msg):
        if not args.quiet:
            print(msg, file=sys.stderr, flush=True)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU; runs across several GPUs are not supported (their slab "
              "decomposition is a design, not code). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2607_20650_amd import lbm, workloads

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    sc = workloads.karman()  # 4096 x 1024, Re = 100
    cells = sc.nx * sc.ny
    updated = int((sc.flags == 0).sum() - (sc.flags[:, 0] == 0).sum())  # fluid + outlet, inlet column excluded
    log(f"workload karman {sc.nx}x{sc.ny}, tau={sc.tau:.5f}, fluid fraction "
        f"{1 - sc.flags.mean():.4f}")

    variants = {}
    if not args.no_sweep:
        variants = sweep(sc, torch, lbm, args.sweep_steps, args.sweep_reps, SCHEMES, LAYOUTS, PRECISIONS, log)

    def best(prec):
        cands = {k: v for k, v in variants.items() if k.endswith("/" + prec)}
        if not cands:
            return ("NPTL", "stream")
        k = max(cands, key=lambda k: cands[k]["mlups_median"])
        s, l, _ = k.split("/")
        return s, l

    scheme, layout = best("fp32")
    if args.scheme:
        scheme = args.scheme
    if args.layout:
        layout = args.layout

    # ---- headline: exactly --steps updates of the chosen FP32 variant
    sim = lbm.Simulation.from_scenario(sc, scheme=scheme, layout=layout, precision="fp32", bundle=50)
    sim.step(args.warmup)
    sim.sync()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(sim.stream)
    sim.step(args.steps)
    e1.record(sim.stream)
    sim.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    info = sim.info()
    st, diag = sim.diag()
    sim.close()
    value = cells * args.steps / (ev_ms * 1e-3) / 1e6
    log(f"headline {scheme}/{layout}/fp32: {args.steps} updates, {ev_ms:.1f} ms (events), {wall * 1e3:.1f} ms wall, "
        f"{value:.0f} MLUPS; diag status {st}, mass {diag[0]:.6f}")

    bpu = 72
    launch_s = ev_ms * 1e-3 / args.steps
    achieved = bpu * cells / launch_s / 1e9
    kernel_key = f"{kernel_name(scheme, layout, 'fp32', info['tile_x'])}/{layout}/fp32"
    traffic = stored_traffic(kernel_key)
    # practical peak: plain and non-temporal copies far beyond the caches
    probes = {f"{m}_{sz}gib": round(lbm.bandwidth_probe(m, sz << 30, reps=5), 1)
              for m in ("copy", "copy_nt") for sz in (1, 4)}
    copy_gbs = max(probes.values())
    working_set = info["device_bytes"]
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kernel_key, "bytes_per_launch": bpu * cells, "avg_launch_us": round(launch_s * 1e6, 2),
                "working_set_mb": round(working_set / 2 ** 20, 1),
                "cache_resident": working_set <= MALL_BYTES,
                "copy_probe_gbs": round(copy_gbs, 1), "copy_probes": probes,
                "frac_of_copy_probe": round(achieved / copy_gbs, 4)}
    log(f"copy probes: {probes}")

    # ---- 16-bit storage: speed of the fastest variant of each format, and its
    # velocity error after 10000 updates against the stored FP64 oracle field
    # of this workload (every node within 3 cells of a boundary node plus
    # 131072 interior nodes)
    fp16 = {}
    golden = load_golden("karman_10000")
    v32 = variants.get(f"{scheme}/{layout}/fp32", {}).get("mlups_median", value)
    for prec in ("fp16s", "fp16sr", "fp16c", "fp16csr"):
        if not any(k.endswith("/" + prec) for k in variants):
            continue
        s16, l16 = best(prec)
        v16 = variants[f"{s16}/{l16}/{prec}"]["mlups_median"]
        ent = {"variant": f"{s16}/{l16}", "mlups": v16, "ratio_vs_fp32": round(v16 / v32, 3),
               "hbm_frac": round(v16 * 1e6 * 36 / 1e9 / HBM_PEAK_GBS, 4)}
        if golden is not None:
            ent["velocity_error_after_%d" % int(golden["steps"])] = accuracy(lbm, sc, s16, l16, prec,
                                                                             golden)["velocity_error"]
        fp16[prec] = ent
        log(f"{prec}: {s16}/{l16} {v16:.0f} MLUPS ({ent['ratio_vs_fp32']:.3f}x FP32), "
            f"error {ent.get('velocity_error_after_10000', 'n/a')}")

    serving = None
    if not args.no_serving:
        try:
            from paper_2607_20650_amd import serve
            serving = serve.bench_summary(log=log)
        except ImportError:
            serving = None

    hbm_ref = None if args.no_sweep else hbm_reference(torch, lbm, workloads, log, (scheme, layout))
    roofline_offcache = None
    if hbm_ref:
        hv = hbm_ref["variants"][f"{scheme}/{layout}/fp32"]
        bk = max(hbm_ref["variants"], key=lambda k: hbm_ref["variants"][k]["mlups"])
        roofline_offcache = {
            "bound": "hbm", "workload": hbm_ref["workload"], "variant": f"{scheme}/{layout}/fp32",
            "achieved": hv["algorithmic_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hv["frac_of_8tbs"],
            "avg_launch_us": hv["avg_launch_us"], "frac_of_copy_probe": round(hv["algorithmic_gbs"] / copy_gbs, 4),
            "best_variant": bk, "best_achieved": hbm_ref["variants"][bk]["algorithmic_gbs"],
            "best_frac": hbm_ref["variants"][bk]["frac_of_8tbs"],
            "best_frac_of_copy_probe": round(hbm_ref["variants"][bk]["algorithmic_gbs"] / copy_gbs, 4)}
    porous = None if args.no_sweep else porous_block(torch, lbm, workloads, variants, log)
    channel = channel_block(lbm, workloads, log)
    mem_limit = None if (args.no_sweep or args.no_memory_limit) else memory_limit(torch, lbm, workloads, log)

    d3 = None if (args.no_sweep or args.no_d3q19) else d3q19_sweep(torch, lbm, workloads, log)

    cpu = None if args.no_cpu else cpu_baseline(sc, args.cpu_seconds, log)

    line = {
        "metric": "D2Q9 BGK MLUPS (FP32, best scheme x layout) on the 4096x1024 Karman case",
        "value": round(value, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ev_ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "karman-4096x1024-re100", "nx": sc.nx, "ny": sc.ny, "scheme": scheme,
                   "layout": layout, "storage": "fp32", "tile": [info["tile_x"], info["tile_y"]],
                   "graph_bundle": info["bundle"]},
        "hbm_frac": round(achieved / HBM_PEAK_GBS, 4),
        "mlups_fluid": round(value * updated / cells, 1),
        "roofline": roofline,
        "roofline_offcache": roofline_offcache,
        "cpu_baseline": cpu,
        "fp16": fp16 or None,
        "hbm_reference": hbm_ref,
        "porous": porous,
        "channel": channel,
        "memory_limit": mem_limit,
        "d3q19": d3,
        "serving": serving,
        "variants": variants,
        "wall_ms": round(wall * 1e3, 2),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
