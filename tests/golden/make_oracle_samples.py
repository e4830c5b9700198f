#!/usr/bin/env python3
"""Write oracle reference fields for the full-size long runs.

Calls only the FP64 oracle (oracle/) and the seeded input generators; nothing
from the HIP path.  For each workload it stores, after the workload's full
step count, the oracle's rho - 1 and u on a stratified node set:

  * every updated (fluid or outlet) node within 3 cells (Chebyshev distance,
    periodic wrap) of a node that is not plain fluid -- solid, inlet or
    outlet -- i.e. every node whose update involves a boundary rule or lies
    next to one ("near" stratum);
  * N_INTERIOR further updated nodes drawn uniformly from the rest (seeded,
    "interior" stratum).

The node set is stored as two bit masks over the (ny, nx) grid (numpy
packbits, row-major) and the values as float32 in row-major order of the
selected nodes (float32 keeps |du| / u_max below 1e-7, far under every
tolerance the tests apply).  Also stored: the oracle's u_max over all fluid /
outlet nodes, the slit-style permeability nu <u_x> / g_x over all nodes for
forced workloads, and the FP64 "noise floor": the same run with the initial
populations multiplied by (1 + 2^-24 r), r ~ U[-1, 1] (seed 7), compared with
the unperturbed run (max |du| / u_max over all fluid / outlet nodes) -- the
best agreement any FP32-storage implementation can expect.

    python tests/golden/make_oracle_samples.py [channel] [karman] [porous] [--out DIR]

Run time: two oracle runs per workload (8.2e3 x 2000, 4.2e10 and 8.4e10 node
updates).  The 128x64 channel has fewer nodes than N_INTERIOR, so its file
holds the whole field.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2607_20650_amd import workloads as W  # noqa: E402

N_INTERIOR = 131072
NEAR = 3  # cells


def scenario(name):
    if name == "channel":
        return W.channel(), 2000
    if name == "karman":
        return W.karman(), 10000
    if name == "porous":
        return W.porous(), 20000
    raise ValueError(name)


def near_boundary(types: np.ndarray) -> np.ndarray:
    """Nodes within NEAR cells (Chebyshev, periodic wrap) of a non-fluid node."""
    nonfluid = types != oracle.FLUID
    near = np.zeros_like(nonfluid)
    for dy in range(-NEAR, NEAR + 1):
        for dx in range(-NEAR, NEAR + 1):
            near |= np.roll(nonfluid, (dy, dx), axis=(0, 1))
    return near


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*", default=["karman", "porous"])
    ap.add_argument("--out", default=HERE)
    args = ap.parse_args()
    for name in args.names:
        sc, steps = scenario(name)
        t = time.time()
        o = oracle.Oracle.from_scenario(sc)
        upd = (o.types == oracle.FLUID) | (o.types == oracle.OUTLET)
        o.run(steps)
        rho, ux, uy = o.macros()
        print(f"{name}: oracle {sc.nx}x{sc.ny} {steps} updates in {time.time() - t:.0f}s on {oracle.threads()} "
              f"threads", flush=True)
        umag = np.hypot(ux, uy)
        umax = float(umag[upd].max())
        # perturbed twin
        t = time.time()
        o2 = oracle.Oracle.from_scenario(sc)
        rng = np.random.default_rng(7)
        st = o2.state
        st *= 1.0 + 2.0 ** -24 * (2.0 * rng.random(st.shape) - 1.0)
        o2.set_state(st)
        o2.run(steps)
        _, ux2, uy2 = o2.macros()
        floor = float(np.hypot(ux2 - ux, uy2 - uy)[upd].max() / umax)
        del o2, ux2, uy2
        print(f"{name}: perturbed twin in {time.time() - t:.0f}s, floor {floor:.3e}", flush=True)
        near = near_boundary(o.types) & upd
        rest = np.flatnonzero((upd & ~near).ravel())
        pick = np.random.default_rng(2607).choice(rest, size=min(N_INTERIOR, rest.size), replace=False)
        sel = near.copy()
        sel.ravel()[pick] = True
        extra = {}
        if sc.g[0] != 0.0:
            nu = (sc.tau - 0.5) / 3.0
            extra["permeability"] = nu * float(ux.mean()) / sc.g[0]
        np.savez_compressed(os.path.join(args.out, f"oracle_{name}_{steps}.npz"),
                            sel_bits=np.packbits(sel.ravel()), near_bits=np.packbits(near.ravel()),
                            drho=(rho - 1.0)[sel].astype(np.float32), ux=ux[sel].astype(np.float32),
                            uy=uy[sel].astype(np.float32), umax=umax, floor=floor, steps=steps, nx=sc.nx,
                            ny=sc.ny, tau=sc.tau, near_cells=NEAR, **extra)
        print(f"{name}: wrote {int(sel.sum())} nodes ({int(near.sum())} within {NEAR} cells of a boundary node), "
              f"umax {umax:.6e} {extra}", flush=True)


if __name__ == "__main__":
    main()
