"""Full-size GPU parity at the benchmark workloads' real sizes.

* 4096x1024 Karman case, 10000 updates, and 2048^2 porous medium, 20000
  updates: every scheme x layout x precision against oracle samples stored by
  tests/golden/make_oracle_samples.py (oracle only).  FP32 tolerance
  max(1e-5, stored FP64 noise floor); FP16S-SR (stochastic rounding) <= 1e-2
  on the Karman case; FP16S (round to nearest even) and the porous FP16 errors
  are reported with loose sanity bounds.
* 2^31-node plate grid (65536 x 32768), one-lattice schemes (NPOL, NSOL, AA)
  in bundle and stream layouts, and the 46341 x 23170 two-lattice comparison grid, 200
  updates: interior windows against light-cone-cropped oracle runs (a node's
  value after n updates depends only on nodes within n cells).

Set LBM_REPORT=<path> to also write every measured error to a JSON file.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import INFLOW_OUTFLOW, PERIODIC
from paper_2607_20650_amd import workloads as W
from tests.helpers import ALL_LAYOUTS, ALL_PRECISIONS, ALL_SCHEMES

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
REPORT = {}


def _report(key, value):
    REPORT[key] = value
    path = os.environ.get("LBM_REPORT")
    if path:
        with open(path, "w") as f:
            json.dump(REPORT, f, indent=1, sort_keys=True)


def _golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated (tests/golden/make_oracle_samples.py)")
    return np.load(path)


def _sample_error(u, g):
    dux = u[0][g["y"], g["x"]].astype(np.float64) - g["ux"]
    duy = u[1][g["y"], g["x"]].astype(np.float64) - g["uy"]
    return float(np.hypot(dux, duy).max() / float(g["umax"]))


@pytest.mark.parametrize("precision", ALL_PRECISIONS)
def test_karman_10000_all_variants(precision):
    from paper_2607_20650_amd.lbm import Simulation
    g = _golden("oracle_karman_10000.npz")
    sc = W.karman()
    tol = {"fp32": max(1e-5, float(g["floor"])), "fp16sr": 1e-2, "fp16s": 0.2, "fp16csr": 2e-3, "fp16c": 5e-2}[precision]
    errs = {}
    for scheme in ALL_SCHEMES:
        for layout in ALL_LAYOUTS:
            with Simulation.from_scenario(sc, scheme=scheme, layout=layout, precision=precision, bundle=50) as sim:
                sim.step(int(g["steps"]))
                _, u = sim.macros(device=True)
                sim.sync()
                u = u.cpu().numpy()
            errs[f"{scheme}/{layout}"] = _sample_error(u, g)
    _report(f"karman_10000/{precision}", {"errors": errs, "floor": float(g["floor"]), "tolerance": tol})
    for k, e in errs.items():
        assert e <= tol, (k, precision, e, tol)


@pytest.mark.parametrize("precision", ALL_PRECISIONS)
def test_porous_20000_all_variants(precision):
    from paper_2607_20650_amd.lbm import Simulation
    g = _golden("oracle_porous_20000.npz")
    sc = W.porous()
    tol = max(1e-5, float(g["floor"])) if precision == "fp32" else 0.5
    errs, perm = {}, {}
    nu = (sc.tau - 0.5) / 3.0
    for scheme in ALL_SCHEMES:
        for layout in ALL_LAYOUTS:
            with Simulation.from_scenario(sc, scheme=scheme, layout=layout, precision=precision, bundle=50) as sim:
                sim.step(int(g["steps"]))
                _, u = sim.macros(device=True)
                sim.sync()
                ux_mean = float(u[0].double().mean().item())
                u = u.cpu().numpy()
            errs[f"{scheme}/{layout}"] = _sample_error(u, g)
            perm[f"{scheme}/{layout}"] = nu * ux_mean / sc.g[0]
    k_ref = float(g["permeability"])
    perm_err = {k: abs(v - k_ref) / abs(k_ref) for k, v in perm.items()}
    _report(f"porous_20000/{precision}", {"errors": errs, "floor": float(g["floor"]), "tolerance": tol,
                                          "permeability_ref": k_ref, "permeability_rel_err": perm_err,
                                          "solid_fraction": sc.meta["solid_fraction"]})
    for k, e in errs.items():
        assert np.isfinite(e) and e <= tol, (k, precision, e, tol)
    if precision == "fp32":
        for k, e in perm_err.items():
            assert e <= max(1e-5, float(g["floor"])), (k, e)


# ------------------------------------------------------------- 2^31 nodes
STEPS_BIG = 200
WINDOWS = [  # (x0, x1, y0, y1) interiors to compare; oracle crops add a halo
    (15600, 16500, 16000, 16700),  # plate leading edge / mid-chord region
    (0, 700, 16000, 16500),        # inlet
]


def _crop_check(sim, sc, windows):
    """Compare interior windows of the GPU field with cropped oracle runs."""
    import torch
    _, u = sim.macros(device=True)
    sim.sync()
    h = STEPS_BIG + 2
    worst = 0.0
    for (x0, x1, y0, y1) in windows:
        cx0, cx1 = max(0, x0 - h), min(sc.nx, x1 + h)
        cy0, cy1 = max(0, y0 - h), min(sc.ny, y1 + h)
        crop = sc.flags[cy0:cy1, cx0:cx1]
        xa = sc.x_axis if (cx0 == 0) else PERIODIC
        ya = sc.y_axis if (cy0 == 0 and cy1 == sc.ny) else PERIODIC
        if cx0 != 0 and cx1 == sc.nx:
            xa = INFLOW_OUTFLOW
        ref = oracle.Oracle(crop, sc.tau, xa, ya, sc.u_in, sc.g, sc.u0).run(STEPS_BIG)
        _, ux, uy = ref.macros()
        # the window itself: at least h from every fake crop edge (real
        # domain edges keep their true boundary rules)
        ix0, ix1 = x0 - cx0, x1 - cx0
        iy0, iy1 = y0 - cy0, y1 - cy0
        gx = u[0, cy0 + iy0:cy0 + iy1, cx0 + ix0:cx0 + ix1].cpu().numpy().astype(np.float64)
        gy = u[1, cy0 + iy0:cy0 + iy1, cx0 + ix0:cx0 + ix1].cpu().numpy().astype(np.float64)
        rx, ry = ux[iy0:iy1, ix0:ix1], uy[iy0:iy1, ix0:ix1]
        upd = ((ref.types == oracle.FLUID) | (ref.types == oracle.OUTLET))[iy0:iy1, ix0:ix1]
        assert upd.sum() > 1000
        err = np.hypot(gx - rx, gy - ry)[upd].max() / np.hypot(rx, ry)[upd].max()
        worst = max(worst, float(err))
    del u
    torch.cuda.empty_cache()
    return worst


@pytest.fixture(scope="module")
def plate_big():
    return W.plate()  # 65536 x 32768 = 2^31 nodes


@pytest.mark.parametrize("scheme,layout", [("NPOL", "bundle"), ("NPOL", "stream"), ("NSOL", "bundle"),
                                           ("NSOL", "stream"), ("AA", "bundle"), ("AA", "stream")])
def test_plate_2pow31_one_lattice(plate_big, scheme, layout):
    from paper_2607_20650_amd.lbm import OK, Simulation
    sc = plate_big
    assert sc.nx * sc.ny == 2 ** 31
    with Simulation.from_scenario(sc, scheme=scheme, layout=layout, precision="fp32", bundle=50) as sim:
        info = sim.info()
        assert info["device_bytes"] >= 9 * 4 * 2 ** 31  # one full lattice, 64-bit offsets
        sim.step(STEPS_BIG)
        st, d = sim.diag()
        assert st == OK and np.isfinite(d[0])
        err = _crop_check(sim, sc, WINDOWS)
    _report(f"plate_2pow31/{scheme}/{layout}", {"crop_error": err})
    assert err <= 1e-5, err


def test_plate_two_lattice_comparison_grid():
    from paper_2607_20650_amd.lbm import OK, Simulation
    sc = W.plate(nx=46341, ny=23170)
    with Simulation.from_scenario(sc, scheme="NPTL", layout="stream", precision="fp32", bundle=50) as sim:
        sim.step(STEPS_BIG)
        st, d = sim.diag()
        assert st == OK and np.isfinite(d[0])
        cx, cy = int(sc.nx / 4), int(sc.ny / 2)
        err = _crop_check(sim, sc, [(cx - 1100, cx - 300, cy - 300, cy + 300), (0, 600, cy - 200, cy + 200)])
    _report("plate_46341x23170/NPTL/stream", {"crop_error": err})
    assert err <= 1e-5, err
