"""GPU parity of the D3Q19 extension against its FP64 oracle (oracle/d3q19).

All calls go through the C ABI (lbm3_* -> liblbm.so).  Tolerances as in the
2-D tests: shifted populations after random-state updates FP32 <= 2e-6,
16-bit storage <= 5e-4 absolute; velocity max |du| / u_max FP32 <= 1e-5; all
variants of one precision bitwise equal.
"""
import numpy as np
import pytest

from oracle import d3q19 as o3
from paper_2607_20650_amd import workloads as W
from tests.helpers import ALL_PRECISIONS, fp16_round

pytestmark = pytest.mark.gpu

W3 = o3.constants()[3]
SCHEMES3 = ["NPTL", "AA"]
LAYOUTS3 = ["stream", "collision", "blocked"]

CASES3 = {
    # name: nx, ny, nz, axes (x, y, z), p_solid, u_in, g, tile, seed
    "periodic-20x13x11": (20, 13, 11, (o3.PERIODIC, o3.PERIODIC, o3.PERIODIC), 0.15, (0, 0, 0),
                          (1e-5, -2e-6, 3e-6), (0, 0), 1),
    "closed-17x12x10-t16x4": (17, 12, 10, (o3.CLOSED, o3.CLOSED, o3.CLOSED), 0.1, (0, 0, 0), (0, 0, 0), (16, 4), 2),
    "mixed-70x9x7": (70, 9, 7, (o3.PERIODIC, o3.CLOSED, o3.PERIODIC), 0.1, (0, 0, 0), (2e-6, 0, 0), (64, 4), 3),
    "inout-37x14x9": (37, 14, 9, (o3.INFLOW_OUTFLOW, o3.CLOSED, o3.PERIODIC), 0.1, (0.05, 0.01, -0.01),
                      (0, 0, 0), (0, 0), 4),
    "inout-2x3x4": (2, 3, 4, (o3.INFLOW_OUTFLOW, o3.PERIODIC, o3.CLOSED), 0.0, (0.04, 0.0, 0.02), (0, 0, 0),
                    (16, 1), 5),
    # degenerate extents: one node along an axis (both borders at once; periodic wraps onto itself)
    "flat-16x9x1": (16, 9, 1, (o3.PERIODIC, o3.PERIODIC, o3.PERIODIC), 0.1, (0, 0, 0), (1e-5, 2e-6, 0), (0, 0), 6),
    "line-1x6x5": (1, 6, 5, (o3.PERIODIC, o3.CLOSED, o3.PERIODIC), 0.0, (0, 0, 0), (0, 3e-6, -1e-6), (0, 0), 7),
    "closed-1x4x3": (1, 4, 3, (o3.CLOSED, o3.CLOSED, o3.CLOSED), 0.0, (0, 0, 0), (0, 0, 0), (0, 0), 8),
    # 64-wide collision-layout patches 8 and 2 rows tall (staged kernels), ragged in x and y
    "periodic-130x11x5-t64x8": (130, 11, 5, (o3.PERIODIC, o3.PERIODIC, o3.PERIODIC), 0.1, (0, 0, 0),
                                (2e-6, -1e-6, 1e-6), (64, 8), 10),
    "inout-100x13x6-t64x2": (100, 13, 6, (o3.INFLOW_OUTFLOW, o3.CLOSED, o3.CLOSED), 0.1, (0.04, 0.0, 0.01),
                             (0, 0, 0), (64, 2), 11),
    # a full 256-wide block row with a ragged tail and periodic borders on every axis
    "periodic-300x7x6": (300, 7, 6, (o3.PERIODIC, o3.PERIODIC, o3.PERIODIC), 0.05, (0, 0, 0), (1e-6, 0, 1e-6),
                         (0, 0), 9),
}


def _variants(axes):
    return [(s, l) for s in SCHEMES3 for l in LAYOUTS3]


def _upd(types):
    return (types == o3.FLUID) | (types == o3.OUTLET)


@pytest.mark.parametrize("precision", ALL_PRECISIONS)
@pytest.mark.parametrize("case", list(CASES3))
def test_random_state_all_variants_3d(case, precision):
    from paper_2607_20650_amd.lbm import Simulation3
    nx, ny, nz, axes, p, u_in, g, tile, seed = CASES3[case]
    flags = W.random_flags3(nx, ny, nz, p, seed)
    tau = 0.6 + 0.04 * seed
    st = W.random_state3(nx, ny, nz, 0.02, seed=100 + seed, dtype=np.float32)
    if precision != "fp32":
        st = fp16_round(st)
    ref = o3.Oracle3(flags, tau, *axes, u_in=u_in, g=g)
    ref.set_state(st.astype(np.float64) + W3[:, None, None, None])
    steps = 12
    ref.run(steps)
    fin_ref = ref.incoming() - W3[:, None, None, None]
    mask = _upd(ref.types)
    tol = 2e-6 if precision == "fp32" else 5e-4
    first = None
    for scheme, layout in _variants(axes):
        # blocks above 256 threads exist for the staged collision-layout kernels only
        t = tile if layout == "collision" or tile[0] * tile[1] <= 256 else (0, 0)
        with Simulation3(flags, tau, *axes, u_in=u_in, g=g, scheme=scheme, layout=layout, precision=precision,
                         tile=t) as sim:
            sim.set_state(st)
            sim.step(steps)
            fin = sim.populations()
        err = np.abs(fin.astype(np.float64) - fin_ref)[:, mask].max() if mask.any() else 0.0
        assert err <= tol, f"{scheme}/{layout}/{precision}: max |df| = {err:.3e}"
        if first is None:
            first = fin
        else:
            assert np.array_equal(fin, first), f"{scheme}/{layout}/{precision} differs bitwise"


def _velocity_error(u, ref_u, mask):
    d = np.sqrt(((u.astype(np.float64) - ref_u) ** 2).sum(axis=0))[mask]
    return float(d.max() / np.sqrt((ref_u ** 2).sum(axis=0))[mask].max())


def test_duct_sphere_fp32():
    """Duct with a sphere, inlet and outlet, 300 updates: both schemes in
    every layout within 1e-5 of the oracle's velocity and bitwise equal."""
    from paper_2607_20650_amd.lbm import Simulation3
    sc = W.duct_sphere()
    ref = o3.Oracle3.from_scenario(sc).run(sc.steps)
    _, ref_u = ref.macros()
    mask = _upd(ref.types)
    first = None
    for scheme, layout in _variants((sc.x_axis, sc.y_axis, sc.z_axis)):
        with Simulation3.from_scenario(sc, scheme=scheme, layout=layout) as sim:
            sim.step(sc.steps)
            rho, u = sim.macros()
        assert _velocity_error(u, ref_u, mask) <= 1e-5, (scheme, layout)
        if first is None:
            first = u
        else:
            assert np.array_equal(u, first)


@pytest.mark.parametrize("precision", ["fp32", "fp16sr", "fp16csr"])
def test_sphere_array_all_variants(precision):
    """Periodic sphere array driven by a body force, 400 updates: every
    variant bitwise equal within a precision; FP32 within 1e-5 of the oracle,
    the stochastically rounded 16-bit formats within 2e-2."""
    from paper_2607_20650_amd.lbm import Simulation3
    sc = W.sphere_array(n=40, radius=7.0, tau=0.6, gx=2e-5, steps=400)
    ref = o3.Oracle3.from_scenario(sc).run(sc.steps)
    _, ref_u = ref.macros()
    mask = _upd(ref.types)
    first = None
    for scheme, layout in _variants((sc.x_axis, sc.y_axis, sc.z_axis)):
        with Simulation3.from_scenario(sc, scheme=scheme, layout=layout, precision=precision) as sim:
            sim.step(sc.steps)
            _, u = sim.macros()
        err = _velocity_error(u, ref_u, mask)
        assert err <= (1e-5 if precision == "fp32" else 2e-2), (scheme, layout, err)
        if first is None:
            first = u
        else:
            assert np.array_equal(u, first), (scheme, layout)


@pytest.mark.parametrize("layout", LAYOUTS3)
def test_aa_odd_counts_and_state_load_at_odd_parity_3d(layout):
    """AA with an inlet and outlet read out after an odd count (swap form), a
    state loaded at odd parity (outlet side buffer refilled), continued:
    bitwise equal to NPTL doing the same."""
    from paper_2607_20650_amd.lbm import Simulation3
    nx, ny, nz = 24, 11, 9
    flags = W.random_flags3(nx, ny, nz, 0.1, 7)
    st = W.random_state3(nx, ny, nz, 0.02, seed=8, dtype=np.float32)
    st2 = W.random_state3(nx, ny, nz, 0.02, seed=9, dtype=np.float32)
    out = {}
    for scheme in SCHEMES3:
        with Simulation3(flags, 0.7, o3.INFLOW_OUTFLOW, o3.CLOSED, o3.PERIODIC, u_in=(0.04, 0.01, 0),
                         g=(1e-5, 0, 0), scheme=scheme, layout=layout) as sim:
            sim.set_state(st)
            sim.step(7)
            a = sim.populations()
            sim.set_state(st2)
            sim.step(5)
            out[scheme] = (a, sim.populations())
    assert np.array_equal(out["AA"][0], out["NPTL"][0])
    assert np.array_equal(out["AA"][1], out["NPTL"][1])


def test_sphere_array_256_collision_pull_at_bench_launch():
    """The 256^3 sphere array with the default launch of the bench (the
    z-marching FP32 collision-layout pull, 16 planes per block on 64 x 8
    patches; the three-plane binary16 pull on 64 x 8 patches), 8 updates from
    rest under a body force: FP32 populations bitwise equal to the
    stream-layout pull's, binary16 to the blocked layout's; FP32 velocities on
    two 48^3 windows over the sphere's surface, each spanning several of the
    kernel's 16-plane ranges, within 1e-5 of oracle runs on crops with a
    10-node halo (periodic wraps on small grids are covered above)."""
    from paper_2607_20650_amd.lbm import Simulation3
    steps, h, m = 8, 10, 48
    sc = W.sphere_array(n=256, gx=1e-4)
    n = sc.flags.shape[0]

    def run(layout, precision):
        with Simulation3.from_scenario(sc, scheme="NPTL", layout=layout, precision=precision) as sim:
            sim.step(steps)
            _, u = sim.macros()
            return sim.populations(), u

    f_col, u = run("collision", "fp32")
    f_str, _ = run("stream", "fp32")
    assert np.array_equal(f_col, f_str)
    del f_str
    for x0, y0, z0 in [(64, 104, 104), (150, 60, 140)]:
        ix = np.arange(x0 - h, x0 + m + h) % n
        iy = np.arange(y0 - h, y0 + m + h) % n
        iz = np.arange(z0 - h, z0 + m + h) % n
        ref = o3.Oracle3(sc.flags[np.ix_(iz, iy, ix)], sc.tau, o3.PERIODIC, o3.PERIODIC, o3.PERIODIC,
                         g=sc.g).run(steps)
        _, ru = ref.macros()
        ru = ru[:, h:h + m, h:h + m, h:h + m]
        g = u[:, iz[h:h + m]][:, :, iy[h:h + m]][:, :, :, ix[h:h + m]].astype(np.float64)
        upd = _upd(ref.types)[h:h + m, h:h + m, h:h + m]
        assert upd.sum() > 1000
        err = np.sqrt(((g - ru) ** 2).sum(0))[upd].max() / np.sqrt((ru ** 2).sum(0))[upd].max()
        assert err <= 1e-5, ((x0, y0, z0), err)
    del f_col, u
    f_col, _ = run("collision", "fp16s")
    f_blk, _ = run("blocked", "fp16s")
    assert np.array_equal(f_col, f_blk)


def test_sphere_array_1024_cubed_crops():
    """A 1024^3 sphere array (2^30 nodes, 81.6 GB in place, 64-bit offsets) in
    FP32 AA, 20 updates, checked on three 48^3 windows (sphere surface, a
    periodic corner, the far corner) against oracle runs on crops with a halo
    of 22 nodes: after 20 updates a node depends only on nodes within 20."""
    import torch
    from paper_2607_20650_amd.lbm import Simulation3
    steps, h, m = 20, 22, 48
    sc = W.sphere_array(n=1024, radius=160.0)
    n = sc.flags.shape[0]
    windows = [(330, 490, 490), (-24, -24, 500), (1000, 1000, 1000)]  # (x0, y0, z0), may wrap
    with Simulation3.from_scenario(sc, scheme="AA", layout="stream") as sim:
        sim.step(steps)
        _, u = sim.macros(device=True)
        sim.sync()
        got = []
        for x0, y0, z0 in windows:
            ix = torch.arange(x0, x0 + m, device="cuda") % n
            iy = torch.arange(y0, y0 + m, device="cuda") % n
            iz = torch.arange(z0, z0 + m, device="cuda") % n
            got.append(u[:, iz][:, :, iy][:, :, :, ix].cpu().numpy().astype(np.float64))
        del u
    for (x0, y0, z0), g in zip(windows, got):
        ix = np.arange(x0 - h, x0 + m + h) % n
        iy = np.arange(y0 - h, y0 + m + h) % n
        iz = np.arange(z0 - h, z0 + m + h) % n
        crop = sc.flags[np.ix_(iz, iy, ix)]
        ref = o3.Oracle3(crop, sc.tau, o3.PERIODIC, o3.PERIODIC, o3.PERIODIC, g=sc.g).run(steps)
        _, ru = ref.macros()
        ru = ru[:, h:h + m, h:h + m, h:h + m]
        upd = _upd(ref.types)[h:h + m, h:h + m, h:h + m]
        assert upd.sum() > 1000
        err = np.sqrt(((g - ru) ** 2).sum(0))[upd].max() / np.sqrt((ru ** 2).sum(0))[upd].max()
        assert err <= 1e-5, ((x0, y0, z0), err)


def test_diag_3d_matches_populations_and_conservation():
    """FP64 diagnostics of the D3Q19 extension: mass equals the sum over the
    incoming populations, is conserved by every variant in a periodic box
    (FP32 storage rounding only), the residual is -1 first and positive after
    updates; all variants report the same values."""
    from paper_2607_20650_amd.lbm import OK, Simulation3
    nx, ny, nz = 24, 14, 10
    flags = W.random_flags3(nx, ny, nz, 0.15, 40)
    st = W.random_state3(nx, ny, nz, 0.01, seed=41, dtype=np.float32)
    mask = _upd(o3.Oracle3(flags, 0.8).types)
    seen = None
    for scheme, layout in _variants((o3.PERIODIC,) * 3):
        with Simulation3(flags, 0.8, scheme=scheme, layout=layout) as sim:
            sim.set_state(st)
            s0, d0 = sim.diag()
            assert s0 == OK and d0[4] == -1.0
            f = sim.populations().astype(np.float64)
            assert abs(d0[0] - (1.0 + f.sum(axis=0))[mask].sum()) < 1e-9
            sim.step(30)
            s1, d1 = sim.diag()
            assert s1 == OK and d1[4] > 0
            assert abs(d1[0] - d0[0]) / d0[0] < 1e-6
        if seen is None:
            seen = (d0, d1)
        else:
            assert seen == (d0, d1), (scheme, layout)
