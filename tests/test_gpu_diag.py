"""FP64 diagnostics (lbm_diag, lbm3_diag) against the FP64 oracles.

The diagnostics are the moments of Eq. 2 summed over every fluid and outlet
node: mass M = sum rho = sum_i f_in_i, momentum J = sum_i f_in_i c_i (no g/2
shift), and the residual ||u_t - u_prev|| / ||u_t|| between two calls, with
u = J-per-node + g/2.  Checks, all through the C ABI:

  * mass and momentum equal the FP64 sums over the oracle's incoming
    populations on the same state after the same updates, in every variant;
    bound: each update stores 9 (19) FP32 values per node with at most four
    roundings of 2^-24 |f~|max each, and the exact update conserves mass and
    does not amplify sums, so |dM|, |dJ| <= n * Q * N * 4 * 2^-24 * |f~|max
    after n updates (worst case: every rounding of one sign);
  * the reduction itself: the diagnostics of a state equal the FP64 sums of
    the populations the library reports for it (1e-12 relative);
  * a forced periodic box without solids gains momentum exactly N g per
    update (closed form of the force term 3 w_i (c_i . g));
  * the residual equals the one computed on the host from two velocity
    readouts (FP32 readouts: |dr| <= 1e-6) and the oracle's residual between
    the same update counts (bound from the FP32 velocity tolerance);
  * two calls without an update in between give residual exactly 0; the
    first call and the first call after a state load report -1;
  * a state holding a NaN makes the diagnostics report LBM_EUNSTABLE in every
    precision, in 2-D and 3-D.
"""
import numpy as np
import pytest

import oracle
from oracle import CLOSED, INFLOW_OUTFLOW, PERIODIC
from oracle import d3q19 as o3
from paper_2607_20650_amd import workloads as W
from tests.helpers import ALL_LAYOUTS, ALL_PRECISIONS, ALL_SCHEMES, updated_mask, weights

pytestmark = pytest.mark.gpu

CX, CY = oracle.constants()[:2]
C3 = o3.constants()


def _moments_2d(fin, mask):
    """(mass, jx, jy) in FP64 over mask of unshifted incoming populations."""
    f = fin[:, mask]
    return float(f.sum()), float((CX[:, None] * f).sum()), float((CY[:, None] * f).sum())


def _moments_3d(fin, mask):
    f = fin[:, mask]
    return (float(f.sum()),) + tuple(float((C3[a][:, None] * f).sum()) for a in range(3))


def _round_bound(steps, q, n_nodes, fmax):
    return steps * q * n_nodes * 4 * 2.0 ** -24 * fmax


DIAG_CASES = {
    # name: nx, ny, x_axis, y_axis, p_solid, u_in, g, seed
    "periodic-solids-72x40": (72, 40, PERIODIC, PERIODIC, 0.15, (0.0, 0.0), (2e-6, -1e-6), 51),
    "inout-closed-90x33": (90, 33, INFLOW_OUTFLOW, CLOSED, 0.08, (0.05, 0.0), (0.0, 0.0), 52),
}


@pytest.mark.parametrize("case", list(DIAG_CASES))
def test_diag_mass_momentum_match_oracle_all_variants(case):
    from paper_2607_20650_amd.lbm import OK, Simulation
    nx, ny, xa, ya, p, u_in, g, seed = DIAG_CASES[case]
    flags = W.random_flags(nx, ny, p, seed)
    tau = 0.7
    st = W.random_state(nx, ny, 0.02, seed=seed + 100, dtype=np.float32)
    steps = 40
    ref = oracle.Oracle(flags, tau, xa, ya, u_in, g)
    ref.set_state(st.astype(np.float64) + weights()[:, None, None])
    mask = updated_mask(ref.types)
    m0 = _moments_2d(ref.incoming(), mask)
    ref.run(steps)
    m1 = _moments_2d(ref.incoming(), mask)
    nupd = int(mask.sum())
    tol = _round_bound(steps, 9, nupd, float(np.abs(st).max()))
    seen = None
    for scheme in ALL_SCHEMES:
        for layout in ALL_LAYOUTS:
            with Simulation(flags, tau, xa, ya, u_in, g, scheme=scheme, layout=layout) as sim:
                sim.set_state(st)
                s0, d0 = sim.diag()
                assert s0 == OK and d0[3] == -1.0
                # the reduction: FP64 sums of the populations the library reports
                fg = sim.populations().astype(np.float64) + weights()[:, None, None]
                own = _moments_2d(fg, mask)
                assert np.allclose(d0[:3], own, rtol=1e-12, atol=1e-12 * nupd), (scheme, layout, d0, own)
                # the loaded state is exact in FP32: the oracle's moments up to FP64 order
                assert np.allclose(d0[:3], m0, rtol=0, atol=1e-10 * nupd), (scheme, layout, d0, m0)
                sim.step(steps)
                s1, d1 = sim.diag()
                assert s1 == OK
                err = np.abs(np.array(d1[:3]) - np.array(m1))
                assert (err <= tol).all(), (scheme, layout, err, tol)
                assert d1[3] > 0
            if seen is None:
                seen = (d0, d1)
            else:  # every variant of one precision is bitwise equal, so are its diagnostics
                assert seen == (d0, d1), (scheme, layout)


@pytest.mark.parametrize("precision", ALL_PRECISIONS)
def test_diag_reduction_exact_all_precisions(precision):
    """The FP64 sums equal those of the reported populations in every
    storage precision (the stored values widen exactly)."""
    from paper_2607_20650_amd.lbm import OK, Simulation
    nx, ny = 64, 48
    flags = W.random_flags(nx, ny, 0.1, 61)
    st = W.random_state(nx, ny, 0.02, seed=62, dtype=np.float32)
    mask = updated_mask(oracle.Oracle(flags, 0.8, INFLOW_OUTFLOW, CLOSED).types)
    for scheme in ("NPTL", "AA", "NSOL"):
        with Simulation(flags, 0.8, INFLOW_OUTFLOW, CLOSED, (0.04, 0.0), scheme=scheme, precision=precision) as sim:
            sim.set_state(st)
            sim.step(25)
            s, d = sim.diag()
            assert s == OK
            fg = sim.populations().astype(np.float64) + weights()[:, None, None]
            own = _moments_2d(fg, mask)
            assert np.allclose(d[:3], own, rtol=1e-12, atol=1e-12 * mask.sum()), (scheme, precision, d, own)


@pytest.mark.parametrize("scheme", ALL_SCHEMES)
def test_diag_momentum_grows_by_n_g_per_update(scheme):
    """Periodic box, no solids, body force g, start at rest: the force term
    adds sum_i 3 w_i (c_i . g) c_i = g per node and update, collision keeps
    j, so J(t) = N g t.  Every node holds the same values, so FP32 roundings
    do not average out over nodes: at most a few 2^-24 relative per stored
    value and update, below 1e-4 relative after 200 updates; mass stays N up
    to the rounding bound of the module docstring (|f~| <= 3e-5 (t + 1))."""
    from paper_2607_20650_amd.lbm import OK, Simulation
    nx, ny = 96, 64
    g = (3e-6, -2e-6)
    flags = np.zeros((ny, nx), np.uint8)
    N = nx * ny
    with Simulation(flags, 0.75, PERIODIC, PERIODIC, g=g, scheme=scheme) as sim:
        for t in (0, 50, 200):
            sim.step(t - sim.info()["steps"])
            s, d = sim.diag()
            assert s == OK
            assert abs(d[0] - N) <= _round_bound(max(t, 1), 9, N, 3e-5 * (t + 1)), (scheme, t, d)
            for a in (0, 1):
                want = N * g[a] * t
                assert abs(d[1 + a] - want) <= 1e-4 * abs(N * g[a] * max(t, 1)), (scheme, t, a, d, want)


def test_diag_residual_against_host_and_oracle():
    """A developing Karman flow: the residual between two calls equals the one
    computed from two velocity readouts, and the oracle's."""
    from paper_2607_20650_amd.lbm import OK, Simulation
    sc = W.karman(nx=240, ny=80, cx=60, cy=40, radius=8, u_in=0.05, tau=0.6)
    t1, t2 = 100, 130
    ref = oracle.Oracle.from_scenario(sc).run(t1)
    _, rx1, ry1 = ref.macros()
    ref.run(t2 - t1)
    _, rx2, ry2 = ref.macros()
    mask = updated_mask(ref.types)
    dref = np.sqrt(((rx2 - rx1)[mask] ** 2 + (ry2 - ry1)[mask] ** 2).sum())
    nref = np.sqrt((rx2[mask] ** 2 + ry2[mask] ** 2).sum())
    r_ora = dref / nref
    umax = float(np.hypot(rx2, ry2)[mask].max())
    # FP32 velocities within 1e-5 u_max of the oracle at every node:
    # |dr| <= (||du_1|| + ||du_2|| + r ||du_2||) / ||u_2|| <= (2 + r) 1e-5 u_max sqrt(N) / ||u_2||
    tol_ora = (2 + r_ora) * 1e-5 * umax * np.sqrt(mask.sum()) / nref
    for scheme, layout in (("NPTL", "stream"), ("AA", "bundle"), ("NPOL", "collision"), ("PUSH", "stream")):
        with Simulation.from_scenario(sc, scheme=scheme, layout=layout) as sim:
            s, d = sim.diag()
            assert s == OK and d[3] == -1.0
            sim.step(t1)
            _, u1 = sim.macros()
            s, d = sim.diag()
            assert s == OK and d[3] > 0  # against the start
            sim.step(t2 - t1)
            _, u2 = sim.macros()
            s, d = sim.diag()
            assert s == OK
            a1, a2 = u1.astype(np.float64), u2.astype(np.float64)
            r_host = np.sqrt(((a2 - a1)[:, mask] ** 2).sum()) / np.sqrt((a2[:, mask] ** 2).sum())
            assert abs(d[3] - r_host) <= 1e-6, (scheme, layout, d[3], r_host)
            assert abs(d[3] - r_ora) <= tol_ora, (scheme, layout, d[3], r_ora, tol_ora)
            assert r_ora > 1e-3  # the flow is developing: a meaningful residual


@pytest.mark.parametrize("precision", ALL_PRECISIONS)
def test_diag_residual_zero_without_change(precision):
    """Two calls on an unchanged state give residual exactly 0 (the previous
    velocities are kept in FP64, as computed); the first call, and the first
    call after a state load, give -1."""
    from paper_2607_20650_amd.lbm import OK, Simulation
    nx, ny = 64, 40
    flags = W.random_flags(nx, ny, 0.1, 65)
    st = W.random_state(nx, ny, 0.02, seed=66, dtype=np.float32)
    for scheme in ("NPTL", "AA", "NSOL"):
        with Simulation(flags, 0.9, INFLOW_OUTFLOW, CLOSED, (0.04, 0.0), scheme=scheme, precision=precision) as sim:
            sim.set_state(st)
            sim.step(11)  # an odd count: AA holds its swap form
            s, d = sim.diag()
            assert s == OK and d[3] == -1.0
            s, d = sim.diag()
            assert s == OK and d[3] == 0.0, (scheme, precision, d)
            sim.step(5)
            s, d = sim.diag()
            assert s == OK and d[3] > 1e-4, (scheme, precision, d)
            sim.set_state(st)
            s, d = sim.diag()
            assert s == OK and d[3] == -1.0


@pytest.mark.parametrize("precision", ALL_PRECISIONS)
def test_diag_reports_unstable_on_nan(precision):
    from paper_2607_20650_amd.lbm import EUNSTABLE, OK, Simulation
    nx, ny = 48, 32
    flags = W.random_flags(nx, ny, 0.1, 71)
    st = W.random_state(nx, ny, 0.01, seed=72, dtype=np.float32)
    types = oracle.Oracle(flags, 0.8).types
    ys, xs = np.nonzero(types == oracle.FLUID)
    for scheme in ("NPTL", "AA", "NPOL"):
        with Simulation(flags, 0.8, scheme=scheme, precision=precision) as sim:
            sim.set_state(st)
            s, d = sim.diag()
            assert s == OK and np.isfinite(d[:3]).all()
            bad = st.copy()
            bad[5, ys[7], xs[7]] = np.nan
            sim.set_state(bad)
            s, d = sim.diag()
            assert s == EUNSTABLE, (scheme, precision, s, d)
            assert not np.isfinite(d[0])
            sim.step(3)  # the NaN spreads; the status stays
            s, d = sim.diag()
            assert s == EUNSTABLE


# ------------------------------------------------------------------ D3Q19
def test_diag3_mass_momentum_match_oracle_all_variants():
    from paper_2607_20650_amd.lbm import OK, Simulation3
    nx, ny, nz = 30, 14, 10
    axes = (o3.INFLOW_OUTFLOW, o3.CLOSED, o3.PERIODIC)
    flags = W.random_flags3(nx, ny, nz, 0.1, 81)
    st = W.random_state3(nx, ny, nz, 0.02, seed=82, dtype=np.float32)
    tau, u_in, g = 0.7, (0.04, 0.01, 0.0), (0.0, 0.0, 1e-6)
    steps = 30
    ref = o3.Oracle3(flags, tau, *axes, u_in=u_in, g=g)
    ref.set_state(st.astype(np.float64) + C3[3][:, None, None, None])
    mask = (ref.types == o3.FLUID) | (ref.types == o3.OUTLET)
    m0 = _moments_3d(ref.incoming(), mask)
    ref.run(steps)
    m1 = _moments_3d(ref.incoming(), mask)
    nupd = int(mask.sum())
    tol = _round_bound(steps, 19, nupd, float(np.abs(st).max()))
    seen = None
    for scheme in ("NPTL", "AA"):
        for layout in ("stream", "collision", "blocked"):
            with Simulation3(flags, tau, *axes, u_in=u_in, g=g, scheme=scheme, layout=layout) as sim:
                sim.set_state(st)
                s0, d0 = sim.diag()
                assert s0 == OK and d0[4] == -1.0
                fg = sim.populations().astype(np.float64) + C3[3][:, None, None, None]
                own = _moments_3d(fg, mask)
                assert np.allclose(d0[:4], own, rtol=1e-12, atol=1e-12 * nupd), (scheme, layout, d0, own)
                assert np.allclose(d0[:4], m0, rtol=0, atol=1e-10 * nupd), (scheme, layout, d0, m0)
                sim.step(steps)
                s1, d1 = sim.diag()
                assert s1 == OK and d1[4] > 0
                err = np.abs(np.array(d1[:4]) - np.array(m1))
                assert (err <= tol).all(), (scheme, layout, err, tol)
            if seen is None:
                seen = (d0, d1)
            else:
                assert seen == (d0, d1), (scheme, layout)


def test_diag3_momentum_growth_and_residual():
    """Periodic 3-D box without solids under a body force: J(t) = N g t; the
    residual between two calls equals the host value from two readouts."""
    from paper_2607_20650_amd.lbm import OK, Simulation3
    nx, ny, nz = 40, 24, 16
    g = (2e-6, 1e-6, -3e-6)
    flags = np.zeros((nz, ny, nx), np.uint8)
    N = nx * ny * nz
    with Simulation3(flags, 0.8, g=g, scheme="AA", layout="blocked") as sim:
        s, d = sim.diag()
        assert s == OK and d[4] == -1.0
        sim.step(60)
        _, u1 = sim.macros()
        s, d = sim.diag()
        assert s == OK
        for a in range(3):
            assert abs(d[1 + a] - N * g[a] * 60) <= 1e-5 * abs(N * g[a] * 60), (a, d)
        sim.step(40)
        _, u2 = sim.macros()
        s, d = sim.diag()
        assert s == OK
        for a in range(3):
            assert abs(d[1 + a] - N * g[a] * 100) <= 1e-5 * abs(N * g[a] * 100), (a, d)
        a1, a2 = u1.astype(np.float64), u2.astype(np.float64)
        r_host = np.sqrt(((a2 - a1) ** 2).sum()) / np.sqrt((a2 ** 2).sum())
        # uniform acceleration: u(t) = g (t + 1/2), so r = 40 / 100.5
        assert abs(r_host - 40 / 100.5) <= 1e-4
        assert abs(d[4] - r_host) <= 1e-6, (d[4], r_host)


@pytest.mark.parametrize("precision", ALL_PRECISIONS)
def test_diag3_reports_unstable_on_nan(precision):
    from paper_2607_20650_amd.lbm import EUNSTABLE, OK, Simulation3
    nx, ny, nz = 20, 12, 8
    flags = W.random_flags3(nx, ny, nz, 0.1, 91)
    st = W.random_state3(nx, ny, nz, 0.01, seed=92, dtype=np.float32)
    types = o3.Oracle3(flags, 0.8).types
    zs, ys, xs = np.nonzero(types == o3.FLUID)
    for scheme in ("NPTL", "AA"):
        with Simulation3(flags, 0.8, scheme=scheme, layout="blocked", precision=precision) as sim:
            sim.set_state(st)
            s, d = sim.diag()
            assert s == OK
            bad = st.copy()
            bad[3, zs[11], ys[11], xs[11]] = np.nan
            sim.set_state(bad)
            s, d = sim.diag()
            assert s == EUNSTABLE, (scheme, precision, s, d)
            sim.step(2)
            s, d = sim.diag()
            assert s == EUNSTABLE
