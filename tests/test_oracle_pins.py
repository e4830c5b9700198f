"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these tests compares the oracle with itself: each checks a printed
constant, a closed form, an invariant, a special case, or an independent
brute-force formulation (tests/brute_ref.py: push + ghost-column outlet).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import CLOSED, INFLOW_OUTFLOW, PERIODIC, Oracle
from paper_2607_20650_amd import workloads as W
from tests import brute_ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "d2q9_paper.json")


# ------------------------------------------------------------------ constants
def test_velocity_set_and_weights_match_paper():
    """Fig. 2 (b) direction order and the Eq. 2 weights."""
    gold = json.load(open(GOLDEN))
    cx, cy, opp, w = oracle.constants()
    for i, name in enumerate(gold["arrows_in_order"]):
        vx, vy = gold["arrow_vectors"][name]
        assert (cx[i], cy[i]) == (vx, vy), name
    for i, frac in gold["weights"].items():
        num, den = map(int, frac.split("/"))
        assert w[int(i)] == num / den
    for i in range(9):
        assert (cx[opp[i]], cy[opp[i]]) == (-cx[i], -cy[i])
    # bundles of Fig. 2 (c) group the directions by c_y
    for b, names in enumerate(gold["bundles_fig2c"]):
        idx = [gold["arrows_in_order"].index(n) for n in names]
        assert all(cy[i] == b - 1 for i in idx)


def test_equilibrium_moments_closed_form():
    """Moments of the D2Q9I equilibrium (Eq. 2): sum = rho, first moment = v,
    second moment = rho/3 I + v v (incompressible model: no 1/rho)."""
    cx, cy, _, _ = oracle.constants()
    rng = np.random.default_rng(1)
    for _ in range(20):
        rho = 1 + 0.1 * rng.standard_normal()
        vx, vy = 0.1 * rng.standard_normal(2)
        f = oracle.equilibrium(rho, vx, vy)
        assert abs(f.sum() - rho) < 1e-15
        assert abs((f * cx).sum() - vx) < 1e-15
        assert abs((f * cy).sum() - vy) < 1e-15
        assert abs((f * cx * cx).sum() - (rho / 3 + vx * vx)) < 1e-15
        assert abs((f * cy * cy).sum() - (rho / 3 + vy * vy)) < 1e-15
        assert abs((f * cx * cy).sum() - vx * vy) < 1e-15


# ---------------------------------------------------------------- invariants
def test_equilibrium_fixed_point():
    """Uniform feq(1, u0) in a periodic box without force is a fixed point."""
    flags = np.zeros((12, 16), np.uint8)
    o = Oracle(flags, tau=0.7, x_axis=PERIODIC, y_axis=PERIODIC, u0=(0.03, -0.02))
    f0 = o.state.copy()
    o.run(1000)
    assert np.abs(o.state - f0).max() <= 1e-14


def test_uniform_flow_inlet_outlet_fixed_point():
    """Uniform flow u_in through an inlet / zero-gradient outlet channel with a
    periodic y axis stays exactly uniform (both boundary rules are consistent
    with the free stream)."""
    flags = np.zeros((10, 24), np.uint8)
    o = Oracle(flags, tau=0.65, x_axis=INFLOW_OUTFLOW, y_axis=PERIODIC, u_in=(0.05, 0.01), u0=(0.05, 0.01))
    o.run(300)
    rho, ux, uy = o.macros()
    # rounding of 300 FP64 updates only (a wrong rule moves these by >= 1e-6)
    assert np.abs(rho - 1).max() < 1e-12
    assert np.abs(ux - 0.05).max() < 1e-12 and np.abs(uy - 0.01).max() < 1e-12


def _sums(o):
    fin = o.incoming()
    cx, cy, _, _ = oracle.constants()
    upd = (o.types == oracle.FLUID) | (o.types == oracle.OUTLET)
    m = fin.sum(axis=0)[upd].sum()
    jx = np.tensordot(cx, fin, axes=(0, 0))[upd].sum()
    jy = np.tensordot(cy, fin, axes=(0, 0))[upd].sum()
    return m, jx, jy


def test_conservation_periodic_no_force():
    flags = np.zeros((16, 20), np.uint8)
    o = Oracle(flags, tau=0.8, x_axis=PERIODIC, y_axis=PERIODIC)
    st = W.random_state(20, 16, 0.01, seed=3) + oracle.equilibrium(1, 0, 0)[:, None, None]
    o.set_state(st)
    m0, jx0, jy0 = _sums(o)
    o.run(200)
    m1, jx1, jy1 = _sums(o)
    assert abs(m1 - m0) / abs(m0) < 1e-12
    assert abs(jx1 - jx0) < 1e-12 * abs(m0) and abs(jy1 - jy0) < 1e-12 * abs(m0)


def test_momentum_growth_with_force():
    """Periodic box without solids: total momentum grows by N g per step."""
    flags = np.zeros((10, 14), np.uint8)
    g = (2e-5, -1e-5)
    o = Oracle(flags, tau=0.9, x_axis=PERIODIC, y_axis=PERIODIC, g=g)
    st = W.random_state(14, 10, 0.01, seed=4) + oracle.equilibrium(1, 0, 0)[:, None, None]
    o.set_state(st)
    m0, jx0, jy0 = _sums(o)
    n = 140
    o.run(150)
    m1, jx1, jy1 = _sums(o)
    assert abs(m1 - m0) < 1e-12 * m0
    assert abs(jx1 - (jx0 + n * g[0] * 150)) < 1e-12 * m0
    assert abs(jy1 - (jy0 + n * g[1] * 150)) < 1e-12 * m0


def test_mass_conserved_with_random_solids():
    """Halfway bounce-back neither creates nor destroys mass."""
    flags = W.random_flags(24, 18, 0.25, seed=7)
    o = Oracle(flags, tau=0.75, x_axis=PERIODIC, y_axis=CLOSED, g=(1e-5, 0))
    st = W.random_state(24, 18, 0.01, seed=8) + oracle.equilibrium(1, 0, 0)[:, None, None]
    o.set_state(st)
    m0, _, _ = _sums(o)
    o.run(300)
    m1, _, _ = _sums(o)
    assert abs(m1 - m0) / m0 < 1e-12


def test_uniform_forcing_velocity():
    """Periodic, no solids, start at rest: reported u(t) = g (t + 1/2) everywhere."""
    flags = np.zeros((6, 8), np.uint8)
    g = (1e-6, 3e-7)
    o = Oracle(flags, tau=0.8, x_axis=PERIODIC, y_axis=PERIODIC, g=g)
    for t in (0, 1, 50, 400):
        o.run(t - o.t)
        _, ux, uy = o.macros()
        # absolute slack = accumulated rounding of sums of O(1) populations
        # (~1e-16 per step); a missing half step would be off by >= 1.5e-7
        assert np.abs(ux - g[0] * (t + 0.5)).max() < 1e-13
        assert np.abs(uy - g[1] * (t + 0.5)).max() < 1e-13


def test_translation_invariance_bitwise():
    nx, ny = 16, 12
    flags = W.random_flags(nx, ny, 0.2, seed=11)
    st = W.random_state(nx, ny, 0.02, seed=12) + oracle.equilibrium(1, 0, 0)[:, None, None]
    a = Oracle(flags, tau=0.7, g=(1e-5, 2e-6))
    a.set_state(st)
    a.run(30)
    dx, dy = 5, 3
    b = Oracle(np.roll(flags, (dy, dx), axis=(0, 1)), tau=0.7, g=(1e-5, 2e-6))
    b.set_state(np.roll(st, (dy, dx), axis=(1, 2)))
    b.run(30)
    assert np.array_equal(np.roll(a.state, (dy, dx), axis=(1, 2)), b.state)


def test_mirror_symmetry():
    """A channel symmetric about its mid-line keeps u_x even and u_y odd."""
    nx, ny = 41, 21
    flags = W.walls(nx, ny)
    W.add_disc(flags, 12, 10, 3)
    assert np.array_equal(flags, flags[::-1])
    o = Oracle(flags, tau=0.6, x_axis=INFLOW_OUTFLOW, y_axis=CLOSED, u_in=(0.05, 0), u0=(0.05, 0))
    o.run(300)
    _, ux, uy = o.macros()
    assert np.abs(ux - ux[::-1]).max() < 1e-12
    assert np.abs(uy + uy[::-1]).max() < 1e-12
    assert np.abs(ux).max() > 0.04


# -------------------------------------------------------------- closed forms
def poiseuille_closed_form(H, tau, g):
    """Steady halfway-bounce-back Poiseuille profile for the reported velocity
    (pre-collision moment + g/2), BGK with simple forcing; exact on the lattice:
    u(s) = g/(2 nu) [ (H/2)^2 + (16 L - 3)/12 - s^2 ], nu = (tau-1/2)/3,
    L = (tau-1/2)^2, s measured from the channel centre at node positions."""
    nu = (tau - 0.5) / 3
    lam = (tau - 0.5) ** 2
    s = np.arange(H) - (H - 1) / 2
    return g / (2 * nu) * ((H / 2) ** 2 + (16 * lam - 3) / 12 - s * s)


@pytest.mark.parametrize("tau", [0.8, 0.6])
def test_poiseuille_steady_closed_form(tau):
    ny, H, g = 64, 62, 1e-6
    o = Oracle(W.walls(2, ny), tau=tau, x_axis=PERIODIC, y_axis=CLOSED, g=(g, 0))
    nu = (tau - 0.5) / 3
    steps = int(40 * (H / math.pi) ** 2 / nu)
    o.run(steps)
    _, ux, uy = o.macros()
    exact = poiseuille_closed_form(H, tau, g)
    num = ux[1:ny - 1, 0]
    assert np.abs(num - exact).max() / exact.max() < 1e-9
    assert np.abs(uy).max() < 1e-15
    if tau == 0.8:
        assert abs(exact.max() - 4.8031e-3) < 1e-7
    # permeability of the slit over all cells: k = nu <u_x> / g
    k_num = nu * ux[:, 0].mean() / g
    k_exact = nu * exact.sum() / ny / g
    assert abs(k_num - k_exact) / k_exact < 1e-9


def test_poiseuille_startup_series():
    """Start-up from rest against the continuum Fourier series with the
    effective half-width a^2 = (H/2)^2 + (16L-3)/12, at t = 2000 (cfg 128x64)."""
    nx, ny, H, tau, g = 128, 64, 62, 0.8, 1e-6
    o = Oracle(W.walls(nx, ny), tau=tau, x_axis=PERIODIC, y_axis=CLOSED, g=(g, 0))
    o.run(2000)
    _, ux, _ = o.macros()
    nu = (tau - 0.5) / 3
    a2 = (H / 2) ** 2 + (16 * (tau - 0.5) ** 2 - 3) / 12
    a = math.sqrt(a2)
    s = np.arange(H) - (H - 1) / 2
    t = 2000 + 0.5
    u = g / (2 * nu) * (a2 - s * s)
    for n in range(200):
        k = 2 * n + 1
        u -= (16 * g * a2 / (nu * math.pi ** 3)) * (-1) ** n / k ** 3 * np.cos(k * math.pi * s / (2 * a)) * \
            math.exp(-k * k * math.pi ** 2 * nu * t / (4 * a2))
    num = ux[1:ny - 1, :]
    assert np.abs(num - num[:, :1]).max() < 1e-17 + 1e-12 * num.max()  # x-invariant
    rel = np.abs(num[:, 0] - u).max() / u.max()
    assert rel < 1e-3, rel
    assert abs(num.max() - 1.8387e-3) < 2e-6


def test_shear_wave_decay_rate():
    """Periodic shear wave u_x = A sin(k y) decays as exp(-nu k^2 t)."""
    n, tau, A = 64, 0.8, 1e-4
    nu = (tau - 0.5) / 3
    k = 2 * math.pi / n
    flags = np.zeros((n, 4), np.uint8)
    o = Oracle(flags, tau=tau, x_axis=PERIODIC, y_axis=PERIODIC)
    y = np.arange(n)
    st = np.zeros((9, n, 4))
    for j in range(n):
        st[:, j, :] = oracle.equilibrium(1.0, A * math.sin(k * j), 0.0)[:, None]
    o.set_state(st)
    amps = []
    for t in (200, 2200):
        o.run(t - o.t)
        _, ux, _ = o.macros()
        amps.append(2 / n * (ux[:, 0] * np.sin(k * y)).sum())
    rate = math.log(amps[0] / amps[1]) / 2000
    assert abs(rate / (nu * k * k) - 1) < 0.01


# ------------------------------------------------------------------ brute force
BRUTE_CASES = [
    # nx, ny, x_axis, y_axis, p_solid, u_in, g, seed
    (8, 8, PERIODIC, PERIODIC, 0.2, (0, 0), (1e-4, -2e-5), 1),
    (7, 5, CLOSED, CLOSED, 0.2, (0, 0), (0, 0), 2),
    (7, 5, PERIODIC, CLOSED, 0.15, (0, 0), (3e-5, 0), 3),
    (16, 9, INFLOW_OUTFLOW, CLOSED, 0.15, (0.05, 0.01), (0, 0), 4),
    (16, 9, INFLOW_OUTFLOW, PERIODIC, 0.2, (0.04, -0.02), (1e-5, 0), 5),
    (9, 16, CLOSED, PERIODIC, 0.25, (0, 0), (0, 2e-5), 6),
    (3, 4, INFLOW_OUTFLOW, CLOSED, 0.0, (0.05, 0), (0, 0), 7),
    (2, 3, INFLOW_OUTFLOW, PERIODIC, 0.0, (0.05, 0.02), (0, 0), 8),
]


@pytest.mark.parametrize("case", BRUTE_CASES, ids=[f"{c[0]}x{c[1]}-{c[2]}{c[3]}" for c in BRUTE_CASES])
def test_oracle_matches_brute_force(case):
    nx, ny, xa, ya, p, u_in, g, seed = case
    flags = W.random_flags(nx, ny, p, seed)
    tau = 0.62 + 0.05 * seed
    o = Oracle(flags, tau=tau, x_axis=xa, y_axis=ya, u_in=u_in, g=g)
    st = W.random_state(nx, ny, 0.02, seed=100 + seed) + oracle.equilibrium(1, 0, 0)[:, None, None]
    o.set_state(st)
    st = o.state  # inlet / solid nodes normalised by the oracle
    b = brute_ref.Brute(flags.tolist(), tau, xa, ya, u_in=u_in, g=g)
    post = brute_ref.to_nested(st)
    upd = (o.types == oracle.FLUID) | (o.types == oracle.OUTLET)
    for k in range(20):
        post = b.step(post)
        o.run(1)
        ref = brute_ref.from_nested(post)
        assert np.abs((ref - o.state)[:, upd]).max() <= 1e-13, f"step {k + 1}"
    # incoming populations used by the readout agree with the brute-force scatter
    b.step(post)
    fin = o.incoming()
    for y in range(ny):
        for x in range(nx):
            if upd[y, x]:
                assert np.abs(np.array(b._last_fin[y][x]) - fin[:, y, x]).max() <= 1e-15


def test_light_cone_crop_equals_full_run():
    """After n steps a node depends only on nodes within n cells; a cropped run
    with arbitrary fake edges agrees with the full run on the interior.  This
    licenses cropped oracle runs for the largest grids."""
    sc = W.karman(nx=160, ny=48, cx=40, cy=24, radius=6, u_in=0.05, tau=0.6)
    full = Oracle.from_scenario(sc).run(20)
    _, uxf, uyf = full.macros()
    x0, x1 = 30, 110
    crop = sc.flags[:, x0:x1]
    c = Oracle(crop, sc.tau, PERIODIC, sc.y_axis, sc.u_in, sc.g, sc.u0).run(20)
    _, uxc, uyc = c.macros()
    h = 20 + 2
    assert np.array_equal(uxf[:, x0 + h:x1 - h], uxc[:, h:-h])
    assert np.array_equal(uyf[:, x0 + h:x1 - h], uyc[:, h:-h])


# --------------------------------------------------------- pressure outlet
def test_pressure_outlet_uniform_flow_fixed_point():
    """Uniform flow u_in = (U, 0) through a velocity inlet and the Zou-He
    pressure outlet (density 1) is an exact fixed point: the rebuilt values
    equal the equilibrium ones.  A wrong normal coefficient (2/3) or a wrong
    diagonal share (1/6) moves the outlet column by O(U)."""
    flags = np.zeros((10, 24), np.uint8)
    o = Oracle(flags, tau=0.65, x_axis=oracle.INFLOW_PRESSURE, y_axis=PERIODIC, u_in=(0.05, 0.0),
               u0=(0.05, 0.0))
    o.run(300)
    rho, ux, uy = o.macros()
    assert np.abs(rho - 1).max() < 1e-12
    assert np.abs(ux - 0.05).max() < 1e-12 and np.abs(uy).max() < 1e-12


@pytest.mark.parametrize("y_axis", [PERIODIC, CLOSED])
def test_pressure_outlet_density_and_tangential_momentum(y_axis):
    """For any state, the incoming values of every outlet node have density
    exactly 1 and zero tangential momentum (the two constraints that define
    the rebuilt values; a sign error in the diagonal split breaks the second)."""
    nx, ny = 30, 17
    flags = W.random_flags(nx, ny, 0.1, seed=41)
    flags[:, -3:] = 0  # the outlet column and its neighbours are fluid
    o = Oracle(flags, tau=0.7, x_axis=oracle.INFLOW_PRESSURE, y_axis=y_axis, u_in=(0.04, 0.0))
    st = W.random_state(nx, ny, 0.02, seed=42) + oracle.equilibrium(1, 0.02, 0.01)[:, None, None]
    o.set_state(st)
    o.run(3)
    fin = o.incoming()
    cx, cy, _, _ = oracle.constants()
    out = o.types[:, -1] == oracle.OUTLET
    assert out.sum() >= ny - 2
    rho = fin[:, :, -1].sum(axis=0)[out]
    jy = np.tensordot(cy, fin[:, :, -1], axes=(0, 0))[out]
    assert np.abs(rho - 1).max() < 1e-14
    assert np.abs(jy).max() < 1e-14


def test_pressure_outlet_changes_only_outlet_incoming_c_x_minus():
    """Against the zero-gradient outlet on the same state, the incoming values
    differ only at outlet nodes and only in the three c_x = -1 directions."""
    nx, ny = 26, 13
    flags = W.random_flags(nx, ny, 0.1, seed=43)
    st = W.random_state(nx, ny, 0.02, seed=44) + oracle.equilibrium(1, 0.03, 0.0)[:, None, None]
    fins = []
    for xa in (INFLOW_OUTFLOW, oracle.INFLOW_PRESSURE):
        o = Oracle(flags, tau=0.8, x_axis=xa, y_axis=CLOSED, u_in=(0.03, 0.0))
        o.set_state(st)
        fins.append(o.incoming())
    d = np.abs(fins[0] - fins[1]) > 0
    cx = oracle.constants()[0]
    assert not d[:, :, :-1].any()
    assert not d[cx != -1].any()
    assert d[cx == -1][:, :, -1].any()


# ------------------------------------------------------------- Neumann inlet
NEUMANN_CASES = [
    # nx, ny, y_axis, p_solid, u_in, seed
    (16, 9, CLOSED, 0.15, (0.05, 0.01), 9),
    (16, 9, PERIODIC, 0.2, (0.04, -0.02), 10),
    (2, 5, PERIODIC, 0.0, (0.05, 0.02), 11),
    (5, 4, CLOSED, 0.3, (0.03, 0.0), 12),
]


@pytest.mark.parametrize("case", NEUMANN_CASES, ids=[f"{c[0]}x{c[1]}-{c[2]}" for c in NEUMANN_CASES])
def test_neumann_inlet_matches_brute_force(case):
    """The Neumann-density inlet against the push formulation, where each inlet
    row scatters feq(rho, u_in) with rho summed from its own row's node in
    column 1: a wrong source row (c_y sign) or a stale density fails here,
    since the random state gives every row of column 1 its own density."""
    nx, ny, ya, p, u_in, seed = case
    flags = W.random_flags(nx, ny, p, seed)
    flags[:, 0] = 0
    tau = 0.6 + 0.04 * seed
    o = Oracle(flags, tau=tau, x_axis=oracle.NEUMANN_OUTFLOW, y_axis=ya, u_in=u_in)
    st = W.random_state(nx, ny, 0.02, seed=200 + seed) + oracle.equilibrium(1, 0, 0)[:, None, None]
    o.set_state(st)
    st = o.state
    b = brute_ref.Brute(flags.tolist(), tau, INFLOW_OUTFLOW, ya, u_in=u_in, neumann=True)
    post = brute_ref.to_nested(st)
    upd = (o.types == oracle.FLUID) | (o.types == oracle.OUTLET)
    for k in range(12):
        post = b.step(post)
        o.run(1)
        ref = brute_ref.from_nested(post)
        assert np.abs((ref - o.state)[:, upd]).max() <= 1e-13, f"step {k + 1}"
    b.step(post)
    fin = o.incoming()
    for y in range(ny):
        for x in range(nx):
            if upd[y, x]:
                assert np.abs(np.array(b._last_fin[y][x]) - fin[:, y, x]).max() <= 1e-15


def test_neumann_inlet_uniform_flow_fixed_point_at_any_density():
    """Uniform flow at density 1.03 through a Neumann inlet and a zero-gradient
    outlet is an exact fixed point, and the inlet reads density 1.03; with the
    Dirichlet inlet (density 1) the same state is not."""
    flags = np.zeros((8, 20), np.uint8)
    st = np.repeat(np.repeat(oracle.equilibrium(1.03, 0.05, 0.0)[:, None, None], 8, 1), 20, 2)
    o = Oracle(flags, tau=0.7, x_axis=oracle.NEUMANN_OUTFLOW, y_axis=PERIODIC, u_in=(0.05, 0.0))
    o.set_state(st)
    o.run(200)
    rho, ux, uy = o.macros()
    assert np.abs(rho - 1.03).max() < 1e-12
    assert np.abs(ux - 0.05).max() < 1e-12 and np.abs(uy).max() < 1e-12
    d = Oracle(flags, tau=0.7, x_axis=INFLOW_OUTFLOW, y_axis=PERIODIC, u_in=(0.05, 0.0))
    d.set_state(st)
    d.run(5)
    assert np.abs(d.macros()[0][:, :2] - 1.03).max() > 1e-3


def test_neumann_inlet_and_pressure_outlet_compose():
    """With both the Neumann inlet and the pressure outlet, the incoming values
    equal the pressure-outlet-only ones everywhere but the inlet column and the
    three inlet-fed directions (c_x = +1) of column 1, and the Neumann-only ones everywhere but
    the three c_x = -1 directions of the outlet column."""
    nx, ny = 18, 11
    flags = W.random_flags(nx, ny, 0.1, seed=51)
    flags[:, :2] = 0
    st = W.random_state(nx, ny, 0.02, seed=52) + oracle.equilibrium(1, 0.03, 0.0)[:, None, None]
    fin = {}
    for xa in (oracle.INFLOW_PRESSURE, oracle.NEUMANN_OUTFLOW, oracle.NEUMANN_PRESSURE):
        o = Oracle(flags, tau=0.8, x_axis=xa, y_axis=PERIODIC, u_in=(0.03, 0.0))
        o.set_state(st)
        fin[xa] = o.incoming()
    cx = oracle.constants()[0]
    both = fin[oracle.NEUMANN_PRESSURE]
    d_in = np.abs(both - fin[oracle.INFLOW_PRESSURE]) > 0
    d_out = np.abs(both - fin[oracle.NEUMANN_OUTFLOW]) > 0
    assert not d_in[cx != 1][:, :, 1:].any() and not d_in[:, :, 2:].any()
    assert d_in[cx == 1][:, :, 1].all()
    assert d_in[:, :, 0].all()  # the inlet nodes' own values: feq at the row's density
    assert not d_out[cx != -1].any() and not d_out[:, :, :-1].any()
    assert d_out[cx == -1][:, :, -1].any()


# ------------------------------------------------------- full-way bounce-back
FULLWAY_CASES = [
    # nx, ny, x_axis, y_axis, p_solid, u_in, g, seed
    (8, 8, PERIODIC, PERIODIC, 0.25, (0, 0), (1e-4, -2e-5), 31),
    (7, 6, CLOSED, CLOSED, 0.2, (0, 0), (0, 0), 32),
    (12, 7, INFLOW_OUTFLOW, CLOSED, 0.2, (0.05, 0.01), (0, 0), 33),
    (10, 9, INFLOW_OUTFLOW, PERIODIC, 0.3, (0.04, -0.02), (1e-5, 0), 34),
]


@pytest.mark.parametrize("case", FULLWAY_CASES, ids=[f"{c[0]}x{c[1]}-{c[2]}{c[3]}" for c in FULLWAY_CASES])
def test_fullway_bounce_back_matches_brute_force(case):
    """Full-way bounce-back against the push formulation in which solid nodes
    receive what is pushed into them and push it back reversed one update
    later; random states give every solid node its own values."""
    nx, ny, xa, ya, p, u_in, g, seed = case
    flags = W.random_flags(nx, ny, p, seed)
    if xa == INFLOW_OUTFLOW:
        flags[:, 0] = 0
    tau = 0.62 + 0.01 * seed
    o = Oracle(flags, tau=tau, x_axis=xa, y_axis=ya, u_in=u_in, g=g, fullway=True)
    st = W.random_state(nx, ny, 0.02, seed=300 + seed) + oracle.equilibrium(1, 0, 0)[:, None, None]
    o.set_state(st)
    st = o.state
    b = brute_ref.Brute(flags.tolist(), tau, xa, ya, u_in=u_in, g=g, fullway=True)
    post = brute_ref.to_nested(st)
    hold = (o.types == oracle.FLUID) | (o.types == oracle.OUTLET) | (o.types == oracle.SOLID)
    assert (o.types == oracle.SOLID).sum() >= 3
    for k in range(12):
        post = b.step(post)
        o.run(1)
        ref = brute_ref.from_nested(post)
        assert np.abs((ref - o.state)[:, hold]).max() <= 1e-13, f"step {k + 1}"


@pytest.mark.parametrize("tau", [0.8, 0.6])
def test_fullway_poiseuille_steady_state_equals_halfway(tau):
    """In a steady state the value a wall returns no longer depends on when it
    left, so full-way and halfway bounce-back share the steady Poiseuille
    profile with the wall midway between the last fluid and the first solid
    row (the closed form pinned above)."""
    ny, H, g = 64, 62, 1e-6
    o = Oracle(W.walls(2, ny), tau=tau, x_axis=PERIODIC, y_axis=PERIODIC, g=(g, 0), fullway=True)
    nu = (tau - 0.5) / 3
    o.run(int(40 * (H / math.pi) ** 2 / nu))
    _, ux, uy = o.macros()
    exact = poiseuille_closed_form(H, tau, g)
    assert np.abs(ux[1:ny - 1, 0] - exact).max() / exact.max() < 1e-9
    assert np.abs(uy).max() < 1e-14


def test_fullway_conserves_mass_of_fluid_and_solid_together():
    """Solid nodes hold populations: the total over fluid and solid nodes is
    conserved exactly (the reversal only reorders a node's values), while
    mass held in the walls changes as values pass through them."""
    flags = W.random_flags(24, 20, 0.25, seed=35)
    o = Oracle(flags, tau=0.7, fullway=True)
    o.set_state(W.random_state(24, 20, 0.02, seed=36) + oracle.equilibrium(1, 0, 0)[:, None, None])
    solid = o.types == oracle.SOLID
    m0, s0 = o.state.sum(), o.state[:, solid].sum()
    o.run(50)
    assert abs(o.state.sum() - m0) < 1e-14 * m0
    assert abs(o.state[:, solid].sum() - s0) > 1e-6
