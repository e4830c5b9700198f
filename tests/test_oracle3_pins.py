"""Pins of the FP64 D3Q19 oracle against what the mathematics fixes.

None of these compares the 3-D oracle with itself: each checks the isotropy
conditions that determine the velocity set's weights, closed forms and
invariants, an independent push formulation on tiny grids
(tests/brute3_ref.py), or the exact reduction of plane-invariant D3Q19 flow to
the (separately pinned) D2Q9 oracle.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import d3q19 as o3
from tests import brute3_ref

CX, CY, CZ, W = o3.constants()
C = np.stack([CX, CY, CZ], axis=1)


# ------------------------------------------------------------------ velocity set
def test_velocity_set_and_weights_from_isotropy():
    """The 19 vectors with components in {-1, 0, 1} and |c|^2 <= 2, opposite
    = 18 - i, rest at 9; the weights are the solution of the isotropy
    conditions (sum w = 1, sum w c_a c_b = d_ab / 3, fourth moment
    (d d + d d + d d) / 9) for shells |c|^2 = 0, 1, 2."""
    want = sorted((c for c in itertools.product((-1, 0, 1), repeat=3) if sum(a * a for a in c) <= 2),
                  key=lambda c: (c[2], c[1], c[0]))
    assert [tuple(c) for c in C] == want
    assert np.array_equal(C[18 - np.arange(19)], -C) and not C[9].any()
    # solve the isotropy conditions for the three shell weights
    shell = (C * C).sum(1)
    A = np.array([[np.sum(shell == s) for s in (0, 1, 2)],
                  [np.sum((C[:, 0] ** 2)[shell == s]) for s in (0, 1, 2)],
                  [np.sum((C[:, 0] ** 2 * C[:, 1] ** 2)[shell == s]) for s in (0, 1, 2)]], float)
    ws = np.linalg.solve(A, [1.0, 1 / 3, 1 / 9])
    assert np.allclose(W, ws[shell], atol=1e-15)
    d = np.eye(3)
    m2 = np.einsum("i,ia,ib->ab", W, C, C)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", W, C, C, C, C)
    iso4 = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9
    assert abs(W.sum() - 1) < 1e-15 and np.allclose(m2, d / 3, atol=1e-15) and np.allclose(m4, iso4, atol=1e-15)
    assert np.allclose(np.einsum("i,ia->a", W, C), 0) and np.allclose(np.einsum("i,ia,ib,ic->abc", W, C, C, C), 0)


def test_equilibrium_moments_closed_form():
    rng = np.random.default_rng(3)
    for _ in range(20):
        rho = 1 + 0.1 * rng.standard_normal()
        u = 0.1 * rng.standard_normal(3)
        f = o3.equilibrium(rho, *u)
        assert abs(f.sum() - rho) < 1e-14
        assert np.allclose(C.T @ f, u, atol=1e-15)
        assert np.allclose(np.einsum("i,ia,ib->ab", f, C, C), rho / 3 * np.eye(3) + np.outer(u, u), atol=1e-15)


# ------------------------------------------------------------------ invariants
def _random_state(shape, amp, seed):
    rng = np.random.default_rng(seed)
    return W[:, None, None, None] * (1 + amp * rng.standard_normal((19,) + shape))


def test_uniform_flow_fixed_point_and_conservation():
    flags = np.zeros((6, 5, 7), np.uint8)
    o = o3.Oracle3(flags, tau=0.7, u0=(0.03, -0.02, 0.01))
    f0 = o.state.copy()
    o.run(20)
    assert np.abs(o.state - f0).max() < 1e-16
    # random state, random solids: mass conserved; momentum too without solids
    rng = np.random.default_rng(5)
    flags = (rng.random((6, 7, 8)) < 0.2).astype(np.uint8)
    for fl in (flags, np.zeros_like(flags)):
        o = o3.Oracle3(fl, tau=0.8)
        o.set_state(_random_state(fl.shape, 0.05, 6))
        st = o.state
        m0 = st.sum()
        p0 = C.T @ st.reshape(19, -1).sum(axis=1)
        o.run(30)
        assert abs(o.state.sum() - m0) < 1e-12
        if not fl.any():
            assert np.allclose(C.T @ o.state.reshape(19, -1).sum(axis=1), p0, atol=1e-13)


def test_shear_wave_decay_rate():
    """u_x = A sin(k z) in a periodic box decays as exp(-nu k^2 t)."""
    n, tau, A = 48, 0.8, 1e-4
    nu = (tau - 0.5) / 3
    k = 2 * math.pi / n
    o = o3.Oracle3(np.zeros((n, 2, 2), np.uint8), tau=tau)
    st = np.zeros((19, n, 2, 2))
    for z in range(n):
        st[:, z] = o3.equilibrium(1.0, A * math.sin(k * z), 0.0, 0.0)[:, None, None]
    o.set_state(st)
    amps = []
    for t in (200, 1700):
        o.run(t - o.t)
        _, u = o.macros()
        amps.append(2 / n * (u[0, :, 0, 0] * np.sin(k * np.arange(n))).sum())
    rate = math.log(amps[0] / amps[1]) / 1500
    assert abs(rate / (nu * k * k) - 1) < 0.01


# ------------------------------------------------------------------ brute force
BRUTE3_CASES = [
    # shape (nz, ny, nx), axes, p_solid, u_in, g, seed
    ((4, 3, 5), (o3.PERIODIC, o3.PERIODIC, o3.PERIODIC), 0.2, (0, 0, 0), (1e-4, 0, -2e-5), 1),
    ((3, 4, 5), (o3.CLOSED, o3.CLOSED, o3.CLOSED), 0.15, (0, 0, 0), (0, 0, 0), 2),
    ((4, 4, 6), (o3.INFLOW_OUTFLOW, o3.CLOSED, o3.PERIODIC), 0.15, (0.05, 0.01, -0.02), (0, 0, 0), 3),
    ((3, 5, 6), (o3.INFLOW_OUTFLOW, o3.PERIODIC, o3.CLOSED), 0.1, (0.04, 0, 0.01), (1e-5, 0, 0), 4),
    ((3, 3, 2), (o3.INFLOW_OUTFLOW, o3.PERIODIC, o3.PERIODIC), 0.0, (0.05, 0.02, 0), (0, 0, 0), 5),
]


@pytest.mark.parametrize("case", BRUTE3_CASES, ids=[f"{c[0]}-{c[1]}" for c in BRUTE3_CASES])
def test_oracle3_matches_brute_force(case):
    shape, axes, p, u_in, g, seed = case
    rng = np.random.default_rng(seed)
    flags = (rng.random(shape) < p).astype(np.uint8)
    tau = 0.6 + 0.05 * seed
    o = o3.Oracle3(flags, tau, *axes, u_in=u_in, g=g)
    o.set_state(_random_state(shape, 0.1, 50 + seed))
    st = o.state
    b = brute3_ref.Brute3(flags.tolist(), tau, axes, u_in=u_in, g=g)
    nz, ny, nx = shape
    upd = (o.types == o3.FLUID) | (o.types == o3.OUTLET)
    post = {(x, y, z): list(st[:, z, y, x]) for z in range(nz) for y in range(ny) for x in range(nx) if upd[z, y, x]}
    for k in range(8):
        post = b.step(post)
        o.run(1)
        ref = np.zeros_like(st)
        for (x, y, z), v in post.items():
            ref[:, z, y, x] = v
        assert np.abs((ref - o.state)[:, upd]).max() <= 1e-13, f"step {k + 1}"
    b.step(post)
    fin = o.incoming()
    for (x, y, z), v in b.last_fin.items():
        assert np.abs(np.array(v) - fin[:, z, y, x]).max() <= 1e-15


# ------------------------------------------------------- reduction to D2Q9
# D2Q9 plane -> 3-D axes: (3-D axis of the plane's x, of the plane's y, uniform axis)
PLANES = {"y": (0, 2, 1), "z": (0, 1, 2), "x": (1, 2, 0)}


def _embed(a2, axis, n=3):
    """A (rows = plane y, cols = plane x) array -> (nz, ny, nx), uniform along axis."""
    if axis == "y":
        return np.repeat(a2[:, None, :], n, axis=1)
    if axis == "z":
        return np.repeat(a2[None, :, :], n, axis=0)
    return np.repeat(a2[:, :, None], n, axis=2)


def _plane(a3, axis):
    return {"y": a3[:, 0, :], "z": a3[0], "x": a3[:, :, 0]}[axis]


@pytest.mark.parametrize("axis", ["y", "z", "x"])
def test_plane_invariant_flow_reduces_to_d2q9(axis):
    """A D3Q19 state uniform along one axis, with geometry uniform along it
    and populations symmetric in that axis' component (so no velocity along
    it), evolves so that the populations summed over that component equal the
    D2Q9 populations of the plane, exactly: the equilibria, forces,
    bounce-back, inlet and outlet of the two models agree under the summation.
    With the axis permuted this pins streaming along every axis of the 3-D
    oracle to the pinned D2Q9 oracle."""
    from paper_2607_20650_amd import workloads as Wk
    n1, n2 = 24, 11
    px, py, uni = PLANES[axis]
    flags2 = Wk.random_flags(n1, n2, 0.12, seed=21)
    u_in2, g2 = (0.04, 0.01), (1e-5, -3e-6)
    xa2 = oracle.INFLOW_OUTFLOW if px == 0 else oracle.PERIODIC
    ref = oracle.Oracle(flags2, 0.72, xa2, oracle.CLOSED, u_in2, g2)
    ref.set_state(Wk.random_state(n1, n2, 0.02, seed=22) + oracle.equilibrium(1, 0, 0)[:, None, None])
    st2 = ref.state
    cx2, cy2, _, _ = oracle.constants()
    groups = [[i for i in range(19) if C[i, px] == cx2[j] and C[i, py] == cy2[j]] for j in range(9)]
    f3 = np.zeros((19,) + _embed(st2[0], axis).shape)
    for j, members in enumerate(groups):
        for i in members:
            f3[i] = _embed(st2[j], axis) * W[i] / W[members].sum()
    axes = [o3.PERIODIC] * 3
    axes[px] = o3.INFLOW_OUTFLOW if px == 0 else o3.PERIODIC
    axes[py] = o3.CLOSED
    vec = lambda v: tuple(v[0] if a == px else (v[1] if a == py else 0.0) for a in range(3))
    o = o3.Oracle3(_embed(flags2, axis), 0.72, *axes, u_in=vec(u_in2), g=vec(g2))
    o.set_state(f3)
    ref.run(15)
    o.run(15)
    s3 = o.state
    for j, members in enumerate(groups):
        summed = s3[members].sum(axis=0)
        assert np.abs(_plane(summed, axis) - ref.state[j]).max() < 1e-14, j
        assert np.abs(summed - _embed(_plane(summed, axis), axis)).max() < 1e-15, j
