"""Seeded synthetic inputs for the D2Q9 lattice update: obstacle flag arrays and
request traces.

This module holds input data only (geometry, random draws, trace statistics);
it contains none of the lattice Boltzmann arithmetic, so both the FP64 oracle
tests and the HIP path consume the same arrays from here.

Flags are ``uint8`` arrays of shape ``(ny, nx)``, row-major with ``x`` fastest
(node = y*nx + x), ``y`` growing upwards; value 0 = fluid, 1 = solid.

Scenarios follow the paper's synthetic cases (Section 5: Hagen-Poiseuille
channel, Karman vortex street behind circle / square / plate obstacles, porous
medium with randomly placed solids) at the sizes of the benchmark workloads.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FLUID = 0
SOLID = 1

# Axis kinds (mirror the C enum values of the library header).
PERIODIC = 0
CLOSED = 1
INFLOW_OUTFLOW = 2
INFLOW_PRESSURE = 3  # inlet column and a pressure (Zou-He) outlet column
NEUMANN_OUTFLOW = 4  # Neumann-density inlet and a zero-gradient outlet
NEUMANN_PRESSURE = 5  # Neumann-density inlet and a pressure outlet


@dataclass
class Scenario:
    """One simulation setup: flags plus the physical parameters."""

    name: str
    flags: np.ndarray  # uint8 (ny, nx)
    tau: float
    x_axis: int
    y_axis: int
    u_in: tuple = (0.0, 0.0)
    g: tuple = (0.0, 0.0)
    u0: tuple = (0.0, 0.0)
    steps: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def ny(self) -> int:
        return int(self.flags.shape[0])

    @property
    def nx(self) -> int:
        return int(self.flags.shape[1])


def walls(nx: int, ny: int) -> np.ndarray:
    """Empty channel: rows 0 and ny-1 solid."""
    f = np.zeros((ny, nx), dtype=np.uint8)
    f[0, :] = SOLID
    f[ny - 1, :] = SOLID
    return f


def add_disc(flags: np.ndarray, cx: float, cy: float, r: float, periodic: bool = False) -> None:
    """Mark solid every cell whose centre (x, y) satisfies (x-cx)^2+(y-cy)^2 <= r^2."""
    ny, nx = flags.shape
    x0, x1 = int(math.floor(cx - r)), int(math.ceil(cx + r))
    y0, y1 = int(math.floor(cy - r)), int(math.ceil(cy + r))
    xs = np.arange(x0, x1 + 1)
    ys = np.arange(y0, y1 + 1)
    dx = (xs - cx)[None, :]
    dy = (ys - cy)[:, None]
    inside = dx * dx + dy * dy <= r * r
    if periodic:
        xi = np.mod(xs, nx)
        yi = np.mod(ys, ny)
    else:
        keepx = (xs >= 0) & (xs < nx)
        keepy = (ys >= 0) & (ys < ny)
        inside = inside[np.ix_(keepy, keepx)]
        xi, yi = xs[keepx], ys[keepy]
    sub = flags[np.ix_(yi, xi)]
    sub[inside] = SOLID
    flags[np.ix_(yi, xi)] = sub


def add_square(flags: np.ndarray, cx: float, cy: float, side: float) -> None:
    """Mark solid the cells with |x-cx| <= side/2 and |y-cy| <= side/2."""
    ny, nx = flags.shape
    h = side / 2.0
    xs = np.arange(nx)
    ys = np.arange(ny)
    mx = np.abs(xs - cx) <= h
    my = np.abs(ys - cy) <= h
    flags[np.ix_(my, mx)] = SOLID


def add_segment(flags: np.ndarray, ax: float, ay: float, bx: float, by: float, half_width: float) -> None:
    """Mark solid every cell whose centre lies within ``half_width`` of segment AB.

    Only the bounding box of the segment is visited, so this stays cheap on the
    2^31-cell grid.
    """
    ny, nx = flags.shape
    x0 = max(int(math.floor(min(ax, bx) - half_width)) - 1, 0)
    x1 = min(int(math.ceil(max(ax, bx) + half_width)) + 1, nx - 1)
    y0 = max(int(math.floor(min(ay, by) - half_width)) - 1, 0)
    y1 = min(int(math.ceil(max(ay, by) + half_width)) + 1, ny - 1)
    if x1 < x0 or y1 < y0:
        return
    dxs, dys = bx - ax, by - ay
    L2 = dxs * dxs + dys * dys
    # Row-by-row to bound memory on very long segments.
    xs = np.arange(x0, x1 + 1, dtype=np.float64)
    for y in range(y0, y1 + 1):
        px = xs - ax
        py = float(y) - ay
        t = (px * dxs + py * dys) / L2 if L2 > 0 else np.zeros_like(px)
        t = np.clip(t, 0.0, 1.0)
        qx = px - t * dxs
        qy = py - t * dys
        hit = qx * qx + qy * qy <= half_width * half_width
        if hit.any():
            row = flags[y, x0:x1 + 1]
            row[hit] = SOLID


# ---------------------------------------------------------------- scenarios
def channel(nx: int = 128, ny: int = 64, tau: float = 0.8, gx: float = 1e-6, steps: int = 2000) -> Scenario:
    """Hagen-Poiseuille channel: solid rows 0 and ny-1, periodic in x, body force."""
    return Scenario("channel", walls(nx, ny), tau, PERIODIC, CLOSED, g=(gx, 0.0), steps=steps,
                    meta={"fluid_rows": ny - 2})


def karman(nx: int = 4096, ny: int = 1024, cx: float = 1024.0, cy: float = 512.0, radius: float = 64.0,
           u_in: float = 0.05, tau: float | None = None, reynolds: float = 100.0, steps: int = 10000) -> Scenario:
    """Karman vortex street: walls, equilibrium inlet at x=0, zero-gradient outlet,
    circular cylinder of diameter 2*radius. tau from Re = u_in * D / nu."""
    f = walls(nx, ny)
    add_disc(f, cx, cy, radius)
    if tau is None:
        nu = u_in * (2.0 * radius) / reynolds
        tau = 3.0 * nu + 0.5
    return Scenario("karman", f, tau, INFLOW_OUTFLOW, CLOSED, u_in=(u_in, 0.0), u0=(u_in, 0.0), steps=steps,
                    meta={"diameter": 2.0 * radius, "reynolds": reynolds})


def porous(n: int = 2048, seed: int = 20650, rmin: float = 8.0, rmax: float = 32.0, phi_max: float = 0.30,
           gap: float = 2.0, tau: float = 0.9, gx: float = 1e-6, steps: int = 20000,
           max_failures: int = 20000) -> Scenario:
    """Periodic porous medium of non-overlapping random discs.

    Sequential random addition with ``numpy.random.default_rng(seed)``: radius
    ~ U[rmin, rmax], centre ~ U[0, n)^2; a disc is accepted when its periodic
    centre distance to every accepted disc is >= r + r_j + gap; the process
    stops before the solid fraction would exceed ``phi_max`` (or after
    ``max_failures`` consecutive rejections).
    """
    rng = np.random.default_rng(seed)
    flags = np.zeros((n, n), dtype=np.uint8)
    centres: list[tuple[float, float, float]] = []
    solid = 0
    total = n * n
    failures = 0
    while failures < max_failures:
        r = float(rng.uniform(rmin, rmax))
        cx = float(rng.uniform(0.0, n))
        cy = float(rng.uniform(0.0, n))
        ok = True
        for (qx, qy, qr) in centres:
            dx = abs(cx - qx)
            dx = min(dx, n - dx)
            dy = abs(cy - qy)
            dy = min(dy, n - dy)
            if dx * dx + dy * dy < (r + qr + gap) ** 2:
                ok = False
                break
        if not ok:
            failures += 1
            continue
        failures = 0
        # Count the cells this disc would add (discs never overlap: gap >= 0).
        x0, x1 = int(math.floor(cx - r)), int(math.ceil(cx + r))
        y0, y1 = int(math.floor(cy - r)), int(math.ceil(cy + r))
        xs = np.arange(x0, x1 + 1)
        ys = np.arange(y0, y1 + 1)
        inside = (xs - cx)[None, :] ** 2 + (ys - cy)[:, None] ** 2 <= r * r
        add = int(inside.sum())
        if (solid + add) / total > phi_max:
            break
        sub = flags[np.ix_(np.mod(ys, n), np.mod(xs, n))]
        sub[inside] = SOLID
        flags[np.ix_(np.mod(ys, n), np.mod(xs, n))] = sub
        solid += add
        centres.append((cx, cy, r))
    return Scenario("porous", flags, tau, PERIODIC, PERIODIC, g=(gx, 0.0), steps=steps,
                    meta={"solid_fraction": solid / total, "discs": len(centres), "seed": seed})


def plate(nx: int = 65536, ny: int = 32768, length: float = 4096.0, angle_deg: float = 10.0,
          u_in: float = 0.04, tau: float | None = None, reynolds: float = 1000.0, steps: int = 200,
          half_thickness: float = 1.0) -> Scenario:
    """Flat plate at an angle of attack in a walled channel with inlet and outlet.

    The plate is the set of cells whose centre lies within ``half_thickness`` of
    the segment C +/- (length/2)(cos a, -sin a), C = (nx/4, ny/2)."""
    f = walls(nx, ny)
    a = math.radians(angle_deg)
    cx, cy = nx / 4.0, ny / 2.0
    hx, hy = 0.5 * length * math.cos(a), -0.5 * length * math.sin(a)
    add_segment(f, cx - hx, cy - hy, cx + hx, cy + hy, half_thickness)
    if tau is None:
        nu = u_in * length / reynolds
        tau = 3.0 * nu + 0.5
    return Scenario("plate", f, tau, INFLOW_OUTFLOW, CLOSED, u_in=(u_in, 0.0), u0=(u_in, 0.0), steps=steps,
                    meta={"length": length, "angle_deg": angle_deg})


def obstacle_channel(nx: int, ny: int, kind: str, u_in: float = 0.03, tau: float = 0.8, steps: int = 100) -> Scenario:
    """Walled channel with inlet/outlet and one obstacle (cylinder / square /
    plate) of size D = clamp(round(ny/8), 4, 128) centred at (nx/4, ny/2)."""
    f = walls(nx, ny)
    D = int(min(max(round(ny / 8), 4), 128))
    cx, cy = nx / 4.0, ny / 2.0
    if kind == "cylinder":
        add_disc(f, cx, cy, D / 2.0)
    elif kind == "square":
        add_square(f, cx, cy, float(D))
    elif kind == "plate":
        add_segment(f, cx, cy - D / 2.0, cx, cy + D / 2.0, 1.0)
    else:
        raise ValueError(f"unknown obstacle kind {kind!r}")
    return Scenario(f"{kind}-{nx}x{ny}", f, tau, INFLOW_OUTFLOW, CLOSED, u_in=(u_in, 0.0), u0=(u_in, 0.0),
                    steps=steps, meta={"obstacle": kind, "D": D})


@dataclass
class Request:
    rid: int
    arrival: float  # seconds after trace start
    nx: int
    ny: int
    kind: str
    tau: float
    steps: int

    @property
    def cells(self) -> int:
        return self.nx * self.ny

    def scenario(self) -> Scenario:
        return obstacle_channel(self.nx, self.ny, self.kind, u_in=0.03, tau=self.tau, steps=self.steps)


def request_trace(n: int = 2000, seed: int = 5, rate_per_s: float = 100.0, nx_range=(64, 2048), ny_range=(64, 1024),
                  tau_range=(0.55, 1.2), steps_range=(100, 5000)) -> list[Request]:
    """Poisson stream of independent simulation requests.

    Sizes are log-uniform per axis, obstacle kind uniform over {cylinder,
    square, plate}, tau ~ U[tau_range], steps ~ U{steps_range}; inter-arrival
    gaps ~ Exp(rate_per_s)."""
    rng = np.random.default_rng(seed)
    kinds = ("cylinder", "square", "plate")
    out = []
    t = 0.0
    for k in range(n):
        t += float(rng.exponential(1.0 / rate_per_s))
        nx = int(round(math.exp(rng.uniform(math.log(nx_range[0]), math.log(nx_range[1])))))
        ny = int(round(math.exp(rng.uniform(math.log(ny_range[0]), math.log(ny_range[1])))))
        kind = kinds[int(rng.integers(0, 3))]
        tau = float(rng.uniform(*tau_range))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        out.append(Request(k, t, nx, ny, kind, tau, steps))
    return out


def random_flags(nx: int, ny: int, p_solid: float, seed: int) -> np.ndarray:
    """Independent random solid cells (tiny-grid rule coverage)."""
    rng = np.random.default_rng(seed)
    return (rng.random((ny, nx)) < p_solid).astype(np.uint8)


def random_state(nx: int, ny: int, amplitude: float, seed: int, dtype=np.float64) -> np.ndarray:
    """Random shifted populations f~ (shape (9, ny, nx)) with |f~| <= amplitude."""
    rng = np.random.default_rng(seed)
    return (amplitude * (2.0 * rng.random((9, ny, nx)) - 1.0)).astype(dtype)


# ------------------------------------------------------------------ D3Q19
@dataclass
class Scenario3:
    """One D3Q19 setup: flags (nz, ny, nx) plus the physical parameters."""

    name: str
    flags: np.ndarray  # uint8 (nz, ny, nx)
    tau: float
    x_axis: int
    y_axis: int
    z_axis: int
    u_in: tuple = (0.0, 0.0, 0.0)
    g: tuple = (0.0, 0.0, 0.0)
    u0: tuple = (0.0, 0.0, 0.0)
    steps: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return tuple(int(s) for s in self.flags.shape)


def add_sphere(flags: np.ndarray, cx: float, cy: float, cz: float, r: float) -> None:
    """Mark nodes whose centres lie within distance r of (cx, cy, cz) solid
    (plane by plane, so large grids need no full-size temporaries)."""
    nz, ny, nx = flags.shape
    y, x = np.ogrid[:ny, :nx]
    d2 = (x - cx) ** 2 + (y - cy) ** 2
    for z in range(max(0, int(math.floor(cz - r))), min(nz, int(math.ceil(cz + r)) + 1)):
        flags[z][d2 + (z - cz) ** 2 <= r * r] = SOLID


def sphere_array(n: int = 256, radius: float = 40.0, tau: float = 0.6, gx: float = 1e-6, steps: int = 1000) -> Scenario3:
    """Simple cubic array of spheres: one sphere of radius `radius` centred in a
    periodic n^3 cell, flow driven by a body force along x."""
    f = np.zeros((n, n, n), dtype=np.uint8)
    add_sphere(f, n / 2 - 0.5, n / 2 - 0.5, n / 2 - 0.5, radius)
    return Scenario3(f"sphere-array-{n}^3", f, tau, PERIODIC, PERIODIC, PERIODIC, g=(gx, 0.0, 0.0), steps=steps,
                     meta={"solid_fraction": float(f.mean())})


def duct_sphere(nx: int = 96, ny: int = 40, nz: int = 32, radius: float = 6.0, u_in: float = 0.05,
                tau: float = 0.6, steps: int = 300) -> Scenario3:
    """Rectangular duct (closed y and z sides) with a sphere, inlet at x = 0
    and zero-gradient outlet at x = nx - 1."""
    f = np.zeros((nz, ny, nx), dtype=np.uint8)
    add_sphere(f, nx / 4, ny / 2 - 0.5, nz / 2 - 0.5, radius)
    return Scenario3(f"duct-sphere-{nx}x{ny}x{nz}", f, tau, INFLOW_OUTFLOW, CLOSED, CLOSED, u_in=(u_in, 0.0, 0.0),
                     u0=(u_in, 0.0, 0.0), steps=steps)


def random_flags3(nx: int, ny: int, nz: int, p_solid: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (rng.random((nz, ny, nx)) < p_solid).astype(np.uint8)


def random_state3(nx: int, ny: int, nz: int, amplitude: float, seed: int, dtype=np.float64) -> np.ndarray:
    """Random shifted D3Q19 populations (shape (19, nz, ny, nx)), |f~| <= amplitude."""
    rng = np.random.default_rng(seed)
    return (amplitude * (2.0 * rng.random((19, nz, ny, nx)) - 1.0)).astype(dtype)
