"""Literal brute-force D3Q19 reference for tiny grids (pure Python, float64).

A second formulation used only to pin the 3-D oracle: it streams by *push*
(each node scatters its post-collision values), realises the zero-gradient
outlet with a ghost plane x = nx that copies the last plane, and sends a value
that would enter a solid node or leave through a closed side back into the
sender's opposite slot.  Inlet nodes push feq(1, u_in).  Collision is BGK with
the incompressible equilibrium and the force term 3 w_i (c_i . g).

Shares nothing with ``oracle/``.
"""
from __future__ import annotations

FLUID, SOLID, INLET, OUTLET = 0, 1, 2, 3
PERIODIC, CLOSED, INFLOW_OUTFLOW = 0, 1, 2

# D3Q19 written out by hand: the 6 faces, then the 12 edges, then rest;
# reordered below into (c_z, c_y, c_x) lexicographic order.
_FACES = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
_EDGES = [(1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
          (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
VELOCITIES = sorted(_FACES + _EDGES + [(0, 0, 0)], key=lambda c: (c[2], c[1], c[0]))
WEIGHTS = [1 / 3 if c == (0, 0, 0) else (1 / 18 if sum(abs(a) for a in c) == 1 else 1 / 36) for c in VELOCITIES]


def opposite(i):
    c = VELOCITIES[i]
    return VELOCITIES.index((-c[0], -c[1], -c[2]))


def feq(rho, u):
    uu = u[0] ** 2 + u[1] ** 2 + u[2] ** 2
    out = []
    for c, w in zip(VELOCITIES, WEIGHTS):
        cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2]
        out.append(w * (rho + 3 * cu + 4.5 * cu * cu - 1.5 * uu))
    return out


class Brute3:
    def __init__(self, flags, tau, axes, u_in=(0.0, 0.0, 0.0), g=(0.0, 0.0, 0.0)):
        """flags[z][y][x] (nested lists); axes = (x_axis, y_axis, z_axis)."""
        self.nz, self.ny, self.nx = len(flags), len(flags[0]), len(flags[0][0])
        self.axes, self.tau, self.u_in, self.g = axes, tau, u_in, g
        self.T = {}
        for z in range(self.nz):
            for y in range(self.ny):
                for x in range(self.nx):
                    t = FLUID
                    if flags[z][y][x]:
                        t = SOLID
                    elif axes[0] == INFLOW_OUTFLOW and x == 0:
                        t = INLET
                    elif axes[0] == INFLOW_OUTFLOW and x == self.nx - 1:
                        t = OUTLET
                    self.T[(x, y, z)] = t

    def _wrap(self, axis, v, n):
        """Coordinate after a periodic wrap, or None outside a closed side."""
        if 0 <= v < n:
            return v
        if self.axes[axis] == PERIODIC:
            return v % n
        return None

    def step(self, post):
        """post[(x, y, z)] = list of 19 post-collision values (updated nodes)."""
        nx, ny, nz, T = self.nx, self.ny, self.nz, self.T
        fin = {k: [None] * 19 for k, t in T.items() if t in (FLUID, OUTLET)}
        ein = feq(1.0, self.u_in)
        for (x, y, z), kind in T.items():
            if kind == SOLID:
                continue
            vals = ein if kind == INLET else post[(x, y, z)]
            for i, c in enumerate(VELOCITIES):
                ty, tz = self._wrap(1, y + c[1], ny), self._wrap(2, z + c[2], nz)
                tx = x + c[0]
                back = False
                if ty is None or tz is None:
                    back = True
                elif tx == nx and self.axes[0] == INFLOW_OUTFLOW:
                    # into the ghost plane: dropped (the ghost copies the last
                    # plane), unless the copied node is solid
                    back = T[(nx - 1, ty, tz)] == SOLID
                    if not back:
                        continue
                else:
                    tx = self._wrap(0, tx, nx)
                    if tx is None:
                        back = True
                    elif T[(tx, ty, tz)] == SOLID:
                        back = True
                    elif T[(tx, ty, tz)] in (FLUID, OUTLET):
                        fin[(tx, ty, tz)][i] = vals[i]
                    # into an inlet node: nothing (its values are fixed)
                if back and kind != INLET:
                    fin[(x, y, z)][opposite(i)] = vals[i]
        # the ghost plane pushes copies of the outlet plane back into it
        if self.axes[0] == INFLOW_OUTFLOW:
            for y in range(ny):
                for z in range(nz):
                    if T[(nx - 1, y, z)] != OUTLET:
                        continue
                    for i, c in enumerate(VELOCITIES):
                        if c[0] != -1:
                            continue
                        ty, tz = self._wrap(1, y + c[1], ny), self._wrap(2, z + c[2], nz)
                        if ty is None or tz is None:
                            continue
                        if T[(nx - 1, ty, tz)] in (FLUID, OUTLET):
                            fin[(nx - 1, ty, tz)][i] = post[(nx - 1, y, z)][i]
        out = {}
        for k, f in fin.items():
            assert all(v is not None for v in f), f"unfilled incoming value at {k}"
            rho = sum(f)
            u = [sum(f[i] * VELOCITIES[i][a] for i in range(19)) for a in range(3)]
            e = feq(rho, u)
            out[k] = [f[i] - (f[i] - e[i]) / self.tau
                      + 3 * WEIGHTS[i] * sum(VELOCITIES[i][a] * self.g[a] for a in range(3)) for i in range(19)]
        self.last_fin = fin
        return out
