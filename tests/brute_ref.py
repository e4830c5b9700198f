"""Literal brute-force reference for tiny grids (pure Python, float64).

An independent second formulation used only to pin the oracle: it streams by
*push* (scatter, Eq. 3 read left to right) instead of the oracle's pull, and it
realises the zero-gradient outlet with a ghost column x = nx that copies the
last column, instead of clamping source coordinates.  Halfway bounce-back
sends a value that would enter a solid node (or leave through a closed side)
back into the sender's opposite slot.  The inlet column pushes equilibrium
values at the inlet velocity, with density 1 (Dirichlet) or, with
``neumann=True``, the density of the same row's node next to the inlet
(its post-collision sum, read from the state being streamed).  Collision is Eq. 1 with the D2Q9I equilibrium of Eq. 2
and a simple force term 3 w_i (c_i . g).  With ``fullway=True`` solid nodes
instead hold values: they receive what is pushed into them and send every
value back the opposite way on the next push (full-way bounce-back); closed
sides stay halfway.

Shares nothing with ``oracle/``.
"""
from __future__ import annotations

import math

FLUID, SOLID, INLET, OUTLET = 0, 1, 2, 3
PERIODIC, CLOSED, INFLOW_OUTFLOW = 0, 1, 2

# Fig. 2 (b) arrows: SW S SE W 0 E NW N NE, written out by hand.
ARROWS = [(-1, -1), (0, -1), (1, -1), (-1, 0), (0, 0), (1, 0), (-1, 1), (0, 1), (1, 1)]
WEIGHTS = [1 / 36, 1 / 9, 1 / 36, 1 / 9, 4 / 9, 1 / 9, 1 / 36, 1 / 9, 1 / 36]


def opposite(i):
    cx, cy = ARROWS[i]
    return ARROWS.index((-cx, -cy))


def feq(rho, vx, vy):
    out = []
    for i, (cx, cy) in enumerate(ARROWS):
        vc = vx * cx + vy * cy
        out.append(WEIGHTS[i] * (rho + 3 * vc + 4.5 * vc * vc - 1.5 * (vx * vx + vy * vy)))
    return out


def node_types(flags, x_axis):
    ny, nx = len(flags), len(flags[0])
    t = [[FLUID] * nx for _ in range(ny)]
    for y in range(ny):
        for x in range(nx):
            if flags[y][x]:
                t[y][x] = SOLID
            elif x_axis == INFLOW_OUTFLOW and x == 0:
                t[y][x] = INLET
            elif x_axis == INFLOW_OUTFLOW and x == nx - 1:
                t[y][x] = OUTLET
    return t


class Brute:
    def __init__(self, flags, tau, x_axis, y_axis, u_in=(0.0, 0.0), g=(0.0, 0.0), neumann=False, fullway=False):
        self.ny, self.nx = len(flags), len(flags[0])
        self.types = node_types(flags, x_axis)
        self.tau, self.xa, self.ya = tau, x_axis, y_axis
        self.u_in, self.g, self.neumann, self.fullway = u_in, g, neumann, fullway
        self.holders = (FLUID, OUTLET, SOLID) if fullway else (FLUID, OUTLET)  # nodes that hold values

    def _inlet_values(self, post, y):
        rho = 1.0
        if self.neumann and self.nx > 1 and self.types[y][1] in (FLUID, OUTLET):
            rho = sum(post[y][1])
        return feq(rho, *self.u_in)

    def _target(self, x, y, i):
        """Where a value leaving (x, y) in direction i lands: ('cell', x, y),
        ('ghost', x, y) past the outlet, or ('wall',) for a closed side."""
        cx, cy = ARROWS[i]
        tx, ty = x + cx, y + cy
        if ty < 0 or ty >= self.ny:
            if self.ya == PERIODIC:
                ty %= self.ny
            else:
                return ("wall",)
        if tx < 0 or tx >= self.nx:
            if self.xa == PERIODIC:
                tx %= self.nx
            elif self.xa == INFLOW_OUTFLOW and tx == self.nx:
                return ("ghost", tx, ty)
            else:
                return ("wall",)
        return ("cell", tx, ty)

    def step(self, post):
        """post[y][x][i]: post-collision values of updated nodes (pull state).
        Returns the next post-collision state."""
        nx, ny, T = self.nx, self.ny, self.types
        fin = [[[None] * 9 for _ in range(nx)] for _ in range(ny)]
        # scatter from updated nodes
        for y in range(ny):
            for x in range(nx):
                kind = T[y][x]
                if kind in self.holders:
                    vals = post[y][x]
                elif kind == INLET:
                    vals = self._inlet_values(post, y)
                else:
                    continue
                for i in range(9):
                    tgt = self._target(x, y, i)
                    if tgt[0] == "wall":
                        if kind != INLET:
                            fin[y][x][opposite(i)] = vals[i]
                        continue
                    if tgt[0] == "ghost":
                        # the ghost copies the last-column node in row tgt[2]
                        if T[tgt[2]][nx - 1] == SOLID and kind != INLET and not self.fullway:
                            fin[y][x][opposite(i)] = vals[i]
                        continue
                    _, tx, ty = tgt
                    tk = T[ty][tx]
                    if tk == SOLID and not self.fullway:
                        if kind != INLET:
                            fin[y][x][opposite(i)] = vals[i]
                    elif tk in self.holders:
                        fin[ty][tx][i] = vals[i]
        # ghost column pushes its copies of the outlet column back into the domain
        if self.xa == INFLOW_OUTFLOW:
            for y in range(ny):
                if T[y][nx - 1] not in (OUTLET, SOLID) or (T[y][nx - 1] == SOLID and not self.fullway):
                    continue
                for i in range(9):
                    if ARROWS[i][0] != -1:
                        continue
                    ty = y + ARROWS[i][1]
                    if ty < 0 or ty >= ny:
                        if self.ya == PERIODIC:
                            ty %= ny
                        else:
                            continue
                    if T[ty][nx - 1] in self.holders:
                        fin[ty][nx - 1][i] = post[y][nx - 1][i]
        # collide
        out = [[list(post[y][x]) for x in range(nx)] for y in range(ny)]
        for y in range(ny):
            for x in range(nx):
                if T[y][x] not in self.holders:
                    continue
                f = fin[y][x]
                assert all(v is not None for v in f), f"unfilled incoming value at {(x, y)}"
                if T[y][x] == SOLID:  # full-way: send everything back
                    out[y][x] = [f[opposite(i)] for i in range(9)]
                    continue
                rho = sum(f)
                vx = sum(f[i] * ARROWS[i][0] for i in range(9))
                vy = sum(f[i] * ARROWS[i][1] for i in range(9))
                e = feq(rho, vx, vy)
                for i in range(9):
                    force = 3 * WEIGHTS[i] * (ARROWS[i][0] * self.g[0] + ARROWS[i][1] * self.g[1])
                    out[y][x][i] = f[i] - (f[i] - e[i]) / self.tau + force
        self._last_fin = fin
        return out

    def run(self, post, steps):
        for _ in range(steps):
            post = self.step(post)
        return post


def to_nested(state):
    """(9, ny, nx) array -> post[y][x][i] nested lists."""
    _, ny, nx = state.shape
    return [[[float(state[i, y, x]) for i in range(9)] for x in range(nx)] for y in range(ny)]


def from_nested(post):
    import numpy as np
    ny, nx = len(post), len(post[0])
    a = np.zeros((9, ny, nx))
    for y in range(ny):
        for x in range(nx):
            for i in range(9):
                a[i, y, x] = post[y][x][i]
    return a


def is_finite(v):
    return not (math.isnan(v) or math.isinf(v))
