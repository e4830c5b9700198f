"""CPU model of the one-lattice schemes' tile phases under random schedules.

The one-lattice schemes of Section 3.3 (NPOL: pull with a buffer grid; NSOL:
swap) update the lattice in place, tile by tile.  Inside a tile a barrier puts
every read before every write; across tiles there is no order at all within
an update, so a tile may run before, after or interleaved with its
neighbours.  Values that leave a tile travel through edge buffers that are
double-buffered by update parity: a reader takes what its neighbour published
in the previous update, a writer publishes into the other parity.

This test is a plain NumPy model of that design (the edge-buffer index maps
of the library's buffer grid, restated here: X edges [tile column][side]
[c_y + 1][row], Y edges [tile row][side][c_x + 1][column], corners taken from
the Y edges), run under random interleavings of the tiles' read and write
phases, and compared bit for bit with a plain two-lattice pull on the same
states.  Sources across a closed side or on a solid node bounce back (the
node's own slot of the opposite direction).  The per-node update is a fixed
linear mixing of the nine incoming values: the schedule, not the physics, is
under test, and both sides apply it identically.

Planted mistakes (single-buffered edges; reads and writes of a tile not
separated by the barrier) must make some schedule differ from the reference,
which shows that the fuzzer can see a schedule fault.
"""
from __future__ import annotations

import numpy as np
import pytest

CX = np.array([i % 3 - 1 for i in range(9)])
CY = np.array([i // 3 - 1 for i in range(9)])
OPP = np.array([8 - i for i in range(9)])


def mixing(seed=3):
    rng = np.random.default_rng(seed)
    m = 0.1 * rng.random((9, 9))
    np.fill_diagonal(m, 0.5)
    return m


def collide(f, m):
    """Post-update values of one node from its nine incoming values."""
    return m @ f


def source(x, y, i, nx, ny, periodic_y):
    """Pull source of direction i for node (x, y) (x periodic); None across a
    closed side."""
    sx, sy = (x - CX[i]) % nx, y - CY[i]
    if not 0 <= sy < ny:
        if not periodic_y:
            return None
        sy %= ny
    return sx, sy


def reference(state, solid, steps, m, periodic_y):
    """Two-lattice pull: state[i, y, x] = post-update value f*_i(x, y)."""
    ny, nx = solid.shape
    cur = state.copy()
    for _ in range(steps):
        nxt = np.zeros_like(cur)
        for y in range(ny):
            for x in range(nx):
                if solid[y, x]:
                    continue
                f = np.empty(9)
                for i in range(9):
                    s = source(x, y, i, nx, ny, periodic_y)
                    f[i] = cur[OPP[i], y, x] if s is None or solid[s[1], s[0]] else cur[i, s[1], s[0]]
                nxt[:, y, x] = collide(f, m)
        cur = nxt
    return cur


class OneLattice:
    """One lattice + parity edge buffers, tile phases run in a given order.

    swap=False: NPOL storage (f*_i in slot i); swap=True: NSOL storage (f*_i
    in slot opposite(i)).  single_buffer / no_barrier plant design mistakes."""

    def __init__(self, state, solid, tx, ty, m, periodic_y, swap, single_buffer=False, no_barrier=False):
        self.ny, self.nx = solid.shape
        self.solid, self.tx, self.ty, self.m = solid, tx, ty, m
        self.periodic_y, self.swap = periodic_y, swap
        self.single_buffer, self.no_barrier = single_buffer, no_barrier
        self.ntx, self.nty = -(-self.nx // tx), -(-self.ny // ty)
        rows, cols = self.nty * ty, self.ntx * tx
        self.lat = np.zeros_like(state)
        for i in range(9):
            self.lat[OPP[i] if swap else i] = state[i]
        self.xe = np.full((2, self.ntx, 2, 3, rows), np.nan)
        self.ye = np.full((2, self.nty, 2, 3, cols), np.nan)
        self.publish_all(state, 0)

    def slot(self, i):
        return OPP[i] if self.swap else i

    def tile(self, bx, by):
        return bx * self.tx, by * self.ty, min(bx * self.tx + self.tx, self.nx), min(by * self.ty + self.ty, self.ny)

    def publish(self, fstar, x, y, bx, by, parity):
        x0, y0, x1, y1 = self.tile(bx, by)
        p = 0 if self.single_buffer else parity
        for i in range(9):
            if x == x0 and CX[i] == -1:
                self.xe[p, bx, 0, CY[i] + 1, y] = fstar[i]
            if x == x1 - 1 and CX[i] == 1:
                self.xe[p, bx, 1, CY[i] + 1, y] = fstar[i]
            if y == y0 and CY[i] == -1:
                self.ye[p, by, 0, CX[i] + 1, x] = fstar[i]
            if y == y1 - 1 and CY[i] == 1:
                self.ye[p, by, 1, CX[i] + 1, x] = fstar[i]

    def publish_all(self, state, parity):
        """What the initial state's tiles publish (the library fills the edge
        buffers of parity 0 at creation)."""
        for by in range(self.nty):
            for bx in range(self.ntx):
                x0, y0, x1, y1 = self.tile(bx, by)
                for y in range(y0, y1):
                    for x in range(x0, x1):
                        self.publish(state[:, y, x], x, y, bx, by, parity)

    def incoming(self, x, y, bx, by, parity):
        x0, y0, x1, y1 = self.tile(bx, by)
        p = 0 if self.single_buffer else parity
        f = np.empty(9)
        for i in range(9):
            s = source(x, y, i, self.nx, self.ny, self.periodic_y)
            if s is None or self.solid[s[1], s[0]]:
                f[i] = self.lat[self.slot(OPP[i]), y, x]
                continue
            sx, sy = s
            if x0 <= sx < x1 and y0 <= sy < y1:
                f[i] = self.lat[self.slot(i), sy, sx]
            elif not y0 <= sy < y1:  # across the bottom / top side, corners included
                f[i] = self.ye[p, sy // self.ty, 1 if CY[i] > 0 else 0, CX[i] + 1, sx]
            else:
                f[i] = self.xe[p, sx // self.tx, 1 if CX[i] > 0 else 0, CY[i] + 1, sy]
        return f

    def nodes(self, bx, by):
        x0, y0, x1, y1 = self.tile(bx, by)
        return [(x, y) for y in range(y0, y1) for x in range(x0, x1) if not self.solid[y, x]]

    def read_phase(self, bx, by, t):
        return {xy: self.incoming(xy[0], xy[1], bx, by, t % 2) for xy in self.nodes(bx, by)}

    def write_phase(self, bx, by, t, got):
        for (x, y), f in got.items():
            fstar = collide(f, self.m)
            for i in range(9):
                self.lat[self.slot(i), y, x] = fstar[i]
            self.publish(fstar, x, y, bx, by, (t + 1) % 2)

    def run(self, steps, rng):
        for t in range(steps):
            tiles = [(bx, by) for by in range(self.nty) for bx in range(self.ntx)]
            if self.no_barrier:  # each node reads and writes before the next node reads
                for k in rng.permutation(len(tiles)):
                    bx, by = tiles[k]
                    for x, y in self.nodes(bx, by):
                        self.write_phase(bx, by, t, {(x, y): self.incoming(x, y, bx, by, t % 2)})
                continue
            # a random interleaving of the phases: each tile's read phase
            # precedes its write phase, nothing else is ordered
            pending = [[tiles[k], "read"] for k in rng.permutation(len(tiles))]
            got = {}
            while pending:
                j = int(rng.integers(len(pending)))
                (bx, by), phase = pending[j]
                if phase == "read":
                    got[(bx, by)] = self.read_phase(bx, by, t)
                    pending[j][1] = "write"
                else:
                    self.write_phase(bx, by, t, got.pop((bx, by)))
                    pending.pop(j)

    def state(self):
        out = np.empty_like(self.lat)
        for i in range(9):
            out[i] = self.lat[self.slot(i)]
        return out


def case(nx, ny, p_solid, seed):
    rng = np.random.default_rng(seed)
    solid = rng.random((ny, nx)) < p_solid
    state = rng.standard_normal((9, ny, nx)) * 0.01
    state[:, solid] = 0.0
    return state, solid


CASES = [
    # nx, ny, tile, periodic_y, solid fraction
    (19, 11, (8, 4), True, 0.15),   # ragged tiles on both axes, periodic wrap through a ragged tile
    (16, 12, (4, 4), False, 0.2),   # closed bottom / top sides
    (13, 9, (1, 3), True, 0.1),     # one-column tiles: every node on both x sides
    (10, 7, (10, 7), True, 0.1),    # one tile: every source across a side wraps into itself
]


@pytest.mark.parametrize("swap", [False, True], ids=["npol", "nsol"])
@pytest.mark.parametrize("nx,ny,tile,periodic_y,p_solid", CASES)
def test_random_schedules_equal_two_lattice_pull(nx, ny, tile, periodic_y, p_solid, swap):
    m = mixing()
    state, solid = case(nx, ny, p_solid, seed=nx * 31 + ny)
    steps = 6
    ref = reference(state, solid, steps, m, periodic_y)
    for sched in range(6):
        sim = OneLattice(state, solid, tile[0], tile[1], m, periodic_y, swap)
        sim.run(steps, np.random.default_rng(1000 + sched))
        got = sim.state()
        fluid = ~solid
        assert np.array_equal(got[:, fluid], ref[:, fluid]), (sched, np.nanmax(np.abs(got - ref)))


@pytest.mark.parametrize("fault", ["single_buffer", "no_barrier"])
def test_planted_schedule_faults_are_seen(fault):
    m = mixing()
    nx, ny, tile = 19, 11, (8, 4)
    state, solid = case(nx, ny, 0.15, seed=7)
    steps = 4
    ref = reference(state, solid, steps, m, True)
    differs = False
    for sched in range(6):
        sim = OneLattice(state, solid, tile[0], tile[1], m, True, swap=False, **{fault: True})
        sim.run(steps, np.random.default_rng(2000 + sched))
        got = sim.state()
        if not np.array_equal(got[:, ~solid], ref[:, ~solid]):
            differs = True
            break
    assert differs, f"{fault}: no schedule exposed the planted mistake"
