"""The diagnostics entry point that allocates nothing (lbm_diag_noalloc)
against lbm_diag, through the C ABI.

lbm_diag_noalloc enqueues the same FP64 reductions as lbm_diag with its
reduction partials in a fixed device array of the library; the caller
passes the previous-velocity buffer (device, 2 doubles per node) and a device
output of 4 doubles.  Checks: two calls in a row on one simulation (the second
with a residual against the first), then a call on a smaller grid; mass and
momentum bitwise equal to lbm_diag's (the same kernels in the same order),
the residual equal to lbm_diag's over the same pair of states.
"""
import ctypes

import numpy as np
import pytest

from paper_2607_20650_amd import workloads as W

pytestmark = pytest.mark.gpu


def _noalloc(sim, u_prev, have_prev, out):
    torch = pytest.importorskip("torch")
    st = sim._lib.lbm_diag_noalloc(sim._ctx, ctypes.c_void_p(u_prev.data_ptr() if u_prev is not None else 0),
                                   int(have_prev), ctypes.c_void_p(out.data_ptr()))
    assert st == 0, sim._lib.lbm_last_error(sim._ctx).decode()
    sim.sync()
    return out.cpu().numpy().tolist()


def test_diag_noalloc_matches_diag_two_calls_then_smaller_grid():
    import torch

    from paper_2607_20650_amd.lbm import OK, Simulation
    big = W.karman(nx=320, ny=96, cx=80, cy=48, radius=8, u_in=0.05, tau=0.6)
    small = W.karman(nx=96, ny=40, cx=24, cy=20, radius=4, u_in=0.04, tau=0.7)
    for sc, scheme, layout in ((big, "NPTL", "stream"), (small, "AA", "collision")):
        with Simulation.from_scenario(sc, scheme=scheme, layout=layout) as sim:
            n = sc.nx * sc.ny
            with torch.cuda.stream(sim.stream):
                u_prev = torch.zeros(2 * n, dtype=torch.float64, device="cuda")
                out = torch.full((4,), -7.0, dtype=torch.float64, device="cuda")
            sim.step(60)
            s1, d1 = sim.diag()
            assert s1 == OK and d1[3] == -1.0
            o1 = _noalloc(sim, u_prev, 0, out)
            assert o1[:3] == d1[:3], (o1, d1)  # same kernels, same order: bitwise
            assert o1[3] == -1.0
            sim.step(25)
            s2, d2 = sim.diag()
            o2 = _noalloc(sim, u_prev, 1, out)
            assert s2 == OK and o2[:3] == d2[:3], (o2, d2)
            assert d2[3] > 0 and abs(o2[3] - d2[3]) <= 1e-12 * d2[3], (o2[3], d2[3])
            # without a previous-velocity buffer: no residual
            o3 = _noalloc(sim, None, 0, out)
            assert o3[:3] == d2[:3] and o3[3] == -1.0
