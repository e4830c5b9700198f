"""GPU tests of the continuous-batching serving engine (lbm_server_*)."""
import numpy as np
import pytest

import oracle
from paper_2607_20650_amd import workloads as W
from tests.helpers import updated_mask, velocity_error

pytestmark = pytest.mark.gpu


def _requests():
    """Varied sizes, obstacles, tau and step counts (not multiples of the bundle)."""
    specs = [(64, 64, "cylinder", 0.6, 37), (130, 70, "square", 0.9, 120), (200, 96, "plate", 0.7, 77),
             (96, 150, "cylinder", 1.1, 5), (257, 64, "square", 0.55, 64), (70, 65, "plate", 0.8, 151)]
    return [W.obstacle_channel(nx, ny, kind, u_in=0.03, tau=tau, steps=steps) for nx, ny, kind, tau, steps in specs]


@pytest.mark.parametrize("layout,precision", [("stream", "fp32"), ("bundle", "fp16s"), ("collision", "fp32"),
                                              ("stream", "fp16sr"), ("bundle", "fp16csr")])
def test_each_result_same_alone_and_in_the_mix(layout, precision):
    from paper_2607_20650_amd.lbm import OK, Server, Simulation
    reqs = _requests()
    alone = []
    for sc in reqs:
        with Simulation.from_scenario(sc, scheme="NPTL", layout=layout, precision=precision) as sim:
            sim.step(sc.steps)
            alone.append(sim.macros())
    with Server(1 << 30, max_slots=4, bundle_steps=16, layout=layout, precision=precision) as srv:
        ids = {}
        # staggered submission: later requests arrive while earlier ones run
        for k, sc in enumerate(reqs):
            ids[srv.submit_scenario(sc)] = k
            srv.run_bundle()
        got = {}
        for _ in range(1000):
            srv.run_bundle()
            for rid, st in srv.poll():
                assert st == OK
                got[ids[rid]] = srv.fetch(rid)[1:]
            if len(got) == len(reqs):
                break
        st = srv.stats()
        assert st["pool_used"] == 0 and st["running"] == 0 and st["queued"] == 0
    assert len(got) == len(reqs)
    for k in range(len(reqs)):
        assert np.array_equal(got[k][0], alone[k][0]), k
        assert np.array_equal(got[k][1], alone[k][1]), k


def test_neumann_and_dirichlet_inlets_in_the_mix():
    """Requests with the Neumann inlet (its per-row densities live in the
    request's pool block) share bundles with Dirichlet ones: each result equals
    the request run alone, bitwise, and the oracle within 1e-5."""
    from paper_2607_20650_amd.lbm import OK, Server, Simulation
    kinds = [W.NEUMANN_PRESSURE, W.INFLOW_OUTFLOW, W.NEUMANN_OUTFLOW, W.INFLOW_PRESSURE]
    reqs = []
    for k, xa in enumerate(kinds):
        sc = W.obstacle_channel(96 + 40 * k, 64 + 8 * k, ("cylinder", "square", "plate", "cylinder")[k], u_in=0.04,
                                tau=0.6 + 0.1 * k, steps=41 + 13 * k)
        sc.x_axis = xa
        reqs.append(sc)
    alone = []
    for sc in reqs:
        with Simulation.from_scenario(sc, scheme="NPTL", layout="stream", precision="fp32") as sim:
            sim.step(sc.steps)
            alone.append(sim.macros())
    with Server(1 << 28, max_slots=3, bundle_steps=16) as srv:
        ids = {}
        for k, sc in enumerate(reqs):
            ids[srv.submit_scenario(sc)] = k
            srv.run_bundle()
        got = {}
        for _ in range(1000):
            srv.run_bundle()
            for rid, st in srv.poll():
                assert st == OK
                got[ids[rid]] = srv.fetch(rid)[1:]
            if len(got) == len(reqs):
                break
        assert srv.stats()["pool_used"] == 0
    for k, sc in enumerate(reqs):
        assert np.array_equal(got[k][0], alone[k][0]), k
        assert np.array_equal(got[k][1], alone[k][1]), k
        ref = oracle.Oracle.from_scenario(sc).run(sc.steps)
        rho_ref, ux, uy = ref.macros()
        assert velocity_error(got[k][1], ux, uy, updated_mask(ref.types)) <= 1e-5, k
        inlet = ref.types == oracle.INLET
        assert np.abs(got[k][0][inlet] - rho_ref[inlet]).max() < 1e-6, k


def test_admission_by_footprint_and_parity():
    """A budget that holds about two requests: the others wait in the queue,
    everything finishes, memory returns to the pool, results match the oracle."""
    from paper_2607_20650_amd.lbm import OK, Server
    reqs = [W.obstacle_channel(256, 128, "cylinder", u_in=0.03, tau=0.7, steps=60 + 10 * k) for k in range(5)]
    foot = 2 * 9 * 4 * 256 * 128 + 2 * 256 * 128 + 4096
    with Server(int(2.5 * foot), max_slots=8, bundle_steps=20) as srv:
        ids = [srv.submit_scenario(sc) for sc in reqs]
        srv.run_bundle()
        s = srv.stats()
        assert s["running"] == 2 and s["queued"] == 3
        res = {}
        for _ in range(1000):
            srv.run_bundle()
            for rid, st in srv.poll():
                res[rid] = srv.fetch(rid)
            if len(res) == len(ids):
                break
        assert srv.stats()["pool_used"] == 0
    for rid, sc in zip(ids, reqs):
        st, rho, u = res[rid]
        assert st == OK
        ref = oracle.Oracle.from_scenario(sc).run(sc.steps)
        _, ux, uy = ref.macros()
        assert velocity_error(u, ux, uy, updated_mask(ref.types)) <= 1e-5


def test_oversized_request_rejected_without_leak():
    from paper_2607_20650_amd.lbm import ENOMEM, LbmError, Server
    with Server(4 << 20, max_slots=2) as srv:
        big = W.obstacle_channel(1024, 512, "cylinder")
        with pytest.raises(LbmError) as e:
            srv.submit_scenario(big, steps=10)
        assert e.value.status == ENOMEM
        small = W.obstacle_channel(64, 64, "plate", steps=3)
        rid = srv.submit_scenario(small)
        zero = srv.submit_scenario(small, steps=0)
        done = {}
        for _ in range(100):
            srv.run_bundle()
            for r, st in srv.poll():
                done[r] = srv.fetch(r)[0]
            if len(done) == 2:
                break
        assert set(done) == {rid, zero}
        assert srv.stats()["pool_used"] == 0
