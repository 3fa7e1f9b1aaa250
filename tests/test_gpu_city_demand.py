"""The city with its travel demand, GPU against the oracle over the whole
hour.

2,000,000 trips between 400 zones of the 40k-node city, drawn from a gravity
model (zone mass = node count, deterrence exp(-d / 3 km)), departing at
uniform steps over one hour and routed on shortest paths: the workload shape
of the paper's city-scale runs (Sec. IV-A: real city maps with their demand,
3600 one-second steps), here synthetic.  Vehicles enter through the departure
queues, move, change lanes, cross signalised junctions and arrive, so every
rule of the step runs at city scale.

The GPU runs in the benchmark's launch shape (captured 16-step graphs, XCD-
contiguous tiles).  The whole state (ids, lanes, route cursors, positions,
speeds, accelerations) and the counters equal the oracle's bit for bit at
steps 100, 200, 300 and at the end of the hour, and so does the number of
vehicles still waiting to depart; the macroscopic outputs (mean speed over the run, trips,
mean trip time) are then within 1 % by construction, and asserted.
"""
import sys

import numpy as np
import pytest

from paper_2405_12520_amd import scenarios as S
from test_gpu_parity import compare_state, sim_cls  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _macro(c, sv):
    """(mean speed over all vehicle-steps, trips, mean trip time)."""
    vs, arrived, ttime = int(c[:, 6].sum()), int(c[:, 2].sum()), int(c[:, 3].sum())
    return float(sv.sum()) / max(vs, 1), arrived, ttime / max(arrived, 1)


@pytest.mark.timeout(900)
def test_city_demand_hour(sim_cls):  # noqa: F811
    from oracle import OracleSim, max_threads
    sc = S.city_demand()
    _say(f"city demand: {sc.summary()}")
    g = sim_cls(sc)
    g.set_launch(xcd_remap=1)
    o = OracleSim(sc)
    o.set_threads(max_threads())
    t = 0
    for stop in (100, 200, 300, 3600):
        g.step(stop - t)
        o.step(stop - t)
        t = stop
        where = f"city demand t={t}"
        assert compare_state(g.state(), o.state(), where) == 0, where
        cg, svg, err = g.counters()
        co, svo = o.counters()
        assert err == 0
        assert np.array_equal(cg, co), (where, cg, co)
        np.testing.assert_array_equal(svg, svo)
        assert len(g.pending()) == o.pending, where
        _say(f"{where}: {o.n_active} active, {int(co[0, 2])} arrived, "
             f"{int(co[0, 1])} insert failures")
    mg, mo = _macro(cg, svg), _macro(co, svo)
    _say(f"macro GPU {mg} oracle {mo}")
    assert mo[1] > 0
    for x, y in zip(mg, mo):
        assert abs(x - y) <= 0.01 * abs(y)
    g.close()
