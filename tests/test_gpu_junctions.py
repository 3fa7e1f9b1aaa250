"""Junction internal lanes on the GPU against the oracle.

The hand-built junction states of tests/test_oracle_junctions.py (yielding
to an approaching vehicle or an occupied connector, not yielding, the lane
change toward the lanes that continue a route, a vehicle taken through the
junction from a lane that does not continue its route, the way through a
connector) are compared after every step: state bit for bit, decisions,
neighbours, flags (32: lane does not continue the route, 64: yield) and
margins.  Then whole runs with the map builder's connectors: the
intersection workload for the full hour, the 10x10 grid workload, and a
city network, state and counters bit for bit at several steps.
"""
import sys

import numpy as np
import pytest

import test_oracle_junctions as TJ
from paper_2405_12520_amd import junctions as J
from paper_2405_12520_amd import scenarios as S
from test_gpu_parity import compare_debug, compare_state, sim_cls  # noqa: F401

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _cases():
    opp_lane = int(TJ._left_turner().road_lane0[TJ.S_IN])
    yield "yield_approach", TJ._left_turner([dict(id=2, route=[TJ.S_IN, TJ.N_OUT], lane=opp_lane,
                                                   s=470.0, v=10.0)]), 4
    yield "no_yield_far", TJ._left_turner([dict(id=2, route=[TJ.S_IN, TJ.N_OUT], lane=opp_lane,
                                                 s=400.0, v=10.0)]), 4
    yield "no_yield_standing", TJ._left_turner([dict(id=2, route=[TJ.S_IN, TJ.N_OUT],
                                                      lane=opp_lane, s=495.0, v=0.0)]), 4
    yield "wrong_lane_change", TJ._state([dict(id=1, route=[TJ.N_IN, TJ.E_OUT], lane=1, s=300.0,
                                               v=10.0)], params=dict(p_lc=1.0)), 3
    yield "wrong_lane_forced", TJ._state([dict(id=1, route=[TJ.N_IN, TJ.E_OUT], lane=1, s=495.0,
                                               v=10.0)], params=dict(p_lc=0.0)), 4
    yield "through_connector", TJ._state([dict(id=1, route=[TJ.N_IN, TJ.E_OUT], lane=0, s=470.0,
                                               v=12.0)]), 12
    # a right turn: the one-lane connector ends on the out-road's right lane
    yield "right_turn_exit", TJ._state([dict(id=1, route=[TJ.N_IN, TJ.W_OUT], lane=1, s=470.0,
                                             v=10.0)]), 10
    for t0 in (0, 1):
        vs = [dict(id=1, route=[TJ.N_IN, TJ.E_OUT], lane=lane, s=300.0, v=10.0)
              for lane in (0,)] + [dict(id=2, route=[TJ.N_IN, TJ.E_OUT], lane=0, s=330.0, v=4.0)]
        yield f"bias_t{t0}", J.with_junction_lanes(TJ._state_plain(vs, t0=t0, p_lc=1.0)), 3


CASES = list(_cases())


@pytest.mark.parametrize("name,sc,steps", CASES, ids=[c[0] for c in CASES])
def test_junction_case(sim_cls, name, sc, steps):  # noqa: F811
    from oracle import OracleSim
    _say("junction case", name)
    g = sim_cls(sc, debug=True)
    o = OracleSim(sc)
    for t in range(steps):
        g.step(1)
        o.step(1)
        assert compare_state(g.state(), o.state(), f"{name} t={t}") == 0
        da, db = g.debug(), o.debug()
        compare_debug(da, db, f"{name} t={t}")
        assert np.array_equal(da["flags"], db["flags"]), (name, t, da["flags"], db["flags"])
        assert np.array_equal(da["margin"].view(np.uint32), db["margin"].view(np.uint32))
    cg, _, err = g.counters()
    co, _ = o.counters()
    assert err == 0 and np.array_equal(cg, co), (name, cg, co)
    g.close()


def _run_pair(sim_cls, sc, stops, name, launch=None):
    from oracle import OracleSim, max_threads
    g = sim_cls(sc)
    if launch:
        g.set_launch(**launch)
    o = OracleSim(sc)
    o.set_threads(max_threads())
    t = 0
    for stop in stops:
        g.step(stop - t)
        o.step(stop - t)
        t = stop
        where = f"{name} t={t}"
        assert compare_state(g.state(), o.state(), where) == 0, where
        cg, svg, err = g.counters()
        co, svo = o.counters()
        assert err == 0
        assert np.array_equal(cg, co), (where, cg, co)
        np.testing.assert_array_equal(svg, svo)
        _say(f"{where}: {o.n_active} active, {int(co[0, 2])} arrived")
    g.close()
    return co


def test_intersection_with_junction_lanes_full_hour(sim_cls):  # noqa: F811
    sc = J.with_junction_lanes(S.intersection())
    _say("intersection with junction lanes", sc.meta["junction_lanes"]["connectors"])
    co = _run_pair(sim_cls, sc, (50, 300, 600, 3600), "intersection+jl")
    assert co[0, 2] == sc.n_veh                      # everybody arrives


def test_grid_with_junction_lanes(sim_cls):  # noqa: F811
    sc = J.with_junction_lanes(S.grid(10, 20000, horizon=3600))
    _say("grid with junction lanes", sc.summary())
    co = _run_pair(sim_cls, sc, (100, 600, 1800, 3600), "grid+jl", launch=dict(xcd_remap=1))
    assert co[0, 2] > 15000


@pytest.mark.timeout(900)
def test_city_with_junction_lanes(sim_cls):  # noqa: F811
    """The city network (200 x 200 lattice) with connectors in every junction
    its vehicles cross: 200k vehicles pre-placed on 16-road walks."""
    sc = J.with_junction_lanes(S.city_snapshot(200_000, hops=16))
    _say("city with junction lanes", sc.summary(), sc.meta["junction_lanes"]["connectors"])
    _run_pair(sim_cls, sc, (20, 60, 150), "city+jl", launch=dict(xcd_remap=1))


def test_dynamic_lane_parity(sim_cls):  # noqa: F811
    """The same movement taken away from and given back to a lane on both
    sides; states, decisions and flags after every step."""
    from oracle import OracleSim
    sc = TJ.dynamic_lane_case().with_params(p_lc=0.5)
    straight = TJ._conn(sc, TJ.N_IN, TJ.S_OUT)
    l1 = TJ._lane(sc, TJ.N_IN, 1)
    g = sim_cls(sc, debug=True)
    o = OracleSim(sc)
    for t, allowed in enumerate([0, 0, 1, 0, 1, 1]):
        g.set_lane_turns([l1], [straight], [allowed])
        o.set_lane_turns([l1], [straight], [allowed])
        g.step(1)
        o.step(1)
        assert compare_state(g.state(), o.state(), f"dynamic t={t}") == 0
        da, db = g.debug(), o.debug()
        compare_debug(da, db, f"dynamic t={t}")
        assert np.array_equal(da["flags"], db["flags"]), (t, da["flags"], db["flags"])
    from paper_2405_12520_amd.moss import MossError
    with pytest.raises(MossError):
        g.set_lane_turns([TJ._lane(sc, TJ.N_IN, 1)], [TJ._conn(sc, TJ.N_IN, TJ.E_OUT)], [1])
    g.close()
