"""Runtime control on the GPU vs the oracle: the same signal phases, speed
limits and lane closures given to both between steps leave identical states
(bit for bit), on a grid under max-pressure control, under random
speed-limit changes and under random lane closures, and on the hand-built
lane-restriction states of tests/rule_cases.py (decisions and neighbours
compared every step)."""
import sys

import numpy as np
import pytest

import rule_cases as RC
from paper_2405_12520_amd import scenarios as S

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sim_cls():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_12520_amd.moss import Simulator
    return Simulator


def _same(g, o, where):
    a, b = g.state(), o.state()
    for f in ("id", "lane", "cursor"):
        assert np.array_equal(a[f], b[f]), (where, f)
    for f in ("s", "v", "a"):
        assert np.array_equal(a[f].view(np.uint32), b[f].view(np.uint32)), (where, f)


def test_max_pressure_control_parity(sim_cls):
    from oracle import OracleSim
    from paper_2405_12520_amd.control import MaxPressure
    sc = S.grid(10, 12000, horizon=900)
    _say("max pressure")
    g = sim_cls(sc)
    o = OracleSim(sc)
    ctl = MaxPressure(sc, period=10)
    switched = 0
    for k in range(60):
        before = ctl.phase.copy()
        ctl.run(g, 10, also=o)
        switched += int((ctl.phase != before).sum())
        if k % 6 == 5:
            _same(g, o, f"t={10 * (k + 1)}")
    _same(g, o, "end")
    assert switched > 0
    g.close()


def test_speed_limit_changes_parity(sim_cls):
    from oracle import OracleSim
    sc = S.grid(10, 8000, horizon=600)
    _say("speed limits")
    g = sim_cls(sc)
    o = OracleSim(sc)
    rng = np.random.default_rng(3)
    for k in range(8):
        lanes = rng.choice(sc.n_lanes, 200, replace=False).astype(np.int32)
        vl = rng.choice([5.0, 8.33, 11.11, 16.67], 200).astype(np.float32)
        g.set_lane_vlim(lanes, vl)
        o.set_lane_vlim(lanes, vl)
        g.step(40)
        o.step(40)
        _same(g, o, f"t={40 * (k + 1)}")
    g.close()


def test_control_rejects_bad_arguments(sim_cls):
    from paper_2405_12520_amd.moss import MossError
    sc = S.intersection()
    g = sim_cls(sc)
    g.step(100)
    st = g.state()
    with pytest.raises(MossError):
        g.set_signal_phase([1], [0])          # node 1 has no signal
    with pytest.raises(MossError):
        g.set_signal_phase([0], [-2])
    with pytest.raises(MossError):
        g.set_lane_vlim([sc.n_lanes], [10.0])
    with pytest.raises(MossError):
        g.set_lane_vlim([0], [0.0])
    st2 = g.state()
    for f in st:
        assert np.array_equal(st[f], st2[f])
    g.close()


def test_lane_closures_parity(sim_cls):
    """Random closures and reopenings on the 10x10 grid (three-lane roads),
    a road's lanes never all closed; departures, transfers and lane changes
    run into them for 480 steps."""
    from oracle import OracleSim
    sc = S.grid(10, 12000, horizon=600)
    _say("lane closures")
    g = sim_cls(sc)
    o = OracleSim(sc)
    rng = np.random.default_rng(5)
    road = np.repeat(np.arange(sc.n_roads), sc.road_nlanes)
    closed = np.zeros(sc.n_lanes, bool)
    for k in range(12):
        lanes = rng.choice(sc.n_lanes, 150, replace=False).astype(np.int32)
        want = rng.random(150) < 0.7
        for l, w in zip(lanes, want):
            r = road[l]
            l0 = sc.road_lane0[r]
            others = closed[l0:l0 + sc.road_nlanes[r]].sum() - closed[l]
            closed[l] = bool(w) and others < sc.road_nlanes[r] - 1
        flags = closed[lanes].astype(np.int32)
        g.set_lane_closed(lanes, flags)
        o.set_lane_closed(lanes, flags)
        g.step(40)
        o.step(40)
        _same(g, o, f"closures t={40 * (k + 1)}")
        cg, _, err = g.counters()
        co, _ = o.counters()
        assert err == 0 and np.array_equal(cg, co)
    assert closed.sum() > 100
    g.close()


CLOSURES = RC.closure_cases()


@pytest.mark.parametrize("name,sc,closed,steps", CLOSURES, ids=[c[0] for c in CLOSURES])
def test_lane_closure_case(sim_cls, name, sc, closed, steps):
    from oracle import OracleSim
    from test_gpu_parity import compare_debug
    _say("closure case", name)
    g = sim_cls(sc, debug=True)
    o = OracleSim(sc)
    if closed:
        g.set_lane_closed(closed, [1] * len(closed))
        o.set_lane_closed(closed, [1] * len(closed))
    for t in range(steps):
        g.step(1)
        o.step(1)
        _same(g, o, f"{name} t={t}")
        da, db = g.debug(), o.debug()
        compare_debug(da, db, f"{name} t={t}")
        assert np.array_equal(da["flags"], db["flags"]), (name, t)
    cg, _, err = g.counters()
    co, _ = o.counters()
    assert err == 0 and np.array_equal(cg, co), (name, cg, co)
    g.close()


def test_lane_closure_rejects_bad_batches(sim_cls):
    from paper_2405_12520_amd.moss import MossError
    g = sim_cls(RC.slow_leader_change())
    g.set_lane_closed([0], [1])
    with pytest.raises(MossError):
        g.set_lane_closed([1], [1])                 # road 0 would have no open lane
    with pytest.raises(MossError):
        g.set_lane_closed([0, 1], [1, 1])
    with pytest.raises(MossError):
        g.set_lane_closed([99], [1])
    g.set_lane_closed([1, 0], [1, 0])               # judged as a whole: one stays open
    from oracle import OracleSim
    o = OracleSim(RC.slow_leader_change())
    o.set_lane_closed([1], [1])
    g.step(2)
    o.step(2)
    _same(g, o, "after the refused batches")
    assert g.state()["lane"].tolist() == [0, 0]     # both moved out of the closed lane 1
    g.close()
