"""Pins of the oracle's runtime control (CPU): a held signal phase stops the
other group's approaches until released; a lowered speed limit brings free
traffic down to it; a closed lane admits no vehicle (hand-built toy states
from tests/rule_cases.py with hand-computed outcomes)."""
import numpy as np
import pytest

from paper_2405_12520_amd import scenarios as S


def _first_road(sc):
    return sc.route_roads[sc.route_off[:-1]]


def _road_of_lane(sc):
    return np.repeat(np.arange(sc.n_roads), sc.road_nlanes)


@pytest.mark.parametrize("held, stopped", [(0, (2, 6)), (1, (0, 4))])
def test_held_phase_stops_the_other_group(held, stopped):
    """Intersection (N/S approaches = group 0): holding one phase keeps every
    vehicle that entered on an approach of the other group on that approach;
    releasing the node to its fixed-time plan lets them through."""
    from oracle import OracleSim
    sc = S.intersection()
    o = OracleSim(sc)
    o.set_signal_phase([0], [held])
    origin = dict(zip(sc.veh_id.tolist(), _first_road(sc).tolist()))
    road = _road_of_lane(sc)
    seen = 0
    for _ in range(10):
        o.step(60)
        st = o.state()
        for i, l in zip(st["id"].tolist(), st["lane"].tolist()):
            if origin[i] in stopped:
                seen += 1
                assert road[l] == origin[i], (i, road[l])
    assert seen > 0
    arrived_held = o.counters()[0][0, 2]
    o.set_signal_phase([0], [-1])
    o.step(600)
    st = o.state()
    crossed = [i for i, l in zip(st["id"].tolist(), st["lane"].tolist())
               if origin[i] in stopped and road[l] != origin[i]]
    assert o.counters()[0][0, 2] > arrived_held or crossed


def test_signal_control_rejects_unsignalised_nodes():
    from oracle import OracleSim
    o = OracleSim(S.intersection())
    with pytest.raises(ValueError):
        o.set_signal_phase([1], [0])


def test_lowered_speed_limit_is_reached_from_above():
    from oracle import OracleSim
    net = S.corridor([3000.0], 1, vlim=16.67)
    vehicles = [dict(id=k, route=[0], lane=0, s=200.0 * k, v=14.0, v0=14.0) for k in range(10)]
    sc = S.with_vehicles("free", net, vehicles)
    o = OracleSim(sc)
    o.step(20)
    v = o.state()["v"]
    assert v.min() > 13.0
    o.set_lane_vlim([0], [8.0])
    o.step(1)
    assert o.state()["v"].max() < v.max()            # braking from the next step on
    o.step(40)
    v = o.state()["v"]
    assert v.max() <= 8.0 + 1e-3 and v.min() > 7.9


# ------------------------------------------------------ lane restriction --

def _lane_after(sc, closed, steps):
    from oracle import OracleSim
    o = OracleSim(sc)
    if closed:
        o.set_lane_closed(closed, [1] * len(closed))
    o.step(steps)
    st = o.state()
    return o, st


@pytest.mark.parametrize("k, closed, lane", [(2, [], 5), (2, [5], 4), (2, [4, 5], 3),
                                             (1, [4], 3), (0, [3], 4)])
def test_transfer_takes_the_nearest_open_lane(k, closed, lane):
    """Road 1 has lanes 3, 4, 5.  From lane index k the vehicle enters
    min(k, 2); if that lane is closed, the nearest open one, the lower of two
    equally near."""
    import rule_cases as RC
    _, st = _lane_after(RC.transfer_into(k), closed, 1)
    assert st["lane"].tolist() == [lane]
    assert st["s"].tolist() == [20.0]


def test_no_lane_change_into_a_closed_lane():
    import rule_cases as RC
    o, st = _lane_after(RC.slow_leader_change(), [], 1)
    assert dict(zip(st["id"].tolist(), st["lane"].tolist()))[1] == 0
    o, st = _lane_after(RC.slow_leader_change(), [0], 1)
    assert dict(zip(st["id"].tolist(), st["lane"].tolist()))[1] == 1
    assert (o.debug()["flags"] & 3).tolist() == [0, 0]      # not even evaluated


def test_lookahead_follows_the_open_lane():
    import rule_cases as RC
    from oracle import OracleSim
    for closed, leader in (([], 0xFFFFFFFF), ([3], 2)):
        o = OracleSim(RC.lookahead_into(bool(closed)))
        if closed:
            o.set_lane_closed(closed, [1])
        o.step(1)
        d = o.debug()
        lead = dict(zip(d["id"].tolist(), d["leader"].tolist()))
        assert lead[1] == leader


def test_closed_lane_holds_its_departure_queue():
    import rule_cases as RC
    from oracle import OracleSim
    o = OracleSim(RC.two_lane_insertion())
    o.set_lane_closed([1], [1])
    o.step(3)
    c, _ = o.counters()
    assert o.n_active == 0 and c[0, 0] == 0 and c[0, 1] == 3
    o.set_lane_closed([1], [0])
    o.step(1)
    assert o.n_active == 1 and o.counters()[0][0, 0] == 1


def test_closing_the_last_open_lane_is_refused():
    import rule_cases as RC
    from oracle import OracleSim
    o = OracleSim(RC.slow_leader_change())
    o.set_lane_closed([0], [1])
    with pytest.raises(ValueError):
        o.set_lane_closed([1], [1])                          # road 0 would have none
    with pytest.raises(ValueError):
        o.set_lane_closed([0, 1], [1, 1])
    o.set_lane_closed([1, 0], [1, 0])                        # judged as a whole: one open
    with pytest.raises(ValueError):
        o.set_lane_closed([99], [1])
