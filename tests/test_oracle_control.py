"""Pins of the oracle's runtime control (CPU): a held signal phase stops the
other group's approaches until released; a lowered speed limit brings free
traffic down to it."""
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
