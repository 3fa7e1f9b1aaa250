"""Pins of the oracle's road and position outputs (CPU).

Positions: worked examples on roads whose geometry fixes the answer by hand,
then geometric invariants on a grid run.  Road measures: counts and mean
speeds recomputed from the state rows.
"""
import math

import numpy as np

from paper_2405_12520_amd import scenarios as S


def _two_roads():
    """Road 0: (0,0) -> (100,0), 2 lanes, length 100 (eastbound).
    Road 1: (100,0) -> (100,200), 1 lane, length 100: the drawn segment is
    twice the road length, so positions scale by 2 along it (northbound)."""
    net = dict(node_x=np.array([0.0, 100.0, 100.0]), node_y=np.array([0.0, 0.0, 200.0]),
               road_from=np.array([0, 1]), road_to=np.array([1, 2]),
               road_length=np.array([100.0, 100.0], np.float32),
               road_nlanes=np.array([2, 1], np.int32),
               road_vlim=np.full(2, 16.67, np.float32), node_cycle=np.zeros(3, np.int32),
               node_phase=np.zeros(3, np.int32), node_offset=np.zeros(3, np.int32),
               road_group=np.full(2, -1, np.int8))
    vehicles = [dict(id=1, route=[0, 1], lane=1, s=25.0, v=0.0),      # road 0, k = 1
                dict(id=2, route=[0, 1], lane=0, s=60.0, v=0.0),      # road 0, k = 0
                dict(id=3, route=[1], lane=2, s=50.0, v=0.0)]         # road 1, k = 0
    return S.with_vehicles("two_roads", net, vehicles)


def test_positions_worked_example():
    from oracle import OracleSim
    o = OracleSim(_two_roads())
    st = o.state()
    x, y, h = o.positions()
    got = {int(i): (x[k], y[k], h[k]) for k, i in enumerate(st["id"])}
    # eastbound: right of travel is -y; lane k is (k + 1/2) * 3.5 m out
    assert got[1] == (25.0, -5.25, 0.0)
    assert got[2] == (60.0, -1.75, 0.0)
    # northbound: right of travel is +x; s = 50 of 100 is half the drawn 200 m
    xb, yb, hb = got[3]
    assert (xb, yb) == (101.75, 100.0)
    assert abs(hb - math.pi / 2) < 1e-15


def _grid_run(steps=150):
    from oracle import OracleSim
    sc = S.grid(6, 2500, horizon=300)
    o = OracleSim(sc)
    o.step(steps)
    return sc, o


def test_road_stats_equal_state_rows():
    sc, o = _grid_run()
    st = o.state()
    cnt, mv = o.road_stats()
    lane_road = np.repeat(np.arange(sc.n_roads), sc.road_nlanes)
    r = lane_road[st["lane"]]
    assert cnt.sum() == st["id"].shape[0] > 100
    np.testing.assert_array_equal(cnt, np.bincount(r, minlength=sc.n_roads))
    sums = np.bincount(r, weights=st["v"].astype(np.float64), minlength=sc.n_roads)
    exp = np.where(cnt > 0, sums / np.maximum(cnt, 1), 0.0)
    np.testing.assert_allclose(mv, exp, rtol=1e-6, atol=1e-6)


def test_position_invariants_on_grid():
    """Each vehicle lies (k + 1/2) * 3.5 m to the right of its road's line,
    at the fraction s / L of the drawn segment, heading along it; vehicles of
    one lane are ordered along the heading as their positions s are."""
    sc, o = _grid_run()
    st = o.state()
    x, y, h = o.positions()
    lane_road = np.repeat(np.arange(sc.n_roads), sc.road_nlanes)
    r = lane_road[st["lane"]]
    k = st["lane"] - sc.road_lane0[r]
    ax, ay = sc.node_x[sc.road_from[r]], sc.node_y[sc.road_from[r]]
    bx, by = sc.node_x[sc.road_to[r]], sc.node_y[sc.road_to[r]]
    dx, dy = bx - ax, by - ay
    seg = np.hypot(dx, dy)
    # signed distance to the right of the directed line A->B (cross product)
    right = ((x - ax) * dy - (y - ay) * dx) / seg
    np.testing.assert_allclose(right, (k + 0.5) * 3.5, atol=1e-9)
    along = ((x - ax) * dx + (y - ay) * dy) / seg
    np.testing.assert_allclose(along, st["s"].astype(np.float64) / sc.road_length[r] * seg,
                               atol=1e-9)
    np.testing.assert_allclose(np.cos(h), dx / seg, atol=1e-12)
    np.testing.assert_allclose(np.sin(h), dy / seg, atol=1e-12)
    same = st["lane"][1:] == st["lane"][:-1]
    proj = along
    assert np.all(proj[1:][same] >= proj[:-1][same])
