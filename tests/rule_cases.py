"""Hand-built toy states whose outcome follows from the model rules alone.

Each builder returns a Scenario (inputs only, no model arithmetic) and the
expected outcome is stated, computed by hand, in the test that uses it.  The
oracle pins (tests/test_oracle_rules.py) check the CPU oracle against those
hand-computed outcomes; the GPU parity tests run the same states through the
HIP library and compare with the oracle.

The numbers are chosen so that the arithmetic is exact in FP32 where a test
relies on a tie or a boundary: vehicles at their desired speed on a free road
have acceleration a_max (1 - 1) = 0 and move exactly v per 1 s step.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from paper_2405_12520_amd import scenarios as S


def insertion_behind_tail(s_tail: float, v_tail: float = 4.0, v0: float = 14.0,
                          lanes: int = 1) -> S.Scenario:
    """One vehicle already on a 500 m lane at s_tail (speed v_tail) and one
    vehicle due to enter the same lane at step 0 (desired speed v0, limit
    16.67 m/s).  Entry speed min(v0, limit, v_tail); the entry needs
    s_tail - len >= s0 + v_entry * T."""
    net = S.corridor([500.0, 100.0], lanes)
    vs = [dict(id=lanes, route=[0, 1], lane=0, s=s_tail, v=v_tail, v0=14.0),
          dict(id=2 * lanes, route=[0, 1], depart=0, v0=v0)]
    return S.with_vehicles("ins_gap", net, vs)


def empty_lane_insertion(v0: float = 20.0) -> S.Scenario:
    """A vehicle due at step 0 on an empty lane with limit 16.67 m/s."""
    net = S.corridor([500.0, 100.0], 1)
    return S.with_vehicles("ins_empty", net, [dict(id=1, route=[0, 1], depart=0, v0=v0)])


def red_approach(s: float, v: float = 15.0, route=(0, 1)) -> S.Scenario:
    """A vehicle on a 300 m road whose downstream junction never shows its
    group (permanently red), at position s with speed v."""
    net = S.corridor([300.0, 100.0], 1, signal=(1, 60, 60, 0, 1))
    return S.with_vehicles("red_approach", net,
                           [dict(id=1, route=list(route), lane=0, s=s, v=v, v0=14.0)])


def cut_in_behind(s_n: float, b_safe: float = 10.0) -> S.Scenario:
    """Even step on a two-lane road: vehicle 1 (lane 1, s = 200, v = 10) has a
    standing leader 20 m ahead; the target lane 0 holds only a standing
    vehicle 3 at s_n.  Politeness 0, p_lc = 1, b_safe as given."""
    net = S.corridor([1000.0, 100.0], 2)
    vs = [dict(id=1, route=[0, 1], lane=1, s=200.0, v=10.0),
          dict(id=2, route=[0, 1], lane=1, s=220.0, v=0.0, v0=0.5),
          dict(id=3, route=[0, 1], lane=0, s=s_n, v=0.0, v0=0.5)]
    return S.with_vehicles("cut_in", net, vs,
                           params=dict(t0=0, p_lc=1.0, politeness=0.0, b_safe=b_safe))


def limits_differ(vlim_target: float, vlim_own: float) -> S.Scenario:
    """Even step on a two-lane road: vehicle 1 (lane 1, s = 200, v = 10,
    v0 = 14) follows vehicle 2 (s = 265, v = 10) at a 60 m gap; the target
    lane 0 is empty.  Lane 0 has limit vlim_target, lane 1 vlim_own."""
    net = S.corridor([1000.0, 100.0], 2)
    vs = [dict(id=1, route=[0, 1], lane=1, s=200.0, v=10.0, v0=14.0),
          dict(id=2, route=[0, 1], lane=1, s=265.0, v=10.0, v0=14.0)]
    sc = S.with_vehicles("limits", net, vs, params=dict(t0=0, p_lc=1.0))
    vl = sc.lane_vlim.copy()
    vl[0], vl[1] = vlim_target, vlim_own
    return dataclasses.replace(sc, lane_vlim=vl.astype(np.float32))


def clamp_fast_follower() -> S.Scenario:
    """Vehicle 1 at 20 m/s one metre behind the rear of a standing vehicle 2
    (s = 100, v0 = 0.5) on a 1000 m single lane with limit 30 m/s."""
    net = S.corridor([1000.0, 100.0], 1, vlim=30.0)
    vs = [dict(id=1, route=[0, 1], lane=0, s=94.0, v=20.0, v0=20.0),
          dict(id=2, route=[0, 1], lane=0, s=100.0, v=0.0, v0=0.5)]
    return S.with_vehicles("clamp", net, vs)


def joiners_tie(id_lane0: int, id_lane1: int) -> S.Scenario:
    """Two vehicles side by side (s = 95, v = v0 = 25) on the two lanes of a
    100 m road that feeds a one-lane road; no lookahead (h_look = 0), so both
    are on a free road at their desired speed, move exactly 25 m and enter
    the next road at exactly s = 20."""
    net = S.corridor([100.0, 200.0], [2, 1], vlim=30.0)
    vs = [dict(id=id_lane0, route=[0, 1], lane=0, s=95.0, v=25.0, v0=25.0),
          dict(id=id_lane1, route=[0, 1], lane=1, s=95.0, v=25.0, v0=25.0)]
    return S.with_vehicles("join_tie", net, vs, params=dict(h_look=0))


def stayer_joiner_tie(id_stayer: int, id_joiner: int) -> S.Scenario:
    """A vehicle at s = 10 on a one-lane 200 m road (v = v0 = 10, last road of
    its route) and one at s = 95 on the 100 m road before it (v = v0 = 25);
    no lookahead.  Both are free at their desired speed: the first stays in
    its lane at s = 20, the second enters that lane at s = 20."""
    net = S.corridor([100.0, 200.0], 1, vlim=30.0)
    vs = [dict(id=id_stayer, route=[1], lane=1, s=10.0, v=10.0, v0=10.0),
          dict(id=id_joiner, route=[0, 1], lane=0, s=95.0, v=25.0, v0=25.0)]
    return S.with_vehicles("stay_join_tie", net, vs, params=dict(h_look=0))


def two_lane_insertion() -> S.Scenario:
    """A vehicle (id 1) due at step 0 on an empty two-lane road: it queues on
    lane 1 mod 2 = 1."""
    net = S.corridor([500.0, 100.0], 2)
    return S.with_vehicles("ins_two", net, [dict(id=1, route=[0, 1], depart=0, v0=14.0)])


def transfer_into(k: int) -> S.Scenario:
    """A vehicle on lane k of a 100 m three-lane road at s = 95, v = v0 = 25,
    no lookahead: free at its desired speed, it moves exactly 25 m and enters
    the next (three-lane, 200 m) road at s = 20, on lane index min(k, 2)
    unless control has closed that lane."""
    net = S.corridor([100.0, 200.0], 3, vlim=30.0)
    return S.with_vehicles("transfer", net,
                           [dict(id=1, route=[0, 1], lane=k, s=95.0, v=25.0, v0=25.0)],
                           params=dict(h_look=0))


def slow_leader_change() -> S.Scenario:
    """Even step on a two-lane road: vehicle 1 (lane 1, s = 200, v = 10)
    behind a standing vehicle 20 m ahead, target lane 0 empty; p_lc = 1.  The
    change is safe and worth it (IDM at a standing leader 15 m away brakes
    hard; the empty lane gives free acceleration)."""
    net = S.corridor([1000.0, 100.0], 2)
    vs = [dict(id=1, route=[0, 1], lane=1, s=200.0, v=10.0),
          dict(id=2, route=[0, 1], lane=1, s=220.0, v=0.0, v0=0.5)]
    return S.with_vehicles("slow_leader", net, vs, params=dict(t0=0, p_lc=1.0))


def lookahead_into(closed_k1: bool) -> S.Scenario:
    """Vehicle 1 on lane 1 of a two-lane 100 m road at s = 90 (v = 10); the
    next two-lane road holds one vehicle, vehicle 2, on lane 0 at s = 30.  The
    lookahead takes lane min(1, 1) = 1, which is empty (no leader), unless
    lane 1 is closed: then lane 0, whose last vehicle 2 leads at gap
    (100 - 90) + 30 - 5 = 35 m."""
    net = S.corridor([100.0, 300.0], 2, vlim=16.67)
    vs = [dict(id=1, route=[0, 1], lane=1, s=90.0, v=10.0),
          dict(id=2, route=[1], lane=2, s=30.0, v=5.0)]
    return S.with_vehicles("lookahead_closed" if closed_k1 else "lookahead_open", net, vs)


# lane restriction cases as (name, scenario, lanes closed before the first
# step, steps) for the GPU parity test
def closure_cases():
    return [
        ("transfer_open", transfer_into(2), [], 2),
        ("transfer_closed_2", transfer_into(2), [5], 2),
        ("transfer_closed_12", transfer_into(2), [4, 5], 2),
        ("transfer_tie", transfer_into(1), [4], 2),
        ("change_open", slow_leader_change(), [], 2),
        ("change_closed", slow_leader_change(), [0], 2),
        ("lookahead_open", lookahead_into(False), [], 2),
        ("lookahead_closed", lookahead_into(True), [3], 2),
        ("queue_closed", two_lane_insertion(), [1], 3),
    ]


def _two_lane(vs, vlim_lane0, vlim_lane1, **params):
    net = S.corridor([1000.0, 100.0], 2)
    sc = S.with_vehicles("two_lane", net, vs, params=dict(t0=0, **params))
    vl = sc.lane_vlim.copy()
    vl[0], vl[1] = vlim_lane0, vlim_lane1
    return dataclasses.replace(sc, lane_vlim=vl.astype(np.float32))


def level_in_target() -> S.Scenario:
    """Even step: vehicle 1 (lane 1, s = 200) and vehicle 3 level with it in
    the target lane 0 (s = 200); p_lc = 1."""
    return _two_lane([dict(id=1, route=[0, 1], lane=1, s=200.0, v=10.0, v0=14.0),
                      dict(id=3, route=[0, 1], lane=0, s=200.0, v=10.0, v0=14.0)],
                     16.67, 16.67, p_lc=1.0)


def old_follower_limits(vlim_target: float, with_follower: bool = True) -> S.Scenario:
    """Even step: vehicle 1 (lane 1, s = 200, v = 8, desired 8) with an old
    follower 2 (lane 1, s = 150, v = 9, desired 15); own lane limit 10 m/s,
    target lane 0 limit vlim_target."""
    vs = [dict(id=1, route=[0, 1], lane=1, s=200.0, v=8.0, v0=8.0)]
    if with_follower:
        vs.append(dict(id=2, route=[0, 1], lane=1, s=150.0, v=9.0, v0=15.0))
    return _two_lane(vs, vlim_target, 10.0)


def new_follower_limits(vlim_own: float, with_follower: bool = True) -> S.Scenario:
    """Even step: vehicle 1 (lane 1, s = 200, v = 8, desired 8) with a new
    follower 3 in the target lane 0 (s = 150, v = 9, desired 15); target lane
    limit 10 m/s, own lane limit vlim_own."""
    vs = [dict(id=1, route=[0, 1], lane=1, s=200.0, v=8.0, v0=8.0)]
    if with_follower:
        vs.append(dict(id=3, route=[0, 1], lane=0, s=150.0, v=9.0, v0=15.0))
    return _two_lane(vs, 10.0, vlim_own)


def entry_behind_two() -> S.Scenario:
    """A one-lane 500 m road holding vehicles at 6 m (v = 4) and 300 m
    (v = 10), and a vehicle due to enter it at step 0."""
    net = S.corridor([500.0, 100.0], 1)
    vs = [dict(id=1, route=[0, 1], lane=0, s=6.0, v=4.0, v0=14.0),
          dict(id=2, route=[0, 1], lane=0, s=300.0, v=10.0, v0=14.0),
          dict(id=3, route=[0, 1], depart=0, v0=14.0)]
    return S.with_vehicles("entry", net, vs)


def clamp_two_chains() -> S.Scenario:
    """One lane with two fast followers (v = 20) each 10 m behind a standing
    vehicle, 200 m apart: both followers overrun their leader in one step
    (braking at most b_max), so the lane has two overlapping pairs with a
    clean pair between them."""
    net = S.corridor([1000.0, 100.0], 1)
    vs = [dict(id=1, route=[0, 1], lane=0, s=85.0, v=20.0, v0=20.0),
          dict(id=2, route=[0, 1], lane=0, s=100.0, v=0.0, v0=0.5),
          dict(id=3, route=[0, 1], lane=0, s=285.0, v=20.0, v0=20.0),
          dict(id=4, route=[0, 1], lane=0, s=300.0, v=0.0, v0=0.5)]
    return S.with_vehicles("clamp_two", net, vs)


# every case above as (name, scenario, steps) for the GPU parity test
def all_cases():
    f32 = np.float32
    return [
        ("ins_exact", insertion_behind_tail(13.0), 3),
        ("ins_below", insertion_behind_tail(float(np.nextafter(f32(13.0), f32(0.0)))), 3),
        ("ins_slow_tail", insertion_behind_tail(100.0), 3),
        ("ins_fast_tail", insertion_behind_tail(100.0, v_tail=15.0), 3),
        ("ins_two_lanes", insertion_behind_tail(13.0, lanes=2), 3),
        ("ins_empty", empty_lane_insertion(), 3),
        ("red_cannot_stop", red_approach(290.0), 4),
        ("red_boundary", red_approach(287.5), 4),
        ("red_past_boundary", red_approach(float(np.nextafter(f32(287.5), f32(1e9)))), 4),
        ("red_last_road", red_approach(200.0, v=10.0, route=(0,)), 20),
        ("cut_in_gap0", cut_in_behind(195.0), 2),
        ("cut_in_gap1", cut_in_behind(194.0), 2),
        ("cut_in_at_b_safe", cut_in_behind(194.0, b_safe=6.0), 2),
        ("limit_low_target", limits_differ(8.0, 16.67), 2),
        ("limit_low_own", limits_differ(16.67, 8.0), 2),
        ("clamp", clamp_fast_follower(), 3),
        ("join_tie_12", joiners_tie(1, 2), 2),
        ("join_tie_21", joiners_tie(2, 1), 2),
        ("stay_join_tie_12", stayer_joiner_tie(1, 2), 2),
        ("stay_join_tie_21", stayer_joiner_tie(2, 1), 2),
        ("level_in_target", level_in_target(), 2),
        ("old_follower_lim12", old_follower_limits(12.0), 2),
        ("old_follower_lim14", old_follower_limits(14.0), 2),
        ("new_follower_lim12", new_follower_limits(12.0), 2),
        ("new_follower_lim14", new_follower_limits(14.0), 2),
        ("entry_behind_two", entry_behind_two(), 3),
        ("clamp_two_chains", clamp_two_chains(), 3),
    ]
