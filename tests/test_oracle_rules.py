"""Oracle pins for single rules, from hand-computed toy states.

Every expected value here is worked out by hand from the rule as stated
(insertion gap and entry speed, the stop-line condition, the last-road
exemption, MOBIL's safety conditions and target-lane acceleration, the
overlap clamp and the (position, id) order of the merge), not read back from
the oracle.  The states are in tests/rule_cases.py; the GPU parity test runs
the same states through the HIP library.

Each test is built so that one plausible slip in the rule it pins -- a
dropped term, the wrong lane's limit, a missing condition, a reversed tie --
changes its outcome.
"""
import math

import numpy as np
import pytest

import rule_cases as RC
from oracle import OracleSim

F32 = np.float32


def _row(st, vid):
    k = np.flatnonzero(st["id"] == vid)
    assert k.shape[0] == 1, f"vehicle {vid} not active"
    return int(k[0])


def _dbg(o, vid):
    d = o.debug()
    k = int(np.flatnonzero(d["id"] == vid)[0])
    return {f: d[f][k] for f in d}


# ------------------------------------------------------- R2 insertion --

def test_insertion_gap_includes_vehicle_length():
    """Entry needs s_tail - len >= s0 + v T with v = min(v0, limit, v_tail):
    with v_tail = 4 the bound is 5 + 2 + 4 * 1.5 = 13 m exactly.  A tail at
    13 m admits the entry (the comparison is >=), the next float below it
    does not (and the refusal is counted)."""
    o = OracleSim(RC.insertion_behind_tail(13.0))
    o.step(1)
    c, _ = o.counters()
    assert (c[0, 0], c[0, 1]) == (1, 0)
    st = o.state()
    k = _row(st, 2)
    assert st["s"][k] == 0.0 and st["v"][k] == F32(4.0)
    o = OracleSim(RC.insertion_behind_tail(float(np.nextafter(F32(13.0), F32(0.0)))))
    o.step(1)
    c, _ = o.counters()
    assert (c[0, 0], c[0, 1]) == (0, 1)
    assert o.n_active == 1 and o.pending == 1


def test_insertion_two_lane_road_uses_id_lane():
    """On a two-lane road vehicle 4 queues on lane 4 mod 2 = 0, behind the
    tail at 13 m: the same bound applies there."""
    o = OracleSim(RC.insertion_behind_tail(13.0, lanes=2))
    o.step(1)
    st = o.state()
    assert st["lane"][_row(st, 4)] == 0


@pytest.mark.parametrize("v_tail,expect", [(4.0, 4.0), (15.0, 14.0)])
def test_insertion_speed_is_min_of_desired_and_tail(v_tail, expect):
    """Entry speed min(v0, limit, v_tail): a slower tail (4 m/s) sets it, a
    faster one (15 m/s) leaves the desired speed 14 m/s.  The entering
    vehicle does not move in its entry step."""
    o = OracleSim(RC.insertion_behind_tail(100.0, v_tail=v_tail))
    o.step(1)
    st = o.state()
    k = _row(st, 2)
    assert st["s"][k] == 0.0
    assert st["v"][k] == F32(expect)
    assert st["a"][k] == 0.0


def test_insertion_on_empty_lane_takes_speed_limit():
    """Empty lane: entry speed min(v0, limit) = min(20, 16.67)."""
    o = OracleSim(RC.empty_lane_insertion(20.0))
    o.step(1)
    st = o.state()
    assert st["v"][0] == F32(16.67)


# ------------------------------------------------------------ R5 signals --

def test_red_ignored_when_vehicle_cannot_stop():
    """Stopping distance v^2 / (2 b_max) = 15^2 / 18 = 12.5 m.  10 m before a
    red stop line the vehicle cannot stop and drives on (no red obstacle);
    at exactly 12.5 m it can (>=), and the red obstacle applies; one float
    further the distance is short of 12.5 m again."""
    o = OracleSim(RC.red_approach(290.0))
    o.step(1)
    assert not (_dbg(o, 1)["flags"] & 4)
    o.step(1)
    st = o.state()
    assert st["lane"][0] == 1       # crossed into the next road
    o = OracleSim(RC.red_approach(287.5))
    o.step(1)
    assert _dbg(o, 1)["flags"] & 4
    o = OracleSim(RC.red_approach(float(np.nextafter(F32(287.5), F32(1e9)))))
    o.step(1)
    assert not (_dbg(o, 1)["flags"] & 4)


def test_last_road_never_waits():
    """A vehicle whose route ends on the road before a permanently red
    junction never sees the red obstacle and arrives at the road end."""
    o = OracleSim(RC.red_approach(200.0, v=10.0, route=(0,)))
    for _ in range(20):
        o.step(1)
        if o.n_active == 0:
            break
        assert not (_dbg(o, 1)["flags"] & 4)
    c, _ = o.counters()
    assert c[0, 2] == 1 and o.n_active == 0


# -------------------------------------------------------------- R7 MOBIL --

def test_cut_in_refused_by_rear_gap_alone():
    """b_safe = 10 and politeness 0, so the new follower's braking (at most
    b_max = 9) never refuses the change and its cost does not enter the
    incentive.  The target lane's follower is standing with its front at
    s_n.  Rear gap s - len - s_n = 0: refused by gap_b > 0 alone (its IDM
    acceleration is the guard -b_max = -9 >= -10).  Rear gap 1 m: IDM
    s* = s0 = 2, a = 2 (1 - 0 - 2^2) = -6 >= -10, safe, and the change is
    made."""
    o = OracleSim(RC.cut_in_behind(195.0))
    o.step(1)
    d = _dbg(o, 1)
    assert d["flags"] & 3 == 1 and d["t_follower"] == 3 and d["margin"] > 1.0
    o = OracleSim(RC.cut_in_behind(194.0))
    o.step(1)
    d = _dbg(o, 1)
    assert d["flags"] & 3 == 2 and d["t_follower"] == 3


def test_cut_in_refused_by_follower_braking():
    """Same rear gap of 1 m with b_safe = 4.5: the new follower would have to
    brake at 6 m/s^2 > 4.5, so the change is refused."""
    o = OracleSim(RC.cut_in_behind(194.0, b_safe=4.5))
    o.step(1)
    assert _dbg(o, 1)["flags"] & 3 == 1


def test_cut_in_at_the_braking_limit():
    """Same rear gap of 1 m with b_safe = 6: the new follower's acceleration
    after the change, 2 (1 - (2/1)^2) = -6, is exact in FP32 and equals
    -b_safe.  MOBIL's safety criterion admits a~_n >= -b_safe, so the change
    is made (a strict comparison would refuse it)."""
    o = OracleSim(RC.cut_in_behind(194.0, b_safe=6.0))
    o.step(1)
    d = _dbg(o, 1)
    assert d["flags"] & 3 == 2 and d["t_follower"] == 3


def _idm64(v, v0e, vl=None, gap=None, a=2.0, b=4.5, s0=2.0, T=1.5):
    free = 1.0 - (v / v0e) ** 4
    if vl is None:
        return a * free
    ss = s0 + max(0.0, v * T + v * (v - vl) / (2.0 * math.sqrt(a * b)))
    return a * (free - (ss / gap) ** 2)


@pytest.mark.parametrize("vt,vo", [(8.0, 16.67), (16.67, 8.0)])
def test_target_lane_acceleration_uses_target_limit(vt, vo):
    """Incentive (a~_c - a_c) with no old or new follower: a_c behind the
    leader 60 m ahead at equal speed in the own lane (v0 = min(14, own
    limit)), a~_c on the empty target lane with v0 = min(14, target limit).
    A target limit of 8 m/s (below the speed 10) makes a~_c = 2 (1 - 1.25^4)
    < 0 and no change; the same road with the limits swapped makes the own
    lane the slow one and the change pays.  Margin inc - 0.1 agrees with the
    textbook IDM in FP64."""
    o = OracleSim(RC.limits_differ(vt, vo))
    o.step(1)
    d = _dbg(o, 1)
    v0 = 14.0
    a_c = _idm64(10.0, min(v0, float(F32(vo))), 10.0, 60.0)
    at_c = _idm64(10.0, min(v0, float(F32(vt))))
    margin = (at_c - a_c) - 0.1
    assert abs(float(d["margin"]) - margin) < 1e-5
    assert d["flags"] & 3 == (2 if margin > 0 else 1)
    assert (margin > 0) == (vt > vo)


# ----------------------------------------------------------- R10 merge --

def test_clamped_follower_takes_leader_speed():
    """Leader: free road from rest, v0 = 0.5: a = 2, v' = 2, s' = 101.
    Follower 1 m behind its rear at 20 m/s brakes at b_max: v' = 11,
    s' = 94 + 20 - 4.5 = 109.5, beyond 101 - 5.  It is clamped to 96 and its
    speed capped at the leader's 2 m/s; one clamp is counted."""
    o = OracleSim(RC.clamp_fast_follower())
    o.step(1)
    st = o.state()
    f, l = _row(st, 1), _row(st, 2)
    assert st["s"][l] == F32(101.0) and st["v"][l] == F32(2.0)
    assert st["s"][f] == F32(96.0) and st["v"][f] == F32(2.0)
    assert st["a"][f] == F32(-9.0)
    assert f == l - 1
    c, _ = o.counters()
    assert c[0, 4] == 1


@pytest.mark.parametrize("a,b", [(1, 2), (2, 1)])
def test_equal_joiners_ordered_by_id(a, b):
    """Two vehicles enter the one-lane road at exactly s = 20 (see
    rule_cases.joiners_tie).  The merge orders equal positions by id: the
    lower id is the row behind, clamped to 20 - len = 15."""
    o = OracleSim(RC.joiners_tie(a, b))
    o.step(1)
    st = o.state()
    lo, hi = _row(st, 1), _row(st, 2)
    assert lo == hi - 1
    assert st["s"][hi] == F32(20.0) and st["s"][lo] == F32(15.0)
    assert st["lane"][lo] == st["lane"][hi] == 2


@pytest.mark.parametrize("stayer,joiner", [(1, 2), (2, 1)])
def test_stayer_and_joiner_tie_ordered_by_id(stayer, joiner):
    """A stayer and a joiner both at exactly s = 20 in one lane: the lower id
    is behind, whichever of the two it is."""
    o = OracleSim(RC.stayer_joiner_tie(stayer, joiner))
    o.step(1)
    st = o.state()
    lo, hi = _row(st, 1), _row(st, 2)
    assert lo == hi - 1
    assert st["s"][hi] == F32(20.0) and st["s"][lo] == F32(15.0)
    c, _ = o.counters()
    assert c[0, 4] == 1
