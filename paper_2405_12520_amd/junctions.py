"""Junction internal lanes: the map builder's lane connectivity inside
intersections (Sec. III-C-1: the map builder reconstructs lane connectivity
within intersections), as an input transformation of a scenario.

Every movement (in-road -> out-road) through a node becomes a short internal
road, the connector, with one lane per in-lane allowed to make that turn.
Lane-level successors tie each such in-lane to its connector lane and each
connector lane to one lane of the out-road.  Conflicting connector lanes
(crossing or merging paths) carry a priority order.  Routes gain the
connector between every two consecutive roads.  This module builds inputs
only: geometry and tables, none of the simulation's arithmetic.

Readings (the paper gives no rule):

* Turn of a movement: the signed angle from the in-road's heading to the
  out-road's; above 45 degrees (anticlockwise) a left turn, below -45 a
  right turn, else straight; the reverse road is a U-turn (taken as left).
* Lane k = 0 is the lane nearest the centre line (the leftmost, as in the
  position output).  Turns allowed per lane on a road of n lanes: n = 1: all;
  n = 2: lane 0 left and straight, lane 1 straight and right; n >= 3: lane 0
  left, the middle lanes straight, the last lane straight and right.  A lane
  whose turns all lack an exit at that node allows every turn there.
* Connector lane i of a movement starts from the i-th allowed in-lane and
  ends on out-lane min(i, n' - 1) for left turns and U-turns, n' - m + i
  (m connector lanes, clipped at 0) for right turns, and min(k, n' - 1) for
  straight movements from in-lane k.
* Connector lengths 16 m straight, 9 m right, 20 m left, 12 m U-turn; speed
  limit the smaller of the two roads', at most 8.33 m/s on turns.
* Paths run straight from the in-lane's stop line (8 m before the node,
  (k + 1/2) * 3.5 m right of the road's axis) to the out-lane's start (8 m
  after it).  Two connector lanes of different in-roads conflict when their
  paths cross or end on the same out-lane.  Priority: straight over right
  over left; between equal turns, the lower connector lane id.  Each
  connector lane lists the conflicting lanes that have priority over it,
  with the in-lane that feeds each.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .scenarios import Scenario, _lane_layout

LANE_W = 3.5          # m, lane width (as in the position output)
HALF_BOX = 8.0        # m, stop line to node centre
CONN_LEN = {"S": 16.0, "R": 9.0, "L": 20.0, "U": 12.0}
TURN_VLIM = 8.33      # m/s
RANK = {"S": 2, "R": 1, "L": 0, "U": 0}


def allowed_turns(n: int, k: int):
    """Turns lane k of an n-lane road may make at a junction (before the
    check against the exits the node has)."""
    if n == 1:
        return {"L", "S", "R", "U"}
    if n == 2:
        return {"L", "S", "U"} if k == 0 else {"S", "R"}
    if k == 0:
        return {"L", "U"}
    if k == n - 1:
        return {"S", "R"}
    return {"S"}


def turn_of(sc: Scenario, r: int, r2: int) -> str:
    if sc.road_from[r2] == sc.road_to[r] and sc.road_to[r2] == sc.road_from[r]:
        return "U"
    ax, ay = sc.node_x[sc.road_from[r]], sc.node_y[sc.road_from[r]]
    bx, by = sc.node_x[sc.road_to[r]], sc.node_y[sc.road_to[r]]
    cx, cy = sc.node_x[sc.road_to[r2]], sc.node_y[sc.road_to[r2]]
    h1 = (bx - ax, by - ay)
    h2 = (cx - bx, cy - by)
    ang = math.atan2(h1[0] * h2[1] - h1[1] * h2[0], h1[0] * h2[0] + h1[1] * h2[1])
    if ang > math.pi / 4:
        return "L"
    if ang < -math.pi / 4:
        return "R"
    return "S"


def _unit(dx, dy):
    n = math.hypot(dx, dy)
    return (dx / n, dy / n) if n > 0 else (1.0, 0.0)


def _stop_point(sc, r, k):
    """Where lane k of road r meets the junction (its stop line)."""
    ax, ay = sc.node_x[sc.road_from[r]], sc.node_y[sc.road_from[r]]
    bx, by = sc.node_x[sc.road_to[r]], sc.node_y[sc.road_to[r]]
    ux, uy = _unit(bx - ax, by - ay)
    off = (k + 0.5) * LANE_W
    return (bx - ux * HALF_BOX + uy * off, by - uy * HALF_BOX - ux * off)


def _start_point(sc, r, k):
    """Where lane k of road r leaves the junction at its upstream node."""
    ax, ay = sc.node_x[sc.road_from[r]], sc.node_y[sc.road_from[r]]
    bx, by = sc.node_x[sc.road_to[r]], sc.node_y[sc.road_to[r]]
    ux, uy = _unit(bx - ax, by - ay)
    off = (k + 0.5) * LANE_W
    return (ax + ux * HALF_BOX + uy * off, ay + uy * HALF_BOX - ux * off)


def _cross(p, q, r, s):
    """Whether segments p-q and r-s cross at a point inside both (shared
    end points and parallel overlaps do not count)."""
    def orient(a, b, c):
        v = (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])
        return 0 if abs(v) < 1e-9 else (1 if v > 0 else -1)
    o1, o2, o3, o4 = orient(p, q, r), orient(p, q, s), orient(r, s, p), orient(r, s, q)
    return o1 * o2 < 0 and o3 * o4 < 0


def with_junction_lanes(sc: Scenario) -> Scenario:
    """The scenario with connector roads in every junction its routes cross
    (all movements of each node the routes use, plus any U-turn a route
    takes), lane successors, conflicts and routes through the connectors."""
    nr0, nl0 = sc.n_roads, sc.n_lanes
    rf, rt = sc.road_from, sc.road_to
    used = set()
    for i in range(sc.n_veh):
        r = sc.route_roads[sc.route_off[i]:sc.route_off[i + 1]]
        used.update(zip(r[:-1].tolist(), r[1:].tolist()))
    nodes = sorted({int(rt[a]) for a, _ in used})
    out_of = {}
    for r in range(nr0):
        out_of.setdefault(int(rf[r]), []).append(r)
    in_of = {}
    for r in range(nr0):
        in_of.setdefault(int(rt[r]), []).append(r)

    conn_road = {}                     # (r, r2) -> connector road id
    c_from, c_len, c_vlim, c_lanes = [], [], [], []
    c_in_lane = []                     # per connector road: in-lane of each of its lanes
    c_out_lane = []                    # per connector road: out-lane of each of its lanes
    c_turn = []
    for j in nodes:
        for r in in_of.get(j, []):
            moves = []
            for r2 in out_of.get(j, []):
                t = turn_of(sc, r, r2)
                if t == "U" and (r, r2) not in used:
                    continue
                moves.append((r2, t))
            present = {t for _, t in moves}
            n = int(sc.road_nlanes[r])
            allow = []
            for k in range(n):
                a = allowed_turns(n, k) & present
                allow.append(a if a else set(present))
            for r2, t in moves:
                ks = [k for k in range(n) if t in allow[k]]
                n2 = int(sc.road_nlanes[r2])
                m = len(ks)
                if t in ("L", "U"):
                    outs = [min(i, n2 - 1) for i in range(m)]
                elif t == "R":
                    outs = [min(max(n2 - m + i, 0), n2 - 1) for i in range(m)]
                else:
                    outs = [min(k, n2 - 1) for k in ks]
                conn_road[(r, r2)] = nr0 + len(c_from)
                c_from.append(j)
                c_len.append(CONN_LEN[t])
                v = min(float(sc.lane_vlim[sc.road_lane0[r]]), float(sc.lane_vlim[sc.road_lane0[r2]]))
                c_vlim.append(v if t == "S" else min(v, TURN_VLIM))
                c_lanes.append(m)
                c_in_lane.append([int(sc.road_lane0[r]) + k for k in ks])
                c_out_lane.append([int(sc.road_lane0[r2]) + k for k in outs])
                c_turn.append(t)

    nc = len(c_from)
    road_from = np.concatenate([rf, np.asarray(c_from, np.int32)]).astype(np.int32)
    road_to = np.concatenate([rt, np.asarray(c_from, np.int32)]).astype(np.int32)
    road_length = np.concatenate([sc.road_length, np.asarray(c_len, np.float32)])
    road_nlanes = np.concatenate([sc.road_nlanes, np.asarray(c_lanes, np.int32)]).astype(np.int32)
    lane0, n_lanes, lane_road = _lane_layout(road_nlanes)
    assert np.array_equal(lane0[:nr0], sc.road_lane0)
    lane_vlim = np.concatenate([sc.lane_vlim, np.repeat(np.asarray(c_vlim, np.float32),
                                                        c_lanes)]).astype(np.float32)
    # scenario of a connector lane: the scenario of the lanes it joins
    conn_scen = []
    for q in range(nc):
        conn_scen += [int(sc.lane_scen[c_in_lane[q][0]])] * c_lanes[q]
    lane_scen = np.concatenate([sc.lane_scen, np.asarray(conn_scen, np.int32)]).astype(np.int32)
    road_group = np.concatenate([sc.road_group, np.full(nc, -1, np.int8)]).astype(np.int8)
    road_internal = np.concatenate([np.zeros(nr0, np.uint8), np.ones(nc, np.uint8)])

    # lane successors
    succ = [[] for _ in range(n_lanes)]
    for q in range(nc):
        l0 = int(lane0[nr0 + q])
        for i in range(c_lanes[q]):
            succ[c_in_lane[q][i]].append(l0 + i)
            succ[l0 + i].append(c_out_lane[q][i])
    succ_off = np.zeros(n_lanes + 1, np.int32)
    succ_off[1:] = np.cumsum([len(x) for x in succ])
    succ_lane = np.asarray([y for x in succ for y in x], np.int32)

    # conflicts between connector lanes of one node, from different in-roads
    geo = {}
    for (r, r2), cr in conn_road.items():
        q = cr - nr0
        for i in range(c_lanes[q]):
            kin = c_in_lane[q][i] - int(sc.road_lane0[r])
            kout = c_out_lane[q][i] - int(sc.road_lane0[r2])
            geo[int(lane0[cr]) + i] = (r, _stop_point(sc, r, kin), _start_point(sc, r2, kout),
                                       c_out_lane[q][i], RANK[c_turn[q]], c_in_lane[q][i])
    by_node = {}
    for (r, r2), cr in conn_road.items():
        q = cr - nr0
        for i in range(c_lanes[q]):
            by_node.setdefault(c_from[q], []).append(int(lane0[cr]) + i)
    conf = [[] for _ in range(n_lanes)]
    for j, lanes in by_node.items():
        for a in lanes:
            ra, pa, qa, oa, ka, _ = geo[a]
            for b in lanes:
                if a == b:
                    continue
                rb, pb, qb, ob, kb, fb = geo[b]
                if ra == rb:
                    continue
                if not (oa == ob or _cross(pa, qa, pb, qb)):
                    continue
                if kb > ka or (kb == ka and b < a):
                    conf[a].append((b, fb))
    conf_off = np.zeros(n_lanes + 1, np.int32)
    conf_off[1:] = np.cumsum([len(x) for x in conf])
    conf_lane = np.asarray([b for x in conf for b, _ in x], np.int32)
    conf_feed = np.asarray([f for x in conf for _, f in x], np.int32)

    # routes through the connectors; placed vehicles keep their road (cursor
    # doubled) and lane
    routes = []
    for i in range(sc.n_veh):
        r = sc.route_roads[sc.route_off[i]:sc.route_off[i + 1]].tolist()
        out = [r[0]]
        for a, b in zip(r[:-1], r[1:]):
            out += [conn_road[(a, b)], b]
        routes.append(out)
    off = np.zeros(sc.n_veh + 1, np.int64)
    off[1:] = np.cumsum([len(x) for x in routes])
    flat = np.asarray([y for x in routes for y in x], np.int32)
    meta = dict(sc.meta, junction_lanes=dict(
        connectors=nc, connector_lanes=int(sum(c_lanes)), regular_roads=nr0, regular_lanes=nl0,
        movements={(int(a), int(b)): int(c) for (a, b), c in conn_road.items()},
        turns={int(nr0 + q): c_turn[q] for q in range(nc)}))
    return dataclasses.replace(
        sc, name=sc.name + "+jl", road_from=road_from, road_to=road_to,
        road_length=road_length.astype(np.float32), road_nlanes=road_nlanes, road_lane0=lane0,
        lane_vlim=lane_vlim, lane_scen=lane_scen, road_group=road_group,
        route_off=off, route_roads=flat, cursor=(sc.cursor * 2).astype(np.int32),
        road_internal=road_internal, lane_succ_off=succ_off, lane_succ=succ_lane,
        lane_conf_off=conf_off, lane_conf=conf_lane, lane_conf_feed=conf_feed, meta=meta)
