"""Seeded synthetic road networks, signal plans and travel demand.

This module is the single source of inputs for both the HIP simulator and the
CPU oracle.  It builds networks, signal timings, vehicle routes and (for
snapshots) initial vehicle placements; it contains none of the simulation
arithmetic (no car-following, lane-changing or integration).

The paper feeds its simulator a road network plus travel demand and measures
it on real city maps and grid networks of 10^0..10^6 vehicles, 3600 one-second
steps (Sec. III-A, Sec. IV-A).  Those maps are not available, so every workload
here is synthetic; the shapes follow the five workloads the project measures:

* ``intersection``  one signalised 4-way junction, 2 lanes x 500 m per arm,
                    200 vehicles departing over 600 s;
* ``grid``          n x n grid, 200 m links, 3 lanes per direction,
                    fixed-time signals with random offsets, shortest-path routes;
* ``city_snapshot`` ~40k-node random planar graph, ~120k lanes, log-normal road
                    lengths (median 150 m), 2M vehicles pre-placed on long routes;
* ``city_demand``   the same city with 2M gravity-model trips over 400 zones
                    departing over one hour on shortest paths;
* ``batch``         256 independent grids (4x4 .. 16x16, 1k..50k vehicles each)
                    joined into one disjoint-union network;
* ``ring`` / ``toy``  small closed-form and brute-force test cases.

Conventions shared by both consumers
------------------------------------
* A road has ``road_nlanes`` lanes numbered ``road_lane0 .. road_lane0+n-1``;
  index ``k`` in the road is ``lane - road_lane0``.  All lanes of a road share
  the road's length.
* ``road_group[r]`` is the signal group of road ``r`` at its downstream node
  (``-1`` means always green); the node's plan is (cycle, phase length,
  offset) in integer steps, cycle 0 meaning unsignalised.
* A vehicle route is a chain of roads, each starting where the previous one
  ends.  Pending vehicles enter their first road at its start; pre-placed
  vehicles (``placed == 1``) start on ``lane`` at front-bumper position ``s``
  with route cursor ``cursor``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional

import numpy as np

# Model constants used by the measured workloads.  a, b, s0, T, politeness
# and threshold are the workload's stated values; the rest are this project's
# readings of points the paper leaves open.
DEFAULT_PARAMS: Dict[str, float] = dict(
    dt=1.0,            # s
    a_max=2.0,         # m/s^2, IDM maximum acceleration
    b=4.5,             # m/s^2, IDM comfortable deceleration
    s0=2.0,            # m, jam distance
    T=1.5,             # s, safe time headway
    length=5.0,        # m, vehicle length
    b_max=9.0,         # m/s^2, physical braking limit
    b_safe=4.5,        # m/s^2, MOBIL safe deceleration of the new follower
    politeness=0.2,    # MOBIL politeness
    a_thr=0.1,         # m/s^2, MOBIL switching threshold
    p_lc=0.5,          # probability of executing a beneficial, safe change
    d_look=300.0,      # m, lookahead distance across junctions
    h_look=3,          # max roads scanned ahead for a leader
    b_mand=1.0,        # m/s^2, lane-change bias toward lanes that continue the route
    tau_yield=3.0,     # s, approach time within which a vehicle with priority is yielded to
    seed=4,            # RNG key for the lane-change draws
    t0=0,              # first step index
)

NETWORK_SEED, DEMAND_SEED, PARAM_SEED, RNG_SEED = 1, 2, 3, 4
SPEED_LIMITS = np.array([11.11, 13.89, 16.67], dtype=np.float32)


@dataclasses.dataclass
class Scenario:
    name: str
    # network
    node_x: np.ndarray
    node_y: np.ndarray
    road_from: np.ndarray
    road_to: np.ndarray
    road_length: np.ndarray
    road_nlanes: np.ndarray
    road_lane0: np.ndarray
    lane_vlim: np.ndarray
    lane_scen: np.ndarray
    # signals
    node_cycle: np.ndarray
    node_phase: np.ndarray
    node_offset: np.ndarray
    road_group: np.ndarray
    # vehicles
    veh_id: np.ndarray
    depart: np.ndarray
    v0: np.ndarray
    route_off: np.ndarray
    route_roads: np.ndarray
    placed: np.ndarray
    lane: np.ndarray
    s: np.ndarray
    v: np.ndarray
    a: np.ndarray
    cursor: np.ndarray
    params: Dict[str, float]
    n_scen: int = 1
    meta: Dict[str, object] = dataclasses.field(default_factory=dict)
    # junction internal lanes (junctions.with_junction_lanes), None without:
    # internal-road flags, lane successors (CSR over lanes) and, per connector
    # lane, the conflicting connector lanes with priority over it and the
    # in-lane feeding each
    road_internal: Optional[np.ndarray] = None
    lane_succ_off: Optional[np.ndarray] = None
    lane_succ: Optional[np.ndarray] = None
    lane_conf_off: Optional[np.ndarray] = None
    lane_conf: Optional[np.ndarray] = None
    lane_conf_feed: Optional[np.ndarray] = None

    @property
    def n_nodes(self) -> int:
        return int(self.node_x.shape[0])

    @property
    def n_roads(self) -> int:
        return int(self.road_from.shape[0])

    @property
    def n_lanes(self) -> int:
        return int(self.lane_vlim.shape[0])

    @property
    def n_veh(self) -> int:
        return int(self.veh_id.shape[0])

    def with_params(self, **kw) -> "Scenario":
        p = dict(self.params)
        p.update(kw)
        return dataclasses.replace(self, params=p)

    def summary(self) -> Dict[str, object]:
        lanes_per_road = np.bincount(self.road_nlanes, minlength=5)[1:5]
        return dict(name=self.name, nodes=self.n_nodes, roads=self.n_roads,
                    lanes=self.n_lanes, vehicles=self.n_veh,
                    placed=int(self.placed.sum()),
                    signalised=int((self.node_cycle > 0).sum()),
                    lane_km=float((self.road_length.astype(np.float64)
                                   * self.road_nlanes).sum() / 1000.0),
                    lanes_per_road=lanes_per_road.tolist(),
                    route_entries=int(self.route_roads.shape[0]),
                    scenarios=self.n_scen)


# ---------------------------------------------------------------------------
# helpers
# ---------------------------------------------------------------------------

def _lane_layout(road_nlanes: np.ndarray):
    lane0 = np.zeros(road_nlanes.shape[0], dtype=np.int32)
    if road_nlanes.shape[0] > 1:
        lane0[1:] = np.cumsum(road_nlanes[:-1], dtype=np.int64).astype(np.int32)
    n_lanes = int(road_nlanes.sum())
    lane_road = np.repeat(np.arange(road_nlanes.shape[0], dtype=np.int32), road_nlanes)
    return lane0, n_lanes, lane_road


def _heading_groups(node_x, node_y, road_from, road_to, signalised):
    """Group 0 = roads whose heading is closer to the x axis, 1 otherwise."""
    dx = node_x[road_to] - node_x[road_from]
    dy = node_y[road_to] - node_y[road_from]
    g = np.where(np.abs(dx) >= np.abs(dy), 0, 1).astype(np.int8)
    g[~signalised[road_to]] = -1
    return g


def _desired_speeds(rng: np.random.Generator, n: int) -> np.ndarray:
    """v0 ~ N(13.9, 1.5) m/s clipped to [8, 20]."""
    return np.clip(rng.normal(13.9, 1.5, size=n), 8.0, 20.0).astype(np.float32)


def _pack_routes(routes):
    off = np.zeros(len(routes) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(r) for r in routes])
    flat = np.concatenate([np.asarray(r, dtype=np.int32) for r in routes]) if routes else \
        np.zeros(0, dtype=np.int32)
    return off, flat


def _empty_placement(n):
    return (np.zeros(n, np.uint8), np.full(n, -1, np.int32), np.zeros(n, np.float32),
            np.zeros(n, np.float32), np.zeros(n, np.float32), np.zeros(n, np.int32))


def _make(name, node_x, node_y, road_from, road_to, road_length, road_nlanes, road_vlim,
          node_cycle, node_phase, node_offset, road_group, veh_id, depart, v0, route_off,
          route_roads, placement=None, params=None, lane_scen=None, n_scen=1, meta=None):
    road_nlanes = np.asarray(road_nlanes, np.int32)
    lane0, n_lanes, lane_road = _lane_layout(road_nlanes)
    lane_vlim = np.asarray(road_vlim, np.float32)[lane_road]
    if lane_scen is None:
        lane_scen = np.zeros(n_lanes, np.int32)
    n = int(len(veh_id))
    if placement is None:
        placement = _empty_placement(n)
    p = dict(DEFAULT_PARAMS)
    if params:
        p.update(params)
    placed, lane, s, v, a, cursor = placement
    return Scenario(
        name=name,
        node_x=np.asarray(node_x, np.float64), node_y=np.asarray(node_y, np.float64),
        road_from=np.asarray(road_from, np.int32), road_to=np.asarray(road_to, np.int32),
        road_length=np.asarray(road_length, np.float32), road_nlanes=road_nlanes,
        road_lane0=lane0, lane_vlim=lane_vlim, lane_scen=np.asarray(lane_scen, np.int32),
        node_cycle=np.asarray(node_cycle, np.int32), node_phase=np.asarray(node_phase, np.int32),
        node_offset=np.asarray(node_offset, np.int32), road_group=np.asarray(road_group, np.int8),
        veh_id=np.asarray(veh_id, np.uint32), depart=np.asarray(depart, np.int32),
        v0=np.asarray(v0, np.float32), route_off=np.asarray(route_off, np.int64),
        route_roads=np.asarray(route_roads, np.int32),
        placed=np.asarray(placed, np.uint8), lane=np.asarray(lane, np.int32),
        s=np.asarray(s, np.float32), v=np.asarray(v, np.float32), a=np.asarray(a, np.float32),
        cursor=np.asarray(cursor, np.int32), params=p, n_scen=n_scen, meta=dict(meta or {}))


# ---------------------------------------------------------------------------
# closed-form / small test networks
# ---------------------------------------------------------------------------

def ring(n_veh: int, circumference: float, v_init: float, *, v0: float = 14.0,
         vlim: float = 30.0, laps: int = 400, params=None) -> Scenario:
    """One single-lane road whose end feeds its own start, vehicles evenly spaced.

    Every vehicle is pre-placed with speed ``v_init`` and a route that repeats
    the ring ``laps`` times, so nobody arrives during a test.
    """
    L = float(circumference)
    spacing = L / n_veh
    s = (np.arange(n_veh, dtype=np.float64) * spacing).astype(np.float32)
    ids = np.arange(n_veh, dtype=np.uint32)
    routes = [[0] * laps for _ in range(n_veh)]
    off, flat = _pack_routes(routes)
    placement = (np.ones(n_veh, np.uint8), np.zeros(n_veh, np.int32), s,
                 np.full(n_veh, v_init, np.float32), np.zeros(n_veh, np.float32),
                 np.zeros(n_veh, np.int32))
    return _make("ring", [0.0], [0.0], [0], [0], [L], [1], [vlim], [0], [0], [0], [-1],
                 ids, np.zeros(n_veh, np.int32), np.full(n_veh, v0, np.float32), off, flat,
                 placement, params)


def corridor(lengths, nlanes, *, vlim=16.67, signal=None, params=None):
    """A straight chain of roads (node i -> node i+1); no vehicles yet.

    ``signal`` = (node, cycle, phase, offset, group_of_incoming_road) puts a
    fixed-time signal on one interior node.
    """
    nr = len(lengths)
    nn = nr + 1
    x = np.cumsum([0.0] + [float(L) for L in lengths])
    cyc = np.zeros(nn, np.int32)
    ph = np.zeros(nn, np.int32)
    off = np.zeros(nn, np.int32)
    grp = np.full(nr, -1, np.int8)
    if signal is not None:
        node, c, p, o, g = signal
        cyc[node], ph[node], off[node] = c, p, o
        grp[node - 1] = g
    nl = np.broadcast_to(np.asarray(nlanes, np.int32), (nr,)).copy()
    return dict(node_x=x, node_y=np.zeros(nn), road_from=np.arange(nr), road_to=np.arange(1, nn),
                road_length=np.asarray(lengths, np.float32), road_nlanes=nl,
                road_vlim=np.full(nr, vlim, np.float32), node_cycle=cyc, node_phase=ph,
                node_offset=off, road_group=grp)


def with_vehicles(name, net: dict, vehicles: list, params=None) -> Scenario:
    """Attach an explicit vehicle list to a network dict from ``corridor``/``toy``.

    Each vehicle is a dict with keys ``id, route`` and optionally ``depart, v0,
    lane, s, v, a, cursor`` (a vehicle with ``lane`` is pre-placed).
    """
    n = len(vehicles)
    ids = np.array([q["id"] for q in vehicles], np.uint32)
    dep = np.array([q.get("depart", 0) for q in vehicles], np.int32)
    v0 = np.array([q.get("v0", 14.0) for q in vehicles], np.float32)
    off, flat = _pack_routes([q["route"] for q in vehicles])
    placed, lane, s, v, a, cur = _empty_placement(n)
    for i, q in enumerate(vehicles):
        if "lane" in q:
            placed[i] = 1
            lane[i] = q["lane"]
            s[i] = q["s"]
            v[i] = q.get("v", 0.0)
            a[i] = q.get("a", 0.0)
            cur[i] = q.get("cursor", 0)
    return _make(name, net["node_x"], net["node_y"], net["road_from"], net["road_to"],
                 net["road_length"], net["road_nlanes"], net["road_vlim"], net["node_cycle"],
                 net["node_phase"], net["node_offset"], net["road_group"], ids, dep, v0, off, flat,
                 (placed, lane, s, v, a, cur), params)


def resume(sc: Scenario, ckpt: dict) -> Scenario:
    """The scenario that continues a run of ``sc`` from a checkpoint (a dict
    with the state rows ``state``, the ids still waiting ``pending`` and the
    next step ``t``, as Simulator.checkpoint returns it).

    A step reads only the vehicle state and the departure queues (Sec.
    III-A), so the active rows become placed vehicles (lane, position, speed,
    previous acceleration, route index), the waiting ones keep their
    departure step, arrived vehicles are dropped and the first step is ``t``.
    Counters of the new run start at zero."""
    st, pend, t = ckpt["state"], np.asarray(ckpt["pending"], np.uint32), int(ckpt["t"])
    order = np.argsort(sc.veh_id, kind="stable")
    sorted_id = sc.veh_id[order]

    def rows_of(ids):
        k = np.searchsorted(sorted_id, ids)
        found = sorted_id[np.minimum(k, len(sorted_id) - 1)] == ids
        if np.any(k >= len(sorted_id)) or not np.all(found):
            raise ValueError("checkpoint names a vehicle the scenario does not have")
        return order[k]

    act = rows_of(np.asarray(st["id"], np.uint32))
    keep = np.concatenate([act, rows_of(pend)])
    if len(np.unique(keep)) != len(keep):
        raise ValueError("a vehicle is both active and pending in the checkpoint")
    n, na = len(keep), len(act)
    lens = sc.route_off[keep + 1] - sc.route_off[keep]
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum(lens)
    src = np.repeat(sc.route_off[keep], lens) + (np.arange(off[-1]) - np.repeat(off[:-1], lens))
    placed = np.zeros(n, np.uint8)
    placed[:na] = 1
    lane = np.zeros(n, np.int32)
    cursor = np.zeros(n, np.int32)
    s, v, a = (np.zeros(n, np.float32) for _ in range(3))
    lane[:na] = st["lane"]
    cursor[:na] = st["cursor"]
    s[:na], v[:na], a[:na] = st["s"], st["v"], st["a"]
    return dataclasses.replace(
        sc, name=f"{sc.name}@{t}", veh_id=sc.veh_id[keep], depart=sc.depart[keep],
        v0=sc.v0[keep], route_off=off, route_roads=sc.route_roads[src].astype(np.int32),
        placed=placed, lane=lane, s=s, v=v, a=a, cursor=cursor, params=dict(sc.params, t0=t))


_CKPT_FIELDS = ("id", "lane", "s", "v", "a", "cursor")


def save_checkpoint(path: str, ckpt: dict) -> None:
    """Writes a checkpoint (resume's input) to an .npz file of plain arrays."""
    arrays = {f"state_{k}": np.asarray(ckpt["state"][k]) for k in _CKPT_FIELDS}
    np.savez(path, pending=np.asarray(ckpt["pending"], np.uint32),
             t=np.int64(ckpt["t"]), **arrays)


def load_checkpoint(path: str) -> dict:
    """Reads a checkpoint written by save_checkpoint (no pickled objects)."""
    with np.load(path, allow_pickle=False) as z:
        return dict(state={k: z[f"state_{k}"].copy() for k in _CKPT_FIELDS},
                    pending=z["pending"].copy(), t=int(z["t"]))


# ---------------------------------------------------------------------------
# grids
# ---------------------------------------------------------------------------

def _grid_network(n: int, spacing: float, lanes: int, rng: np.random.Generator,
                  x0: float = 0.0, y0: float = 0.0):
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    node_x = (x0 + jj.ravel() * spacing).astype(np.float64)
    node_y = (y0 + ii.ravel() * spacing).astype(np.float64)
    und = []
    for i in range(n):
        for j in range(n):
            u = i * n + j
            if j + 1 < n:
                und.append((u, u + 1))
            if i + 1 < n:
                und.append((u, u + n))
    und = np.array(und, dtype=np.int32).reshape(-1, 2)
    road_from = np.empty(2 * len(und), np.int32)
    road_to = np.empty(2 * len(und), np.int32)
    road_from[0::2], road_to[0::2] = und[:, 0], und[:, 1]
    road_from[1::2], road_to[1::2] = und[:, 1], und[:, 0]
    nr = road_from.shape[0]
    road_length = np.full(nr, spacing, np.float32)
    road_nlanes = np.full(nr, lanes, np.int32)
    # both directions of a link share the link's speed limit
    road_vlim = np.repeat(SPEED_LIMITS[rng.integers(0, 3, size=len(und))], 2)
    deg = np.bincount(road_to, minlength=n * n)
    signalised = deg >= 3
    cyc = np.where(signalised, 60, 0).astype(np.int32)
    ph = np.where(signalised, 30, 0).astype(np.int32)
    off = np.where(signalised, rng.integers(0, 60, size=n * n), 0).astype(np.int32)
    grp = _heading_groups(node_x, node_y, road_from, road_to, signalised)
    return node_x, node_y, road_from, road_to, road_length, road_nlanes, road_vlim, cyc, ph, off, grp


def _road_index(road_from, road_to, n_nodes):
    """Dense (from, to) -> road id lookup for small networks."""
    m = np.full((n_nodes, n_nodes), -1, np.int32)
    m[road_from, road_to] = np.arange(road_from.shape[0], dtype=np.int32)
    return m


def _shortest_path_routes(n_nodes, road_from, road_to, road_length, orig, dest, max_hops):
    """Routes (as road lists) along shortest paths from orig[i] to dest[i].

    Uses scipy's Dijkstra on the symmetric node graph; for each destination
    the predecessor tree gives the next hop toward it from every node.
    """
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra

    g = csr_matrix((road_length.astype(np.float64), (road_from, road_to)),
                   shape=(n_nodes, n_nodes))
    dests = np.unique(dest)
    _, pred = dijkstra(g, directed=True, indices=dests, return_predecessors=True)
    # pred[k, x] = predecessor of x on the shortest path dests[k] -> x.  The
    # networks here are symmetric (every road has a reverse of equal length),
    # so walking x -> pred[k, x] follows a shortest path from x to dests[k].
    dk = np.searchsorted(dests, dest)
    ridx = _road_index(road_from, road_to, n_nodes)
    cur = orig.astype(np.int64).copy()
    hops = np.full((orig.shape[0], max_hops), -1, np.int32)
    nh = np.zeros(orig.shape[0], np.int32)
    for h in range(max_hops):
        act = cur != dest
        if not act.any():
            break
        nxt = pred[dk[act], cur[act]]
        hops[act, h] = ridx[cur[act], nxt]
        nh[act] += 1
        cur[act] = nxt
    assert (cur == dest).all(), "route longer than max_hops"
    assert (hops[hops >= 0] >= 0).all()
    off = np.zeros(orig.shape[0] + 1, np.int64)
    off[1:] = np.cumsum(nh)
    # rows are filled left to right, so row-major compaction keeps route order
    mask = np.arange(max_hops)[None, :] < nh[:, None]
    flat = hops[mask]
    return off, flat


def grid(n: int = 10, n_veh: int = 20000, *, lanes: int = 3, spacing: float = 200.0,
         horizon: int = 3600, seed: int = NETWORK_SEED, demand_seed: int = DEMAND_SEED,
         param_seed: int = PARAM_SEED, params=None) -> Scenario:
    """n x n grid: 200 m links, 3 lanes per direction, signals at every node of
    degree >= 3 (cycle 60 s, two 30 s phases, random offsets), vehicles with
    uniform departure steps in [0, horizon) between distinct uniform nodes on
    shortest paths."""
    rng_net = np.random.default_rng(seed)
    (nx_, ny_, rf, rt, rl, rn, rv, cyc, ph, off, grp) = _grid_network(n, spacing, lanes, rng_net)
    rng_d = np.random.default_rng(demand_seed)
    nn = n * n
    orig = rng_d.integers(0, nn, size=n_veh)
    dest = (orig + rng_d.integers(1, nn, size=n_veh)) % nn
    depart = np.sort(rng_d.integers(0, horizon, size=n_veh)).astype(np.int32)
    roff, rflat = _shortest_path_routes(nn, rf, rt, rl, orig, dest, 4 * n)
    v0 = _desired_speeds(np.random.default_rng(param_seed), n_veh)
    ids = np.arange(n_veh, dtype=np.uint32)
    return _make(f"grid{n}x{n}", nx_, ny_, rf, rt, rl, rn, rv, cyc, ph, off, grp, ids, depart,
                 v0, roff, rflat, None, params,
                 meta=dict(seed=seed, demand_seed=demand_seed, horizon=horizon))


def intersection(n_veh: int = 200, *, arm: float = 500.0, lanes: int = 2, horizon: int = 600,
                 seed: int = DEMAND_SEED, param_seed: int = PARAM_SEED,
                 params=None) -> Scenario:
    """Single signalised 4-way junction: 4 arms, each a 500 m in-road and a
    500 m out-road with 2 lanes; fixed-time plan with 60 s cycle and 30 s
    phases (N/S approaches in group 0); 200 vehicles with uniform departures
    over 600 s, a uniform approach and a uniform movement (left, straight,
    right)."""
    # nodes: 0 centre, 1 N, 2 E, 3 S, 4 W
    node_x = np.array([0.0, 0.0, arm, 0.0, -arm])
    node_y = np.array([0.0, arm, 0.0, -arm, 0.0])
    road_from, road_to = [], []
    for a in range(4):          # in-road of arm a: 2a, out-road: 2a+1
        road_from += [1 + a, 0]
        road_to += [0, 1 + a]
    nr = 8
    rl = np.full(nr, arm, np.float32)
    rn = np.full(nr, lanes, np.int32)
    rv = np.full(nr, 16.67, np.float32)
    cyc = np.array([60, 0, 0, 0, 0], np.int32)
    ph = np.array([30, 0, 0, 0, 0], np.int32)
    off = np.zeros(5, np.int32)
    grp = np.full(nr, -1, np.int8)
    for a in range(4):
        grp[2 * a] = 0 if a in (0, 2) else 1      # N/S approaches share the first phase
    rng = np.random.default_rng(seed)
    depart = np.sort(rng.integers(0, horizon, size=n_veh)).astype(np.int32)
    arm_in = rng.integers(0, 4, size=n_veh)
    move = rng.integers(0, 3, size=n_veh)          # 0 right, 1 straight, 2 left
    # arms are numbered clockwise N, E, S, W; a vehicle arriving from arm a
    # heading into the junction turns right onto arm a-1, straight to a+2,
    # left to a+1 (mod 4)
    arm_out = np.where(move == 0, (arm_in + 3) % 4, np.where(move == 1, (arm_in + 2) % 4,
                                                             (arm_in + 1) % 4))
    routes = [[2 * int(a), 2 * int(b) + 1] for a, b in zip(arm_in, arm_out)]
    roff, rflat = _pack_routes(routes)
    v0 = _desired_speeds(np.random.default_rng(param_seed), n_veh)
    ids = np.arange(n_veh, dtype=np.uint32)
    return _make("intersection", node_x, node_y, road_from, road_to, rl, rn, rv, cyc, ph, off,
                 grp, ids, depart, v0, roff, rflat, None, params,
                 meta=dict(seed=seed, horizon=horizon))


# ---------------------------------------------------------------------------
# random walks and snapshot placement
# ---------------------------------------------------------------------------

def _out_csr(road_from, n_nodes):
    order = np.argsort(road_from, kind="stable").astype(np.int32)
    cnt = np.bincount(road_from, minlength=n_nodes)
    start = np.zeros(n_nodes + 1, np.int64)
    start[1:] = np.cumsum(cnt)
    return start, order


def _reverse_road(road_from, road_to, n_nodes):
    key = road_from.astype(np.int64) * n_nodes + road_to
    rkey = road_to.astype(np.int64) * n_nodes + road_from
    order = np.argsort(key)
    pos = np.searchsorted(key[order], rkey)
    pos = np.clip(pos, 0, key.shape[0] - 1)
    rev = order[pos].astype(np.int32)
    rev[key[order][pos] != rkey] = -1
    return rev


def _random_walk_routes(rng, first_road, road_from, road_to, n_nodes, hops):
    """Routes of exactly ``hops`` roads starting with ``first_road``; each
    next road leaves the current road's end node, avoiding an immediate
    U-turn unless the node is a dead end."""
    start, order = _out_csr(road_from, n_nodes)
    rev = _reverse_road(road_from, road_to, n_nodes)
    n = first_road.shape[0]
    routes = np.empty((n, hops), np.int32)
    cur = first_road.astype(np.int64)
    routes[:, 0] = cur
    for h in range(1, hops):
        node = road_to[cur]
        deg = start[node + 1] - start[node]
        pick = start[node] + (rng.random(n) * deg).astype(np.int64)
        nxt = order[pick].astype(np.int64)
        uturn = (nxt == rev[cur]) & (deg > 1)
        alt = start[node] + ((pick - start[node] + 1) % np.maximum(deg, 1))
        nxt = np.where(uturn, order[alt], nxt)
        routes[:, h] = nxt
        cur = nxt
    off = np.arange(n + 1, dtype=np.int64) * hops
    return off, routes.ravel()


def _place_on_lanes(rng, lane_len, n_target, min_spacing=11.0):
    """Spread ``n_target`` vehicles over lanes in proportion to length, evenly
    spaced with +-20 % jitter; front-to-front spacing stays above 0.6 of the
    lane's spacing, which is >= min_spacing."""
    total = float(lane_len.astype(np.float64).sum())
    dens = n_target / total
    cnt = np.floor(lane_len * dens).astype(np.int64)
    cap = np.floor(lane_len / min_spacing).astype(np.int64)
    cnt = np.minimum(cnt, cap)
    short = n_target - int(cnt.sum())
    if short > 0:
        room = cap - cnt
        cand = np.repeat(np.arange(lane_len.shape[0]), np.maximum(room, 0))
        add = rng.choice(cand, size=min(short, cand.shape[0]), replace=False)
        np.add.at(cnt, add, 1)
    lane = np.repeat(np.arange(lane_len.shape[0], dtype=np.int32), cnt)
    first = np.repeat(np.cumsum(cnt) - cnt, cnt)
    j = np.arange(lane.shape[0]) - first
    sp = lane_len[lane] / np.maximum(cnt[lane], 1)
    s = (j + 0.5 + rng.uniform(-0.2, 0.2, size=lane.shape[0])) * sp
    return lane, s.astype(np.float32)


def _placed_speeds(rng, v0, vlim):
    return (np.minimum(v0, vlim) * rng.uniform(0.3, 1.0, size=v0.shape[0])).astype(np.float32)


def _city_network(side: int, target_undirected: int, seed: int):
    """Jittered side x side lattice, random spanning tree plus extra lattice
    links up to target_undirected, two roads per link with 1-4 lanes per
    direction (P = .80, .12, .05, .03), log-normal lengths (median 150 m,
    sigma 0.75, clipped to [20, 2000] m), signals at nodes of degree >= 3."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import minimum_spanning_tree

    rng = np.random.default_rng(seed)
    nn = side * side
    ii, jj = np.meshgrid(np.arange(side), np.arange(side), indexing="ij")
    node_x = (jj.ravel() * 150.0 + rng.uniform(-30, 30, nn)).astype(np.float64)
    node_y = (ii.ravel() * 150.0 + rng.uniform(-30, 30, nn)).astype(np.float64)
    u = (ii * side + jj)
    e_h = np.stack([u[:, :-1].ravel(), u[:, 1:].ravel()], 1)
    e_v = np.stack([u[:-1, :].ravel(), u[1:, :].ravel()], 1)
    edges = np.concatenate([e_h, e_v]).astype(np.int64)
    w = rng.random(edges.shape[0]) + 1e-3
    g = coo_matrix((w, (edges[:, 0], edges[:, 1])), shape=(nn, nn)).tocsr()
    mst = minimum_spanning_tree(g).tocoo()
    tree = set(zip(np.minimum(mst.row, mst.col).tolist(), np.maximum(mst.row, mst.col).tolist()))
    in_tree = np.array([(int(a), int(b)) in tree for a, b in edges])
    extra_n = max(0, target_undirected - int(in_tree.sum()))
    extra = rng.choice(np.flatnonzero(~in_tree), size=extra_n, replace=False)
    keep = np.concatenate([np.flatnonzero(in_tree), np.sort(extra)])
    und = edges[keep]
    ne = und.shape[0]
    lanes_e = rng.choice([1, 2, 3, 4], size=ne, p=[0.80, 0.12, 0.05, 0.03]).astype(np.int32)
    len_e = np.clip(np.exp(rng.normal(math.log(150.0), 0.75, size=ne)), 20.0, 2000.0)
    vlim_e = SPEED_LIMITS[rng.integers(0, 3, size=ne)]
    rf = np.empty(2 * ne, np.int32)
    rt = np.empty(2 * ne, np.int32)
    rf[0::2], rt[0::2] = und[:, 0], und[:, 1]
    rf[1::2], rt[1::2] = und[:, 1], und[:, 0]
    rl = np.repeat(len_e, 2).astype(np.float32)
    rn = np.repeat(lanes_e, 2)
    rv = np.repeat(vlim_e, 2)
    deg = np.bincount(rt, minlength=nn)
    signalised = deg >= 3
    cyc = np.where(signalised, 60, 0).astype(np.int32)
    ph = np.where(signalised, 30, 0).astype(np.int32)
    off = np.where(signalised, rng.integers(0, 60, size=nn), 0).astype(np.int32)
    grp = _heading_groups(node_x, node_y, rf, rt, signalised)

    return node_x, node_y, rf, rt, rl, rn, rv, cyc, ph, off, grp


def city_snapshot(n_veh: int = 2_000_000, *, side: int = 200, target_undirected: int = 46_000,
                  hops: int = 64, seed: int = NETWORK_SEED, demand_seed: int = DEMAND_SEED,
                  param_seed: int = PARAM_SEED, params=None) -> Scenario:
    """City-scale synthetic network with vehicles already on the road.

    ``side`` x ``side`` jittered lattice (40k nodes at side 200); a random
    spanning tree of the lattice plus random extra lattice links up to
    ``target_undirected`` links keeps it connected and planar.  Each link is
    two roads with 1-4 lanes per direction drawn with P = (.80, .12, .05, .03)
    and a log-normal length (median 150 m, sigma 0.75, clipped to
    [20, 2000] m).  Nodes of degree >= 3 carry fixed-time signals (60 s cycle,
    30 s phases, random offsets).  ``n_veh`` vehicles are pre-placed over all
    lanes in proportion to lane length, each on a ``hops``-road random-walk
    route so that arrivals stay rare over a timed window.
    """
    node_x, node_y, rf, rt, rl, rn, rv, cyc, ph, off, grp = _city_network(
        side, target_undirected, seed)
    nn = side * side
    lane0, n_lanes, lane_road = _lane_layout(rn)
    rng_d = np.random.default_rng(demand_seed)
    lane_len = rl[lane_road].astype(np.float64)
    lane, s = _place_on_lanes(rng_d, lane_len, n_veh)
    n = lane.shape[0]
    first_road = lane_road[lane]
    roff, rflat = _random_walk_routes(rng_d, first_road, rf, rt, nn, hops)
    v0 = _desired_speeds(np.random.default_rng(param_seed), n)
    vlim_l = rv[lane_road]
    v = _placed_speeds(rng_d, v0, vlim_l[lane])
    ids = rng_d.permutation(n).astype(np.uint32)
    placement = (np.ones(n, np.uint8), lane, s, v, np.zeros(n, np.float32), np.zeros(n, np.int32))
    return _make("city", node_x, node_y, rf, rt, rl, rn, rv, cyc, ph, off, grp, ids,
                 np.zeros(n, np.int32), v0, roff, rflat, placement, params,
                 meta=dict(seed=seed, demand_seed=demand_seed, side=side))


_scen_lib = None


def _scen():
    """ctypes handle of the generator's host helper (shortest-path routes)."""
    global _scen_lib
    if _scen_lib is None:
        import ctypes as C
        from .build import ensure_scen
        L = C.CDLL(ensure_scen())
        vp = C.c_void_p
        L.scen_next_roads.argtypes = [C.c_int32, C.c_int32, vp, vp, vp, C.c_int32, vp, vp,
                                      C.c_int32]
        L.scen_walk_routes.argtypes = [C.c_int32, vp, vp, C.c_int64, vp, vp, vp, C.c_int32, vp,
                                       vp, vp, C.c_int32]
        _scen_lib = L
    return _scen_lib


def _routes_to(n_nodes, road_from, road_to, road_length, orig, dest, max_hops, threads=None):
    """Shortest-path routes (road lists, packed) from orig[i] to dest[i]: one
    Dijkstra per distinct destination over the reversed road graph (host
    helper, OpenMP)."""
    import os
    p = lambda a: a.ctypes.data_as(__import__("ctypes").c_void_p)   # noqa: E731
    L = _scen()
    thr = threads or int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
    rf = np.ascontiguousarray(road_from, np.int32)
    rt = np.ascontiguousarray(road_to, np.int32)
    rl = np.ascontiguousarray(road_length, np.float32)
    dests, dk = np.unique(np.asarray(dest, np.int32), return_inverse=True)
    dests = dests.astype(np.int32)
    dk = dk.astype(np.int32)
    org = np.ascontiguousarray(orig, np.int32)
    nxt = np.empty((dests.shape[0], n_nodes), np.int32)
    L.scen_next_roads(n_nodes, rf.shape[0], p(rf), p(rt), p(rl), dests.shape[0], p(dests),
                      p(nxt), thr)
    n = org.shape[0]
    ln = np.empty(n, np.int32)
    if L.scen_walk_routes(n_nodes, p(rt), p(nxt), n, p(org), p(dests), p(dk), max_hops, p(ln),
                          None, None, thr) != 0:
        raise ValueError("a trip cannot reach its destination within max_hops roads")
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum(ln)
    flat = np.empty(int(off[-1]), np.int32)
    L.scen_walk_routes(n_nodes, p(rt), p(nxt), n, p(org), p(dests), p(dk), max_hops, None,
                       p(off), p(flat), thr)
    return off, flat


def city_demand(n_veh: int = 2_000_000, *, side: int = 200, target_undirected: int = 46_000,
                horizon: int = 3600, zone_side: int = 20, deterrence: float = 3000.0,
                dest_per_zone: int = 8, seed: int = NETWORK_SEED,
                demand_seed: int = DEMAND_SEED, param_seed: int = PARAM_SEED,
                params=None) -> Scenario:
    """The city network of city_snapshot with its travel demand: n_veh trips
    between zone_side x zone_side zones (square blocks of the lattice) drawn
    from a gravity model -- P(o, d) proportional to m_o m_d exp(-d_od /
    deterrence), zone mass m = node count, d_od the distance between zone
    centroids -- departing at uniform steps in [0, horizon) and following
    shortest paths by length.  A trip starts at a uniform node of its origin
    zone and ends at one of dest_per_zone fixed nodes of its destination zone
    (distinct from its start), which bounds the shortest-path work to one
    tree per such node.  Vehicles wait at the start of their first road until
    they can enter (no pre-placement)."""
    node_x, node_y, rf, rt, rl, rn, rv, cyc, ph, off, grp = _city_network(
        side, target_undirected, seed)
    nn = side * side
    rng = np.random.default_rng(demand_seed)
    blk = side // zone_side
    ii, jj = np.divmod(np.arange(nn), side)
    zone = (np.minimum(ii // blk, zone_side - 1) * zone_side +
            np.minimum(jj // blk, zone_side - 1))
    nz = zone_side * zone_side
    mass = np.bincount(zone, minlength=nz).astype(np.float64)
    cx = np.bincount(zone, weights=node_x, minlength=nz) / mass
    cy = np.bincount(zone, weights=node_y, minlength=nz) / mass
    dist = np.hypot(cx[:, None] - cx[None, :], cy[:, None] - cy[None, :])
    w = mass[:, None] * mass[None, :] * np.exp(-dist / deterrence)
    pair = rng.choice(nz * nz, size=n_veh, p=(w / w.sum()).ravel())
    oz, dz = np.divmod(pair, nz)
    order = np.argsort(zone, kind="stable")
    zstart = np.zeros(nz + 1, np.int64)
    zstart[1:] = np.cumsum(np.bincount(zone, minlength=nz))
    dnodes = np.stack([order[zstart[z] + rng.choice(zstart[z + 1] - zstart[z], dest_per_zone,
                                                    replace=False)] for z in range(nz)])
    dest = dnodes[dz, rng.integers(0, dest_per_zone, size=n_veh)].astype(np.int32)
    orig = order[zstart[oz] + rng.integers(0, zstart[oz + 1] - zstart[oz])].astype(np.int32)
    same = orig == dest
    while same.any():
        k = np.flatnonzero(same)
        orig[k] = order[zstart[oz[k]] + rng.integers(0, zstart[oz[k] + 1] - zstart[oz[k]])]
        same = orig == dest
    depart = np.sort(rng.integers(0, horizon, size=n_veh)).astype(np.int32)
    roff, rflat = _routes_to(nn, rf, rt, rl, orig, dest, 4 * side)
    v0 = _desired_speeds(np.random.default_rng(param_seed), n_veh)
    ids = np.arange(n_veh, dtype=np.uint32)
    return _make("city_demand", node_x, node_y, rf, rt, rl, rn, rv, cyc, ph, off, grp, ids,
                 depart, v0, roff, rflat, None, params,
                 meta=dict(seed=seed, demand_seed=demand_seed, side=side, horizon=horizon,
                           zones=nz, deterrence=deterrence))


def grid_snapshot(n: int, n_veh: int, *, lanes: int = 3, hops: int = 64, seed: int = NETWORK_SEED,
                  demand_seed: int = DEMAND_SEED, param_seed: int = PARAM_SEED,
                  params=None) -> Scenario:
    """A grid with vehicles pre-placed on random-walk routes (parity cases)."""
    rng = np.random.default_rng(seed)
    (nx_, ny_, rf, rt, rl, rn, rv, cyc, ph, off, grp) = _grid_network(n, 200.0, lanes, rng)
    lane0, n_lanes, lane_road = _lane_layout(rn)
    rng_d = np.random.default_rng(demand_seed)
    lane, s = _place_on_lanes(rng_d, rl[lane_road].astype(np.float64), n_veh)
    m = lane.shape[0]
    roff, rflat = _random_walk_routes(rng_d, lane_road[lane], rf, rt, n * n, hops)
    v0 = _desired_speeds(np.random.default_rng(param_seed), m)
    v = _placed_speeds(rng_d, v0, rv[lane_road][lane])
    ids = rng_d.permutation(m).astype(np.uint32)
    placement = (np.ones(m, np.uint8), lane, s, v, np.zeros(m, np.float32), np.zeros(m, np.int32))
    return _make(f"grid{n}x{n}_snapshot", nx_, ny_, rf, rt, rl, rn, rv, cyc, ph, off, grp, ids,
                 np.zeros(m, np.int32), v0, roff, rflat, placement, params)


# ---------------------------------------------------------------------------
# batched scenarios
# ---------------------------------------------------------------------------

def batch_sizes(n_scen: int = 256, *, seed: int = DEMAND_SEED, vmin: float = 1e3,
                vmax: float = 5e4):
    """Vehicle counts log-uniform in [vmin, vmax]; grid side grows with
    log(count) from 4 to 16 so that big demands get big grids."""
    rng = np.random.default_rng(seed + 1000)
    V = np.exp(rng.uniform(math.log(vmin), math.log(vmax), size=n_scen)).astype(np.int64)
    side = np.clip(np.round(4 + 12 * np.log(V / vmin) / math.log(vmax / vmin)), 4, 16)
    return V, side.astype(np.int64)


def batch(n_scen: int = 256, *, horizon: int = 1800, vmin: float = 1e3, vmax: float = 5e4,
          lanes: int = 3, seed: int = NETWORK_SEED, demand_seed: int = DEMAND_SEED,
          param_seed: int = PARAM_SEED, params=None) -> Scenario:
    """Disjoint union of ``n_scen`` independent grid scenarios.

    Scenario ``q`` has V_q vehicles (log-uniform) on a side_q x side_q grid;
    nodes, roads, lanes and vehicle ids are renumbered into one network and
    ``lane_scen`` records which scenario each lane belongs to.
    """
    V, side = batch_sizes(n_scen, seed=demand_seed, vmin=vmin, vmax=vmax)
    parts = []
    node_base = road_base = id_base = 0
    for q in range(n_scen):
        sc = grid(int(side[q]), int(V[q]), lanes=lanes, horizon=horizon, seed=seed * 7919 + q,
                  demand_seed=demand_seed * 7919 + q, param_seed=param_seed * 7919 + q)
        parts.append((sc, node_base, road_base, id_base))
        node_base += sc.n_nodes
        road_base += sc.n_roads
        id_base += sc.n_veh
    cat = lambda f: np.concatenate([f(q, p) for q, p in enumerate(parts)])
    node_x = cat(lambda q, p: p[0].node_x + 5000.0 * (q % 16))
    node_y = cat(lambda q, p: p[0].node_y + 5000.0 * (q // 16))
    rf = cat(lambda q, p: p[0].road_from + p[1])
    rt = cat(lambda q, p: p[0].road_to + p[1])
    rl = cat(lambda q, p: p[0].road_length)
    rn = cat(lambda q, p: p[0].road_nlanes)
    rv = cat(lambda q, p: p[0].lane_vlim[p[0].road_lane0])
    cyc = cat(lambda q, p: p[0].node_cycle)
    ph = cat(lambda q, p: p[0].node_phase)
    off = cat(lambda q, p: p[0].node_offset)
    grp = cat(lambda q, p: p[0].road_group)
    lane_scen = np.concatenate([np.full(p[0].n_lanes, q, np.int32) for q, p in enumerate(parts)])
    ids = cat(lambda q, p: p[0].veh_id.astype(np.int64) + p[3]).astype(np.uint32)
    dep = cat(lambda q, p: p[0].depart)
    v0 = cat(lambda q, p: p[0].v0)
    rflat = cat(lambda q, p: p[0].route_roads + p[2])
    lens = cat(lambda q, p: np.diff(p[0].route_off))
    roff = np.zeros(lens.shape[0] + 1, np.int64)
    roff[1:] = np.cumsum(lens)
    sc = _make("batch", node_x, node_y, rf, rt, rl, rn, rv, cyc, ph, off, grp, ids, dep, v0, roff,
               rflat, None, params, lane_scen=lane_scen, n_scen=n_scen,
               meta=dict(sizes=V.tolist(), sides=side.tolist(), horizon=horizon))
    return sc


# ---------------------------------------------------------------------------
# tiny random networks for brute-force checks
# ---------------------------------------------------------------------------

def toy(seed: int, *, n: int = 3, max_lanes: int = 3, n_placed: int = 40, n_pending: int = 10,
        length_range=(40.0, 120.0), horizon: int = 20, hops: int = 8, params=None) -> Scenario:
    """Small grid with random lane counts and lengths, a random signal plan,
    ``n_placed`` vehicles already on the road (random lanes and positions,
    no overlap) and ``n_pending`` vehicles departing within ``horizon``
    steps."""
    rng = np.random.default_rng(seed)
    (nx_, ny_, rf, rt, rl, rn, rv, cyc, ph, off, grp) = _grid_network(n, 100.0, 1, rng)
    ne = rf.shape[0] // 2
    lanes_e = rng.integers(1, max_lanes + 1, size=ne).astype(np.int32)
    len_e = rng.uniform(*length_range, size=ne).astype(np.float32)
    rn = np.repeat(lanes_e, 2)
    rl = np.repeat(len_e, 2)
    lane0, n_lanes, lane_road = _lane_layout(rn)
    lane_len = rl[lane_road].astype(np.float64)
    # pre-placed vehicles: random lanes, positions drawn on a 7.5 m lattice so
    # that front-to-front distance >= 7.5 > vehicle length
    slots = []
    for l in range(n_lanes):
        m = int(lane_len[l] // 7.5)
        for j in range(m):
            slots.append((l, 7.5 * j + 5.0 + rng.uniform(0.0, 2.4)))
    slots = np.array(slots)
    pick = rng.choice(slots.shape[0], size=min(n_placed, slots.shape[0]), replace=False)
    lane = slots[pick, 0].astype(np.int32)
    s = np.minimum(slots[pick, 1], lane_len[lane] - 0.01).astype(np.float32)
    nP = lane.shape[0]
    roff_p, rflat_p = _random_walk_routes(rng, lane_road[lane], rf, rt, n * n, hops)
    first_pending = rng.integers(0, rf.shape[0], size=n_pending)
    roff_q, rflat_q = _random_walk_routes(rng, first_pending, rf, rt, n * n, hops)
    m = nP + n_pending
    v0 = _desired_speeds(rng, m)
    v = np.zeros(m, np.float32)
    v[:nP] = _placed_speeds(rng, v0[:nP], rv[lane_road][lane])
    placed = np.zeros(m, np.uint8)
    placed[:nP] = 1
    lane_all = np.full(m, -1, np.int32)
    lane_all[:nP] = lane
    s_all = np.zeros(m, np.float32)
    s_all[:nP] = s
    a_all = np.zeros(m, np.float32)
    a_all[:nP] = rng.uniform(-2.0, 1.0, size=nP).astype(np.float32)
    depart = np.zeros(m, np.int32)
    depart[nP:] = rng.integers(0, horizon, size=n_pending)
    roff = np.concatenate([roff_p, roff_q[1:] + roff_p[-1]])
    rflat = np.concatenate([rflat_p, rflat_q])
    ids = rng.permutation(m).astype(np.uint32) * 3 + 7
    placement = (placed, lane_all, s_all, v, a_all, np.zeros(m, np.int32))
    return _make(f"toy{seed}", nx_, ny_, rf, rt, rl, rn, rv, cyc, ph, off, grp, ids, depart, v0,
                 roff, rflat, placement, params)


CONFIGS = {
    "intersection": "single signalised 4-way junction, 2 lanes x 500 m arms, 200 vehicles, 3600 steps",
    "grid10": "10x10 grid, 200 m links, 3 lanes/dir, 20k vehicles, 3600 steps",
    "city": "city-scale synthetic network ~40k nodes / ~120k lanes, 2M vehicles",
    "batch": "256 independent grids 4x4..16x16, 1k-50k vehicles each, 1800 steps",
}
