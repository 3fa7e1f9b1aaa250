"""ctypes binding of the CPU oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
from typing import Dict

import numpy as np

from .build import ensure_built

_lib = None


class OrcInput(C.Structure):
    _fields_ = [
        ("n_nodes", C.c_int32), ("n_roads", C.c_int32), ("n_lanes", C.c_int32),
        ("n_scen", C.c_int32),
        ("road_from", C.c_void_p), ("road_to", C.c_void_p), ("road_nlanes", C.c_void_p),
        ("road_lane0", C.c_void_p), ("road_length", C.c_void_p), ("lane_vlim", C.c_void_p),
        ("lane_scen", C.c_void_p), ("node_x", C.c_void_p), ("node_y", C.c_void_p),
        ("node_cycle", C.c_void_p), ("node_phase", C.c_void_p), ("node_offset", C.c_void_p),
        ("road_group", C.c_void_p),
        ("n_veh", C.c_int32),
        ("veh_id", C.c_void_p), ("depart", C.c_void_p), ("v0", C.c_void_p),
        ("route_off", C.c_void_p), ("route_roads", C.c_void_p), ("placed", C.c_void_p),
        ("lane", C.c_void_p), ("cursor", C.c_void_p), ("s", C.c_void_p), ("v", C.c_void_p),
        ("a", C.c_void_p),
        ("dt", C.c_float), ("a_max", C.c_float), ("b", C.c_float), ("s0", C.c_float),
        ("T", C.c_float), ("length", C.c_float), ("b_max", C.c_float), ("b_safe", C.c_float),
        ("politeness", C.c_float), ("a_thr", C.c_float), ("p_lc", C.c_float),
        ("d_look", C.c_float),
        ("h_look", C.c_int32), ("t0", C.c_int32), ("seed", C.c_uint64),
        ("mode", C.c_int32), ("mlp_theta", C.c_void_p), ("mlp_norm", C.c_void_p),
        ("road_internal", C.c_void_p), ("lane_succ_off", C.c_void_p), ("lane_succ", C.c_void_p),
        ("lane_conf_off", C.c_void_p), ("lane_conf", C.c_void_p), ("lane_conf_feed", C.c_void_p),
        ("b_mand", C.c_float), ("tau_yield", C.c_float),
    ]


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(ensure_built())
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(OrcInput)]
        L.orc_error.restype = C.c_char_p
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_step.argtypes = [C.c_void_p, C.c_int32]
        L.orc_set_threads.argtypes = [C.c_void_p, C.c_int32]
        L.orc_max_threads.restype = C.c_int32
        L.orc_n_active.argtypes = [C.c_void_p]
        L.orc_n_active.restype = C.c_int32
        L.orc_time.argtypes = [C.c_void_p]
        L.orc_time.restype = C.c_int64
        L.orc_pending.argtypes = [C.c_void_p]
        L.orc_pending.restype = C.c_int32
        L.orc_read.argtypes = [C.c_void_p] + [C.c_void_p] * 6
        L.orc_read_debug.argtypes = [C.c_void_p] + [C.c_void_p] * 6
        L.orc_read_debug.restype = C.c_int32
        L.orc_counters.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_road_stats.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_set_signal_phase.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
        L.orc_set_signal_phase.restype = C.c_int
        L.orc_set_lane_vlim.argtypes = [C.c_void_p, C.c_int32, C.c_float]
        L.orc_set_lane_closed.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
        L.orc_set_lane_closed.restype = C.c_int
        L.orc_set_lane_turns.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                         C.c_void_p]
        L.orc_set_lane_turns.restype = C.c_int
        L.orc_read_trips.argtypes = [C.c_void_p] + [C.c_void_p] * 4
        L.orc_positions.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_positions.restype = C.c_int
        L.orc_mlp_sq.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_read_mlp_inputs.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_read_mlp_inputs.restype = C.c_int32
        L.orc_mlp_candidates.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_float,
                                         C.c_float, C.c_int32, C.c_void_p, C.c_void_p]
        L.orc_mlp_candidates.restype = C.c_int32
        L.orc_mlp_candidates_batch.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                               C.c_float, C.c_float, C.c_int32, C.c_void_p,
                                               C.c_void_p, C.c_void_p, C.c_int32]
        L.orc_mlp_forward.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_mlp_forward.restype = C.c_double
        L.orc_philox4x32_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_idm.restype = C.c_float
        L.orc_idm.argtypes = [C.c_float, C.c_float, C.c_int, C.c_float, C.c_float, C.c_float,
                              C.c_float, C.c_float, C.c_float, C.c_float]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


COUNTER_NAMES = ("inserted", "insert_fail", "arrived", "trip_time", "clamps", "lane_changes",
                 "veh_steps", "mlp_eval", "mlp_fallback")


class OracleSim:
    """One oracle simulation built from a :class:`Scenario`."""

    def __init__(self, sc):
        L = lib()
        self._keep = []

        def arr(x, dt):
            a = np.ascontiguousarray(x, dtype=dt)
            self._keep.append(a)
            return _p(a)

        p = sc.params
        inp = OrcInput()
        inp.n_nodes, inp.n_roads, inp.n_lanes, inp.n_scen = sc.n_nodes, sc.n_roads, sc.n_lanes, sc.n_scen
        inp.road_from = arr(sc.road_from, np.int32)
        inp.road_to = arr(sc.road_to, np.int32)
        inp.road_nlanes = arr(sc.road_nlanes, np.int32)
        inp.road_lane0 = arr(sc.road_lane0, np.int32)
        inp.road_length = arr(sc.road_length, np.float32)
        inp.lane_vlim = arr(sc.lane_vlim, np.float32)
        inp.lane_scen = arr(sc.lane_scen, np.int32)
        inp.node_x = arr(sc.node_x, np.float64)
        inp.node_y = arr(sc.node_y, np.float64)
        inp.node_cycle = arr(sc.node_cycle, np.int32)
        inp.node_phase = arr(sc.node_phase, np.int32)
        inp.node_offset = arr(sc.node_offset, np.int32)
        inp.road_group = arr(sc.road_group, np.int8)
        inp.n_veh = sc.n_veh
        inp.veh_id = arr(sc.veh_id, np.uint32)
        inp.depart = arr(sc.depart, np.int32)
        inp.v0 = arr(sc.v0, np.float32)
        inp.route_off = arr(sc.route_off, np.int64)
        inp.route_roads = arr(sc.route_roads, np.int32)
        inp.placed = arr(sc.placed, np.uint8)
        inp.lane = arr(sc.lane, np.int32)
        inp.cursor = arr(sc.cursor, np.int32)
        inp.s = arr(sc.s, np.float32)
        inp.v = arr(sc.v, np.float32)
        inp.a = arr(sc.a, np.float32)
        for k in ("dt", "a_max", "b", "s0", "T", "length", "b_max", "b_safe", "politeness",
                  "a_thr", "p_lc", "d_look"):
            setattr(inp, k, float(p[k]))
        inp.h_look = int(p["h_look"])
        inp.t0 = int(p["t0"])
        inp.seed = int(p["seed"])
        inp.b_mand = float(p.get("b_mand", 1.0))
        inp.tau_yield = float(p.get("tau_yield", 3.0))
        if sc.lane_succ_off is not None:
            inp.road_internal = arr(sc.road_internal, np.uint8)
            inp.lane_succ_off = arr(sc.lane_succ_off, np.int32)
            inp.lane_succ = arr(sc.lane_succ, np.int32)
            inp.lane_conf_off = arr(sc.lane_conf_off, np.int32)
            inp.lane_conf = arr(sc.lane_conf, np.int32)
            inp.lane_conf_feed = arr(sc.lane_conf_feed, np.int32)
        mlp_cfg = p.get("mlp")
        if mlp_cfg is not None:
            inp.mode = 1
            inp.mlp_theta = arr(mlp_cfg["theta"], np.float32)
            inp.mlp_norm = arr(mlp_cfg["norm"], np.float32)
        h = L.orc_create(C.byref(inp))
        if not h:
            raise ValueError("oracle create failed: " + L.orc_error().decode())
        self._h = h
        self.n_scen = sc.n_scen
        self.n_roads = sc.n_roads
        self.n_veh = sc.n_veh

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def step(self, n: int = 1):
        lib().orc_step(self._h, int(n))

    def set_threads(self, n: int):
        """OpenMP threads of the update and merge loops (results do not
        depend on it)."""
        lib().orc_set_threads(self._h, int(n))

    @property
    def n_active(self) -> int:
        return int(lib().orc_n_active(self._h))

    @property
    def t(self) -> int:
        return int(lib().orc_time(self._h))

    @property
    def pending(self) -> int:
        return int(lib().orc_pending(self._h))

    def state(self) -> Dict[str, np.ndarray]:
        n = self.n_active
        out = dict(id=np.empty(n, np.uint32), lane=np.empty(n, np.int32),
                   s=np.empty(n, np.float32), v=np.empty(n, np.float32),
                   a=np.empty(n, np.float32), cursor=np.empty(n, np.int32))
        lib().orc_read(self._h, _p(out["id"]), _p(out["lane"]), _p(out["s"]), _p(out["v"]),
                       _p(out["a"]), _p(out["cursor"]))
        return out

    def debug(self) -> Dict[str, np.ndarray]:
        cap = max(self.n_active, 1) * 4 + 1024
        d = dict(id=np.empty(cap, np.uint32), leader=np.empty(cap, np.uint32),
                 flags=np.empty(cap, np.int32), margin=np.empty(cap, np.float32),
                 t_leader=np.empty(cap, np.uint32), t_follower=np.empty(cap, np.uint32))
        n = lib().orc_read_debug(self._h, _p(d["id"]), _p(d["leader"]), _p(d["flags"]),
                                 _p(d["margin"]), _p(d["t_leader"]), _p(d["t_follower"]))
        return {k: v[:n].copy() for k, v in d.items()}

    def counters(self):
        c = np.zeros((self.n_scen, len(COUNTER_NAMES)), np.int64)
        sv = np.zeros(self.n_scen, np.float64)
        lib().orc_counters(self._h, _p(c), _p(sv))
        return c, sv

    def set_signal_phase(self, nodes, phases):
        for j, p in zip(np.atleast_1d(nodes), np.atleast_1d(phases)):
            if lib().orc_set_signal_phase(self._h, int(j), int(p)) != 0:
                raise ValueError(f"node {j} has no signal")

    def set_lane_vlim(self, lanes, vlims):
        for l, v in zip(np.atleast_1d(lanes), np.atleast_1d(vlims)):
            lib().orc_set_lane_vlim(self._h, int(l), float(np.float32(v)))

    def set_lane_closed(self, lanes, closed):
        ln = np.ascontiguousarray(np.atleast_1d(lanes), np.int32)
        cl = np.ascontiguousarray(np.atleast_1d(closed), np.int32)
        if lib().orc_set_lane_closed(self._h, int(ln.shape[0]), _p(ln), _p(cl)) != 0:
            raise ValueError("lane out of range, or a road would have no open lane")

    def set_lane_turns(self, lanes, roads, allowed):
        ln = np.ascontiguousarray(np.atleast_1d(lanes), np.int32)
        rd = np.ascontiguousarray(np.atleast_1d(roads), np.int32)
        al = np.ascontiguousarray(np.atleast_1d(allowed), np.int32)
        if lib().orc_set_lane_turns(self._h, int(ln.shape[0]), _p(ln), _p(rd), _p(al)) != 0:
            raise ValueError("no junction lanes, or a lane without a successor on the road")

    def road_stats(self):
        """(vehicles per road, mean speed per road)."""
        cnt = np.empty(self.n_roads, np.int32)
        mv = np.empty(self.n_roads, np.float32)
        lib().orc_road_stats(self._h, _p(cnt), _p(mv))
        return cnt, mv

    def trips(self):
        """Per vehicle in ascending id order: dict of id, status (0 waiting,
        1 on the network, 2 arrived), travel time (steps) and distance (m)."""
        n = self.n_veh
        out = dict(id=np.empty(n, np.uint32), status=np.empty(n, np.int32),
                   travel=np.empty(n, np.int32), distance=np.empty(n, np.float64))
        lib().orc_read_trips(self._h, _p(out["id"]), _p(out["status"]), _p(out["travel"]),
                             _p(out["distance"]))
        return out

    def positions(self):
        """(x, y, heading) per state row."""
        n = self.n_active
        x, y, h = (np.empty(n, np.float64) for _ in range(3))
        if lib().orc_positions(self._h, _p(x), _p(y), _p(h)) != 0:
            raise RuntimeError("oracle created without node coordinates")
        return x, y, h

    def mlp_inputs(self):
        """Network mode: (raw closure inputs [n, 8], use [n]: 1 evaluated, 2
        outside the envelope) of the last step, in the order of debug()."""
        n = max(self.n_active, 1) * 4 + 1024
        f = np.empty((n, 8), np.float32)
        u = np.empty(n, np.int8)
        k = lib().orc_read_mlp_inputs(self._h, _p(f), _p(u))
        return f[:k].copy(), u[:k].copy()

    def mlp_sq(self):
        out = np.zeros(self.n_scen, np.float64)
        lib().orc_mlp_sq(self._h, _p(out))
        return out


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def mlp_forward(theta, z):
    th = np.ascontiguousarray(theta, dtype=np.float32)
    zz = np.ascontiguousarray(z, dtype=np.float32)
    return float(lib().orc_mlp_forward(_p(th), _p(zz)))


def mlp_candidates(theta, norm, feat, lo, hi, cap=64, threads=None):
    """Every output an FP32 evaluation of the closure may correctly give for
    each row of raw inputs feat[n, 8], limited to [lo, hi] (oracle
    orc_mlp_candidates): (outputs [n, cap] with the oracle's own value in
    column 0, count [n], info [n, 4] = tied units in layers 1 and 2, input
    combinations, first tied unit)."""
    th = np.ascontiguousarray(theta, dtype=np.float32)
    nm = np.ascontiguousarray(norm, dtype=np.float32)
    f = np.ascontiguousarray(feat, dtype=np.float32).reshape(-1, 8)
    n = f.shape[0]
    out = np.full((n, cap), np.nan, np.float64)
    cnt = np.zeros(n, np.int32)
    info = np.zeros((n, 4), np.int32)
    lib().orc_mlp_candidates_batch(_p(th), _p(nm), n, _p(f), float(lo), float(hi), int(cap),
                                   _p(out), _p(cnt), _p(info),
                                   int(threads if threads else max_threads()))
    return out, cnt, info


def idm(v, v0e, has_leader, v_lead, gap, a_max=2.0, s0=2.0, T=1.5, b=4.5, b_max=9.0):
    """The oracle's FP32 IDM acceleration (reciprocal of 2 sqrt(a_max b)
    formed in double, as in the simulation)."""
    inv_tsab = float(np.float32(1.0 / (2.0 * np.sqrt(a_max * b))))
    return float(lib().orc_idm(v, v0e, int(has_leader), v_lead, gap, a_max, inv_tsab, s0, T,
                               b_max))


def max_threads() -> int:
    """Threads OpenMP uses by default on this host."""
    return int(lib().orc_max_threads())
