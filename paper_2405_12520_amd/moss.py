"""Python binding of libmoss (ctypes): argument marshalling only.

Every simulation step runs in the HIP kernels of ``libmoss.so``; this module
builds the C structs of ``include/moss.h`` from numpy arrays, allocates the
device workspace as a torch tensor and passes torch's current HIP stream.
It raises if the library has not been built -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libmoss.so")

MOSS_OK, MOSS_EINVAL, MOSS_ENOMEM, MOSS_EDEVICE, MOSS_ESTATE = 0, -1, -2, -3, -4
MOSS_FLAG_DEBUG = 1
MOSS_FLAG_TRACE = 2
MOSS_MODE_IDM, MOSS_MODE_MLP = 0, 1
MLP_PARAMS, MLP_NORM = 4801, 32
MLP_STATIC_MAX_SAMPLES = 8192       # MOSS_MLP_STATIC_MAX_SAMPLES
COUNTER_NAMES = ("inserted", "insert_fail", "arrived", "trip_time", "clamps", "lane_changes",
                 "veh_steps", "mlp_eval", "mlp_fallback")
NONE = 0xFFFFFFFF

vp = C.c_void_p


class moss_network(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_roads", C.c_int32), ("n_lanes", C.c_int32),
                ("n_scen", C.c_int32), ("road_from", vp), ("road_to", vp), ("road_nlanes", vp),
                ("road_lane0", vp), ("road_length", vp), ("lane_vlim", vp), ("lane_scen", vp),
                ("node_x", vp), ("node_y", vp), ("road_internal", vp), ("lane_succ_off", vp),
                ("lane_succ", vp), ("lane_conf_off", vp), ("lane_conf", vp),
                ("lane_conf_feed", vp)]


class moss_signals(C.Structure):
    _fields_ = [("node_cycle", vp), ("node_phase", vp), ("node_offset", vp), ("road_group", vp)]


class moss_vehicles(C.Structure):
    _fields_ = [("n", C.c_int32), ("id", vp), ("depart", vp), ("v0", vp), ("route_off", vp),
                ("route_roads", vp), ("placed", vp), ("lane", vp), ("cursor", vp), ("s", vp),
                ("v", vp), ("a", vp)]


class moss_params(C.Structure):
    _fields_ = [("dt", C.c_float), ("a_max", C.c_float), ("b", C.c_float), ("s0", C.c_float),
                ("T", C.c_float), ("length", C.c_float), ("b_max", C.c_float),
                ("b_safe", C.c_float), ("politeness", C.c_float), ("a_thr", C.c_float),
                ("p_lc", C.c_float), ("d_look", C.c_float), ("h_look", C.c_int32),
                ("t0", C.c_int32), ("seed", C.c_uint64), ("flags", C.c_uint32),
                ("mode", C.c_int32), ("mlp_theta", vp), ("mlp_norm", vp),
                ("b_mand", C.c_float), ("tau_yield", C.c_float)]


class moss_state_out(C.Structure):
    _fields_ = [("capacity", C.c_int32), ("device", C.c_int32), ("id", vp), ("lane", vp),
                ("s", vp), ("v", vp), ("a", vp), ("cursor", vp), ("n", C.c_int32),
                ("t", C.c_int64)]


class moss_launch(C.Structure):
    _fields_ = [("graph_steps", C.c_int32), ("update_blocks", C.c_int32),
                ("scatter_blocks", C.c_int32), ("xcd_remap", C.c_int32)]


LAUNCH_FIELDS = tuple(f for f, _ in moss_launch._fields_)

EXPORTS = ("moss_query_workspace", "moss_create", "moss_step", "moss_read_state",
           "moss_read_counters", "moss_read_pending", "moss_read_debug", "moss_step_timed",
           "moss_kernel_name",
           "moss_mlp_scratch_bytes", "moss_mlp_grad", "moss_mlp_grad_static", "moss_mlp_adam", "moss_mlp_predict",
           "moss_read_trace", "moss_read_mlp_error", "moss_set_launch", "moss_get_launch",
           "moss_read_road_stats", "moss_read_positions", "moss_read_trips",
           "moss_set_signal_phase",
           "moss_set_lane_vlim", "moss_set_lane_closed", "moss_set_lane_turns",
           "moss_destroy", "moss_last_error")

_lib = None


def load(path: str = LIB_PATH):
    """Loads libmoss.so; raises FileNotFoundError if it was not built.

    torch is imported first: its HIP runtime must be the one the library
    binds to, or the process would hold two runtimes and device pointers from
    torch would be foreign to the library."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads torch's HIP runtime before the library)
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: build it with paper_2405_12520_amd.build")
    L = C.CDLL(path)
    L.moss_query_workspace.argtypes = [C.POINTER(moss_network), C.POINTER(moss_signals),
                                       C.POINTER(moss_vehicles), C.POINTER(moss_params),
                                       C.POINTER(C.c_size_t)]
    L.moss_create.argtypes = [C.POINTER(moss_network), C.POINTER(moss_signals),
                              C.POINTER(moss_vehicles), C.POINTER(moss_params), vp, C.c_size_t,
                              vp, C.POINTER(vp)]
    L.moss_step.argtypes = [vp, C.c_int32]
    L.moss_read_state.argtypes = [vp, C.POINTER(moss_state_out)]
    L.moss_read_counters.argtypes = [vp, vp, vp, C.POINTER(C.c_uint32)]
    L.moss_read_pending.argtypes = [vp, C.c_int32, vp, C.POINTER(C.c_int32)]
    L.moss_read_debug.argtypes = [vp, C.c_int32, vp, vp, vp, vp, vp, vp,
                                  C.POINTER(C.c_int32)]
    L.moss_step_timed.argtypes = [vp, C.c_int32, vp, C.c_int32, C.POINTER(C.c_int32)]
    L.moss_kernel_name.argtypes = [C.c_int32]
    L.moss_destroy.argtypes = [vp]
    L.moss_mlp_scratch_bytes.argtypes = [C.c_int32]
    L.moss_mlp_grad.argtypes = [vp, vp, vp, C.c_int32, vp, vp, C.c_int32, C.c_float, C.c_float,
                                vp, vp, vp, C.c_size_t, vp]
    L.moss_mlp_grad_static.argtypes = [vp, vp, vp, C.c_int32, vp, vp, C.c_int32, C.c_float,
                                       C.c_float, vp, vp, vp]
    L.moss_mlp_adam.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_float, C.c_float, C.c_float,
                                C.c_float, vp]
    L.moss_mlp_predict.argtypes = [vp, C.c_int32, vp, vp, vp, vp]
    L.moss_read_trace.argtypes = [vp, C.c_int32, C.c_int32, vp, vp, C.POINTER(C.c_int32)]
    L.moss_read_mlp_error.argtypes = [vp, vp]
    L.moss_set_launch.argtypes = [vp, C.POINTER(moss_launch)]
    L.moss_read_road_stats.argtypes = [vp, C.c_int32, vp, vp]
    L.moss_set_signal_phase.argtypes = [vp, vp, vp, C.c_int32]
    L.moss_set_lane_vlim.argtypes = [vp, vp, vp, C.c_int32]
    L.moss_set_lane_closed.argtypes = [vp, vp, vp, C.c_int32]
    L.moss_set_lane_turns.argtypes = [vp, vp, vp, vp, C.c_int32]
    L.moss_read_positions.argtypes = [vp, C.c_int32, C.c_int32, vp, vp, vp, C.POINTER(C.c_int32)]
    L.moss_get_launch.argtypes = [vp, C.POINTER(moss_launch)]
    L.moss_read_trips.argtypes = [vp, C.c_int32, C.c_int32, vp, vp, vp, vp,
                                  C.POINTER(C.c_int32)]
    for f in EXPORTS:
        getattr(L, f).restype = C.c_char_p if f in ("moss_last_error", "moss_kernel_name") \
            else C.c_int
    L.moss_mlp_scratch_bytes.restype = C.c_size_t
    _lib = L
    return L


class MossError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libmoss error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != MOSS_OK:
        raise MossError(rc, load().moss_last_error().decode())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(vp)


def marshal(sc, debug: bool = False, trace: bool = False):
    """C structs (and the numpy arrays they point to) for a Scenario."""
    keep = []

    def arr(x, dt):
        a = np.ascontiguousarray(x, dtype=dt)
        keep.append(a)
        return _ptr(a)

    net = moss_network(sc.n_nodes, sc.n_roads, sc.n_lanes, sc.n_scen,
                       arr(sc.road_from, np.int32), arr(sc.road_to, np.int32),
                       arr(sc.road_nlanes, np.int32), arr(sc.road_lane0, np.int32),
                       arr(sc.road_length, np.float32), arr(sc.lane_vlim, np.float32),
                       arr(sc.lane_scen, np.int32), arr(sc.node_x, np.float64),
                       arr(sc.node_y, np.float64))
    if sc.lane_succ_off is not None:
        net.road_internal = arr(sc.road_internal, np.uint8)
        net.lane_succ_off = arr(sc.lane_succ_off, np.int32)
        net.lane_succ = arr(sc.lane_succ, np.int32)
        net.lane_conf_off = arr(sc.lane_conf_off, np.int32)
        net.lane_conf = arr(sc.lane_conf, np.int32)
        net.lane_conf_feed = arr(sc.lane_conf_feed, np.int32)
    sig = moss_signals(arr(sc.node_cycle, np.int32), arr(sc.node_phase, np.int32),
                       arr(sc.node_offset, np.int32), arr(sc.road_group, np.int8))
    veh = moss_vehicles(sc.n_veh, arr(sc.veh_id, np.uint32), arr(sc.depart, np.int32),
                        arr(sc.v0, np.float32), arr(sc.route_off, np.int64),
                        arr(sc.route_roads, np.int32), arr(sc.placed, np.uint8),
                        arr(sc.lane, np.int32), arr(sc.cursor, np.int32), arr(sc.s, np.float32),
                        arr(sc.v, np.float32), arr(sc.a, np.float32))
    p = sc.params
    flags = (MOSS_FLAG_DEBUG if debug else 0) | (MOSS_FLAG_TRACE if trace else 0)
    mlp_cfg = p.get("mlp")
    prm = moss_params(p["dt"], p["a_max"], p["b"], p["s0"], p["T"], p["length"], p["b_max"],
                      p["b_safe"], p["politeness"], p["a_thr"], p["p_lc"], p["d_look"],
                      int(p["h_look"]), int(p["t0"]), int(p["seed"]), flags,
                      MOSS_MODE_MLP if mlp_cfg is not None else MOSS_MODE_IDM,
                      arr(mlp_cfg["theta"], np.float32) if mlp_cfg is not None else None,
                      arr(mlp_cfg["norm"], np.float32) if mlp_cfg is not None else None,
                      float(p.get("b_mand", 1.0)), float(p.get("tau_yield", 3.0)))
    return net, sig, veh, prm, keep


def moss_query_workspace(net, sig, veh, prm) -> int:
    n = C.c_size_t(0)
    _check(load().moss_query_workspace(C.byref(net), C.byref(sig), C.byref(veh), C.byref(prm),
                                       C.byref(n)))
    return int(n.value)


def moss_create(net, sig, veh, prm, ws_ptr: int, ws_bytes: int, stream: int) -> int:
    h = vp()
    _check(load().moss_create(C.byref(net), C.byref(sig), C.byref(veh), C.byref(prm),
                              vp(ws_ptr), ws_bytes, vp(stream), C.byref(h)))
    return h.value


def moss_step(h: int, n: int):
    _check(load().moss_step(vp(h), int(n)))


def moss_read_state(h: int, out: moss_state_out):
    _check(load().moss_read_state(vp(h), C.byref(out)))
    return out


def moss_read_counters(h: int, n_scen: int):
    cnt = np.zeros((n_scen, len(COUNTER_NAMES)), np.int64)
    sv = np.zeros(n_scen, np.float64)
    err = C.c_uint32(0)
    _check(load().moss_read_counters(vp(h), _ptr(cnt), _ptr(sv), C.byref(err)))
    return cnt, sv, int(err.value)


def moss_read_pending(h: int, capacity: int) -> np.ndarray:
    ids = np.empty(max(capacity, 1), np.uint32)
    n = C.c_int32(0)
    _check(load().moss_read_pending(vp(h), capacity, _ptr(ids), C.byref(n)))
    return ids[:n.value].copy()


def moss_read_debug(h: int, capacity: int):
    d = dict(id=np.empty(capacity, np.uint32), leader=np.empty(capacity, np.uint32),
             flags=np.empty(capacity, np.int32), margin=np.empty(capacity, np.float32),
             t_leader=np.empty(capacity, np.uint32), t_follower=np.empty(capacity, np.uint32))
    n = C.c_int32(0)
    _check(load().moss_read_debug(vp(h), capacity, _ptr(d["id"]), _ptr(d["leader"]),
                                  _ptr(d["flags"]), _ptr(d["margin"]), _ptr(d["t_leader"]),
                                  _ptr(d["t_follower"]), C.byref(n)))
    return {k: v[:n.value].copy() for k, v in d.items()}


def moss_step_timed(h: int, n: int):
    """Runs n steps; returns {kernel name: total milliseconds over the n steps}."""
    ms = np.zeros(32, np.float64)
    k = C.c_int32(0)
    _check(load().moss_step_timed(vp(h), int(n), _ptr(ms), 32, C.byref(k)))
    return {load().moss_kernel_name(i).decode(): float(ms[i]) for i in range(k.value)}


def kernel_names() -> List[str]:
    """Names of the step kernels in moss_step_timed's order."""
    L = load()
    out = []
    while True:
        n = L.moss_kernel_name(len(out))
        if n is None:
            return out
        out.append(n.decode())


def moss_set_launch(h: int, cfg: Dict[str, int]):
    c = moss_launch(**{k: int(cfg[k]) for k in LAUNCH_FIELDS})
    _check(load().moss_set_launch(vp(h), C.byref(c)))


def moss_get_launch(h: int) -> Dict[str, int]:
    c = moss_launch()
    _check(load().moss_get_launch(vp(h), C.byref(c)))
    return {k: int(getattr(c, k)) for k in LAUNCH_FIELDS}


def _dp(x):
    return None if x is None else vp(x.data_ptr())


def mlp_grad(feat, label, theta, norm, *, idx=None, bf16=True, out_lo=-1e30, out_hi=1e30,
             stream=None):
    """(loss, grad) of the closure on a batch of device tensors."""
    import torch
    n = int(idx.shape[0]) if idx is not None else int(feat.shape[0])
    nb = int(load().moss_mlp_scratch_bytes(n))
    scratch = torch.empty(nb, dtype=torch.uint8, device=feat.device)
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=feat.device)
    loss = torch.empty(1, dtype=torch.float32, device=feat.device)
    st = (stream or torch.cuda.current_stream(feat.device)).cuda_stream
    _check(load().moss_mlp_grad(_dp(feat), _dp(label), _dp(idx), n, _dp(theta), _dp(norm),
                                1 if bf16 else 0, out_lo, out_hi, _dp(grad), _dp(loss),
                                _dp(scratch), nb, vp(st)))
    return loss, grad


def mlp_grad_static(feat, label, theta, norm, grad, loss, *, idx=None, bf16=True,
                    out_lo=-1e30, out_hi=1e30, stream=None):
    """mlp_grad through the entry point that allocates nothing: the caller
    passes the outputs grad (float32[MLP_PARAMS]) and loss (float32[1]); the
    library's static scratch holds the intermediates."""
    import torch
    n = int(idx.shape[0]) if idx is not None else int(feat.shape[0])
    st = (stream or torch.cuda.current_stream(feat.device)).cuda_stream
    _check(load().moss_mlp_grad_static(_dp(feat), _dp(label), _dp(idx), n, _dp(theta),
                                       _dp(norm), 1 if bf16 else 0, out_lo, out_hi, _dp(grad),
                                       _dp(loss), vp(st)))
    return loss, grad


def mlp_adam(theta, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    import torch
    st = (stream or torch.cuda.current_stream(theta.device)).cuda_stream
    _check(load().moss_mlp_adam(_dp(theta), _dp(m), _dp(v), _dp(grad), int(step), lr, beta1,
                                beta2, eps, vp(st)))


def mlp_predict(feat, theta, norm, stream=None):
    import torch
    out = torch.empty(feat.shape[0], dtype=torch.float32, device=feat.device)
    st = (stream or torch.cuda.current_stream(feat.device)).cuda_stream
    _check(load().moss_mlp_predict(_dp(feat), int(feat.shape[0]), _dp(theta), _dp(norm),
                                   _dp(out), vp(st)))
    return out


def moss_destroy(h: int):
    _check(load().moss_destroy(vp(h)))


def moss_last_error() -> str:
    return load().moss_last_error().decode()


class Simulator:
    """A simulation of one Scenario on the current torch device and stream."""

    def __init__(self, sc, *, debug: bool = False, trace: bool = False,
                 device: Optional[int] = None, stream=None, coords: bool = True):
        """coords=False creates the simulator without node coordinates
        (positions are then unavailable)."""
        import torch
        load()
        self.sc = sc
        self.n_scen = sc.n_scen
        self.sc_n_roads = sc.n_roads
        self.cap = max(sc.n_veh, 1)
        net, sig, veh, prm, keep = marshal(sc, debug, trace)
        if not coords:
            net.node_x = net.node_y = None
        nbytes = moss_query_workspace(net, sig, veh, prm)
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self.ws.data_ptr()
        aligned = (base + 255) & ~255
        # a stream of its own (default priority): the legacy null stream cannot
        # capture the step graphs
        self.stream = stream if stream is not None else torch.cuda.Stream(dev)
        self.h = moss_create(net, sig, veh, prm, aligned, nbytes, self.stream.cuda_stream)
        self.debug_enabled = debug
        del keep

    def step(self, n: int = 1):
        moss_step(self.h, n)

    def state(self, cursor: bool = True) -> Dict[str, np.ndarray]:
        c = self.cap
        out = dict(id=np.empty(c, np.uint32), lane=np.empty(c, np.int32),
                   s=np.empty(c, np.float32), v=np.empty(c, np.float32),
                   a=np.empty(c, np.float32), cursor=np.empty(c, np.int32))
        so = moss_state_out(c, 0, _ptr(out["id"]), _ptr(out["lane"]), _ptr(out["s"]),
                            _ptr(out["v"]), _ptr(out["a"]),
                            _ptr(out["cursor"]) if cursor else None, 0, 0)
        moss_read_state(self.h, so)
        self.t = int(so.t)
        n = int(so.n)
        res = {k: v[:n].copy() for k, v in out.items()}
        if not cursor:
            res.pop("cursor")
        return res

    def state_device(self):
        """State rows as torch tensors on the simulator's device (device copy)."""
        import torch
        c = self.cap
        dev = self.ws.device
        out = dict(id=torch.empty(c, dtype=torch.int32, device=dev),
                   lane=torch.empty(c, dtype=torch.int32, device=dev),
                   s=torch.empty(c, dtype=torch.float32, device=dev),
                   v=torch.empty(c, dtype=torch.float32, device=dev),
                   a=torch.empty(c, dtype=torch.float32, device=dev))
        so = moss_state_out(c, 1, vp(out["id"].data_ptr()), vp(out["lane"].data_ptr()),
                            vp(out["s"].data_ptr()), vp(out["v"].data_ptr()),
                            vp(out["a"].data_ptr()), None, 0, 0)
        moss_read_state(self.h, so)
        n = int(so.n)
        return {k: v[:n] for k, v in out.items()}

    @property
    def n_active(self) -> int:
        so = moss_state_out(0, 0, None, None, None, None, None, None, 0, 0)
        try:
            moss_read_state(self.h, so)
        except MossError as e:
            if e.code != MOSS_ENOMEM:
                raise
        return int(so.n)

    def counters(self):
        return moss_read_counters(self.h, self.n_scen)

    def pending(self) -> np.ndarray:
        """Ids of the vehicles still waiting to enter (moss_read_pending)."""
        return moss_read_pending(self.h, self.cap)

    def checkpoint(self) -> Dict[str, object]:
        """State rows, pending ids and the next step index: what
        scenarios.resume needs to continue this run in a new simulator."""
        return dict(state=self.state(), pending=self.pending(), t=self.t)

    def step_timed(self, n: int):
        return moss_step_timed(self.h, n)

    def set_signal_phase(self, nodes, phases):
        """Holds phases[i] at nodes[i] from the next step on (-1: fixed-time plan)."""
        j = np.ascontiguousarray(np.atleast_1d(nodes), np.int32)
        p = np.ascontiguousarray(np.atleast_1d(phases), np.int32)
        if j.shape != p.shape:
            raise ValueError("nodes and phases differ in length")
        _check(load().moss_set_signal_phase(vp(self.h), _ptr(j), _ptr(p), int(j.shape[0])))

    def set_lane_vlim(self, lanes, vlims):
        """Speed limits of lanes from the next step on."""
        l = np.ascontiguousarray(np.atleast_1d(lanes), np.int32)
        v = np.ascontiguousarray(np.atleast_1d(vlims), np.float32)
        if l.shape != v.shape:
            raise ValueError("lanes and limits differ in length")
        _check(load().moss_set_lane_vlim(vp(self.h), _ptr(l), _ptr(v), int(l.shape[0])))

    def set_lane_closed(self, lanes, closed):
        """Closes (1) or opens (0) lanes from the next step on."""
        l = np.ascontiguousarray(np.atleast_1d(lanes), np.int32)
        c = np.ascontiguousarray(np.atleast_1d(closed), np.int32)
        if l.shape != c.shape:
            raise ValueError("lanes and flags differ in length")
        _check(load().moss_set_lane_closed(vp(self.h), _ptr(l), _ptr(c), int(l.shape[0])))

    def set_lane_turns(self, lanes, roads, allowed):
        """Lets lanes continue onto roads (1) or not (0) from the next step on
        (junction internal lanes)."""
        l = np.ascontiguousarray(np.atleast_1d(lanes), np.int32)
        r = np.ascontiguousarray(np.atleast_1d(roads), np.int32)
        a = np.ascontiguousarray(np.atleast_1d(allowed), np.int32)
        if not (l.shape == r.shape == a.shape):
            raise ValueError("lanes, roads and flags differ in length")
        _check(load().moss_set_lane_turns(vp(self.h), _ptr(l), _ptr(r), _ptr(a),
                                          int(l.shape[0])))

    def road_stats(self):
        """(vehicles per road [n_roads] int32, mean speed per road [n_roads] float32)."""
        cnt = np.empty(self.sc_n_roads, np.int32)
        mv = np.empty(self.sc_n_roads, np.float32)
        _check(load().moss_read_road_stats(vp(self.h), 0, _ptr(cnt), _ptr(mv)))
        return cnt, mv

    def positions(self):
        """(x, y, heading) of every state row, float64 (host)."""
        c = self.cap
        x, y, hd = (np.empty(c, np.float64) for _ in range(3))
        n = C.c_int32(0)
        _check(load().moss_read_positions(vp(self.h), c, 0, _ptr(x), _ptr(y), _ptr(hd),
                                          C.byref(n)))
        return x[:n.value], y[:n.value], hd[:n.value]

    def trips(self):
        """Per vehicle in ascending id order (host arrays): id, status (0
        waiting, 1 on the network, 2 arrived), travel time (steps) and
        distance (m) since it entered the simulation."""
        c = self.cap
        out = dict(id=np.empty(c, np.uint32), status=np.empty(c, np.int32),
                   travel=np.empty(c, np.int32), distance=np.empty(c, np.float64))
        n = C.c_int32(0)
        _check(load().moss_read_trips(vp(self.h), c, 0, _ptr(out["id"]), _ptr(out["status"]),
                                      _ptr(out["travel"]), _ptr(out["distance"]), C.byref(n)))
        return {k: v[:n.value] for k, v in out.items()}

    def set_launch(self, **cfg):
        """Changes the launch shape (fields of moss_launch; omitted ones keep
        their value).  Results do not depend on it."""
        cur = moss_get_launch(self.h)
        unknown = set(cfg) - set(cur)
        if unknown:
            raise ValueError(f"unknown launch fields {sorted(unknown)}")
        cur.update(cfg)
        moss_set_launch(self.h, cur)

    def launch(self) -> Dict[str, int]:
        return moss_get_launch(self.h)

    def trace(self, device: bool = True):
        """(features [n, 8], IDM labels [n]) of the last step."""
        import torch
        c = self.cap
        if device:
            f = torch.empty((c, MLP_NORM // 4), dtype=torch.float32, device=self.ws.device)
            y = torch.empty(c, dtype=torch.float32, device=self.ws.device)
            fp, yp = f.data_ptr(), y.data_ptr()
        else:
            f = np.empty((c, MLP_NORM // 4), np.float32)
            y = np.empty(c, np.float32)
            fp, yp = f.ctypes.data, y.ctypes.data
        n = C.c_int32(0)
        _check(load().moss_read_trace(vp(self.h), c, 1 if device else 0, vp(fp), vp(yp),
                                      C.byref(n)))
        return f[:n.value], y[:n.value]

    def mlp_error(self):
        out = np.zeros(self.n_scen, np.float64)
        _check(load().moss_read_mlp_error(vp(self.h), _ptr(out)))
        return out

    def debug(self):
        return moss_read_debug(self.h, self.cap)

    def close(self):
        if getattr(self, "h", None):
            moss_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
