"""Launch-shape tuner for a workload (batched scenarios in particular).

The step's launch shape (``moss_launch``: steps per captured graph, workgroups
of the update and of the joiner scatter, XCD-contiguous tile order) changes
how the work is grouped, never what is computed, so it can be chosen by
measurement alone.  The tuner starts from the current shape and tries one
field at a time, keeping a change only when it is faster than the incumbent
measured right next to it (paired windows, so that the state's drift over
the tuning run does not decide).  Winners are cached per (GPU architecture,
workload class) in a JSON file (``MOSS_TUNE_CACHE`` or ``_build/autotune.json``
beside the library).

All timing runs the simulator's own kernels; this module only sequences
calls.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, Optional, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))

# Candidate values per field, tried in this order.
SPACE = {
    "graph_steps": [8, 16, 32, 64],
    "xcd_remap": [0, 1],
    "update_blocks": [0, 512, 1024, 2048, 4096],
    "scatter_blocks": [0, 256, 1024, 4096],
}
WINDOW = 64          # steps per measurement (a multiple of every graph length)
MARGIN = 0.02        # a change must be this much faster to be kept


def cache_path() -> str:
    return os.environ.get("MOSS_TUNE_CACHE", os.path.join(HERE, "_build", "autotune.json"))


def workload_class(sc) -> str:
    """Mode, and vehicles / lanes / scenarios to the nearest power of two."""
    mode = "mlp" if sc.params.get("mlp") else "idm"
    lg = lambda x: int(round(math.log2(max(int(x), 1))))
    return f"{mode}:veh2^{lg(sc.n_veh)}:lanes2^{lg(sc.n_lanes)}:scen2^{lg(sc.n_scen)}"


def _arch() -> str:
    import torch
    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName


def _load_cache() -> Dict[str, dict]:
    p = cache_path()
    if not os.path.exists(p):
        return {}
    with open(p) as f:
        return json.load(f)


def _store_cache(key: str, rec: dict):
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    data = _load_cache()
    data[key] = rec
    tmp = p + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def measure(sim, cfg: Dict[str, int], steps: int = WINDOW) -> float:
    """Milliseconds per step of `steps` steps under launch shape cfg (after
    one warm-up graph, which also captures it)."""
    import torch
    sim.set_launch(**cfg)
    sim.step(max(cfg.get("graph_steps", 0), 2))
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(sim.stream)
    sim.step(steps)
    ev1.record(sim.stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps


def search(sim, *, steps: int = WINDOW, log=None) -> Tuple[Dict[str, int], float]:
    """One pass of coordinate search from the simulator's current shape."""
    best = sim.launch()
    t_best = measure(sim, best, steps)
    for field, values in SPACE.items():
        for v in values:
            if v == best[field]:
                continue
            cand = dict(best, **{field: v})
            t_inc = measure(sim, best, steps)
            t_c = measure(sim, cand, steps)
            if log:
                log(f"[tune] {field}={v}: {t_c:.4f} ms/step vs {t_inc:.4f}")
            if t_c < (1.0 - MARGIN) * t_inc:
                best, t_best = cand, t_c
    sim.set_launch(**best)
    return best, t_best


def tune(sim, sc, *, use_cache: bool = True, steps: int = WINDOW, log=None) -> Dict[str, object]:
    """Applies the cached shape for this workload class, or searches for one
    on `sim` (which advances its state) and caches it.  Returns the record
    {"launch": cfg, "ms_per_step": t, "cached": bool, "key": key}."""
    key = f"{_arch()}|{workload_class(sc)}"
    if use_cache:
        rec = _load_cache().get(key)
        if rec is not None:
            sim.set_launch(**rec["launch"])
            return dict(rec, cached=True, key=key)
    cfg, t = search(sim, steps=steps, log=log)
    rec = dict(launch=cfg, ms_per_step=round(t, 5))
    _store_cache(key, rec)
    return dict(rec, cached=False, key=key)


def apply(sim, rec: Optional[Dict[str, object]]):
    if rec:
        sim.set_launch(**rec["launch"])
