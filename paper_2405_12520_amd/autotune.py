"""Launch-shape tuner for a workload (batched scenarios in particular).

The step's launch shape (``moss_launch``: steps per captured graph, workgroups
of the update and of the joiner scatter, XCD-contiguous tile order) changes
how the work is grouped, never what is computed, so it can be chosen by
measurement alone.  The tuner starts from the default shape and tries one
field at a time, keeping a change when it is faster.  Every candidate is
timed on a fresh simulator created from the same scenario and stepped to the
same point, so all of them time exactly the same work (timing one simulator
while its state evolves confounds the shape with the state: in a dense city
the step cost moves by 20 % within a few hundred steps as queues form and
dissolve).  Winners are cached per (GPU architecture, workload class) in a
JSON file (``MOSS_TUNE_CACHE`` or ``_build/autotune.json`` beside the
library).

All timing runs the simulator's own kernels; this module only sequences
calls.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, Optional, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))

# Candidate values per field, tried in this order after the default shape.
DEFAULT = dict(graph_steps=16, update_blocks=0, scatter_blocks=0, xcd_remap=0)
SPACE = {
    "xcd_remap": [1],
    "graph_steps": [32],
    "update_blocks": [1024, 4096],
    "scatter_blocks": [256],
}
WINDOW = 128         # steps per measurement (a multiple of every graph length)
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


def search(make_sim, warmup: int, *, steps: int = WINDOW,
           log=None) -> Tuple[Dict[str, int], float]:
    """Coordinate search from the default shape; make_sim() returns a new
    simulator at the scenario's first step."""
    def trial(cfg):
        sim = make_sim()
        try:
            sim.set_launch(**cfg)
            sim.step(warmup)
            return measure(sim, cfg, steps)
        finally:
            sim.close()

    best = dict(DEFAULT)
    t_best = trial(best)
    if log:
        log(f"[tune] default {best}: {t_best:.4f} ms/step")
    for field, values in SPACE.items():
        for v in values:
            if v == best[field]:
                continue
            cand = dict(best, **{field: v})
            t_c = trial(cand)
            if log:
                log(f"[tune] {field}={v}: {t_c:.4f} ms/step vs {t_best:.4f}")
            if t_c < (1.0 - MARGIN) * t_best:
                best, t_best = cand, t_c
    return best, t_best


def tune(make_sim, sc, warmup: int, *, use_cache: bool = True, steps: int = WINDOW,
         log=None) -> Dict[str, object]:
    """The cached shape for this workload class, or one found by search (and
    then cached).  Returns {"launch": cfg, "ms_per_step": t, "cached": bool,
    "key": key}; apply it to a simulator with apply()."""
    key = f"{_arch()}|{workload_class(sc)}"
    if use_cache:
        rec = _load_cache().get(key)
        if rec is not None:
            return dict(rec, cached=True, key=key)
    cfg, t = search(make_sim, warmup, steps=steps, log=log)
    rec = dict(launch=cfg, ms_per_step=round(t, 5))
    _store_cache(key, rec)
    return dict(rec, cached=False, key=key)


def apply(sim, rec: Optional[Dict[str, object]]):
    if rec:
        sim.set_launch(**rec["launch"])
