"""Benchmark: vehicle-steps per second of the per-step microscopic update on
one MI355X, with the roofline of the dominant kernel and the CPU oracle's
throughput on the host as a baseline.

Workload (default): the city-scale synthetic network (200 x 200 jittered
lattice, ~40k nodes, ~120k lanes, log-normal road lengths with median 150 m)
with 2,000,000 vehicles pre-placed on long random-walk routes, IDM + MOBIL,
dt = 1 s, FP32 state.  Inputs are generated on the host, copied to the GPU
once, and are resident in HBM when the timed region starts.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "vehicle-steps/sec at 2M vehicles + HBM GB/s vs peak; MLP vs IDM on same GPU"
HBM_PEAK_GBS = 8000.0

# Algorithmic HBM bytes per vehicle and launch of the two per-vehicle kernels
# (the minimum each must move; lane tables and neighbour reads are on-chip
# reuse): k_update reads 7 state fields (lane, s, v, id, route ptr, next road,
# v0 = 28 B) and writes a 6-field proposal (24 B; id and v0 alternate between
# two buffers by step parity instead of being copied); k_merge reads the
# proposal and the old id/v0 (32 B) and writes the 8-field state (32 B).
ALGO_BYTES = {"k_update": 28 + 24, "k_merge": 32 + 32}
# Whole step: the two per-vehicle kernels plus about 40 B per lane for the
# lane-count scans, lane starts, tails and red flags.
STEP_LANE_BYTES = 40


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def load_traffic(kernel):
    """Measured HBM bytes per launch from the committed counter summary, if it
    was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    from paper_2405_12520_amd.profile_summary import kernel_sources_sha
    if rec.get("source_sha") != kernel_sources_sha():
        return None
    # the summary names template kernels with their arguments: the benchmark's
    # kernel is the one whose base name matches (the IDM variant)
    for name, k in rec.get("kernels", {}).items():
        if name.split("<")[0] == kernel:
            return k.get("bytes_per_launch")
    return None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sc, steps, steps_mt):
    """The oracle as it stands on the host: one thread over `steps` steps,
    then all the threads OpenMP is given (OMP_NUM_THREADS) over `steps_mt`
    further steps of the same run.  The two give the same bits; the
    multi-thread rate is the reported value."""
    from oracle import OracleSim, max_threads
    nthr = max_threads()
    say(f"[bench] cpu oracle: {steps} steps on 1 thread, {steps_mt} on {nthr}")
    t0 = time.perf_counter()
    o = OracleSim(sc)
    t_create = time.perf_counter() - t0

    def run(k, threads):
        o.set_threads(threads)
        c0 = o.counters()[0][:, 6].sum()
        t0 = time.perf_counter()
        o.step(k)
        dt = time.perf_counter() - t0
        return (o.counters()[0][:, 6].sum() - c0) / dt, dt

    v1, dt1 = run(steps, 1)
    vn, dtn = run(steps_mt, nthr)
    say(f"[bench] cpu oracle: 1 thread {v1:.4g}, {nthr} threads {vn:.4g} vehicle-steps/s")
    return dict(value=float(vn), unit="vehicle-steps/s", cores=int(nthr), kind="oracle",
                single_thread_value=float(v1), nproc=os.cpu_count(),
                affinity=len(os.sched_getaffinity(0)), cpu_model=cpu_model(),
                sample=f"the {sc.n_veh}-vehicle city snapshot: {steps} steps on one thread "
                       f"({dt1:.1f} s), then {steps_mt} steps on {nthr} OpenMP threads "
                       f"({dtn:.1f} s); create {t_create:.1f} s not timed")


MLP_FLOP = 2 * (8 * 64 + 64 * 64 + 64)      # multiply-adds of one evaluation, x2
BF16_PEAK_TFLOPS = 2500.0


def graph_len_for(steps, tuned):
    """Steps per captured graph for a timed region of `steps` steps: the
    tuned length when it divides them, else the even divisor of `steps` (at
    most 256) nearest to it, so that every timed step runs inside a whole
    graph replay rather than kernel by kernel (the work is the same)."""
    if tuned <= 0 or steps % tuned == 0:
        return tuned
    divs = [g for g in range(2, min(steps, 256) + 1, 2) if steps % g == 0]
    return min(divs, key=lambda g: (abs(g - tuned), -g)) if divs else tuned


def fit_graphs(sim, steps):
    """Sets the simulator's graph length for a timed region of `steps` steps
    (graph_len_for); the graphs are captured here, outside the timing.
    Returns the launch shape in use."""
    g = sim.launch()["graph_steps"]
    g2 = graph_len_for(steps, g)
    if g2 != g:
        sim.set_launch(graph_steps=g2)
    return sim.launch()


def timed_steps(sim, steps):
    import torch
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    c0 = sim.counters()[0]
    ev0.record(sim.stream)
    sim.step(steps)
    ev1.record(sim.stream)
    torch.cuda.synchronize()
    c1 = sim.counters()[0]
    return ev0.elapsed_time(ev1), c1 - c0


def bench_mlp(sc, args):
    """Same city snapshot with the learned closure (trained on the 10x10 grid
    workload) in place of IDM inside its envelope."""
    import torch
    from paper_2405_12520_amd import closure
    from paper_2405_12520_amd.moss import Simulator
    path = closure.DEFAULT_PATH
    if os.path.exists(path):
        theta, norm = closure.load(path)
        src = "loaded " + os.path.relpath(path, ROOT)
    else:
        say("[bench] training the closure on the grid workload")
        theta, norm, _ = closure.build_closure(path, log=say)
        src = "trained in this run"
    msc = sc.with_params(mlp=dict(theta=theta, norm=norm))
    rec = None
    if not args.no_tune:
        # network mode has its own launch shape (its update block holds the
        # weights in LDS, so persistent blocks copy them fewer times)
        from paper_2405_12520_amd import autotune
        t0 = time.time()
        rec = autotune.tune(lambda: Simulator(msc), msc, args.warmup, log=say)
        torch.cuda.empty_cache()
        say(f"[bench] network-mode launch shape {rec['launch']} "
            f"({'cached' if rec['cached'] else 'searched'} in {time.time() - t0:.1f} s)")
    sim = Simulator(msc)
    if rec:
        autotune.apply(sim, rec)
    launch = fit_graphs(sim, args.steps)
    sim.step(args.warmup)
    sq0 = sim.mlp_error().sum()
    ms, dc = timed_steps(sim, args.steps)
    sq1 = sim.mlp_error().sum()
    veh_steps = int(dc[:, 6].sum())
    n_eval = int(dc[:, 7].sum())
    n_fb = int(dc[:, 8].sum())
    kms = sim.step_timed(20)
    upd_ms = kms["k_update"] / 20
    evals_per_launch = n_eval / args.steps
    tflops = evals_per_launch * MLP_FLOP / (upd_ms * 1e-3) / 1e12
    sim.close()
    torch.cuda.empty_cache()
    rms = float(np.sqrt((sq1 - sq0) / max(n_eval, 1)))
    say(f"[bench] mlp mode: {veh_steps / (ms / 1e3):.4g} vehicle-steps/s, RMS vs IDM {rms:.4f}, "
        f"fallback {n_fb / max(veh_steps, 1):.4f}")
    return dict(value=round(veh_steps / (ms / 1e3), 1), unit="vehicle-steps/s",
                ms_per_step=round(ms / args.steps, 5), rms_accel_error_vs_idm=round(rms, 5),
                fallback_rate=round(n_fb / max(veh_steps, 1), 5), weights=src, launch=launch,
                roofline=dict(bound="mfma", kernel="k_update<mlp>", dtype="bf16",
                              achieved=round(tflops, 2), peak=BF16_PEAK_TFLOPS, unit="TFLOP/s",
                              frac=round(tflops / BF16_PEAK_TFLOPS, 5),
                              flop_per_eval=MLP_FLOP, kernel_ms=round(upd_ms, 5)))


def big_city():
    """City network tiled 2 x 2 (160k nodes, 482k lanes) with 8M vehicles
    pre-placed: a working set (state + proposals + joiner records, 96 B per
    vehicle) far beyond the 256 MB Infinity Cache, so the kernels' bytes come
    from HBM."""
    from paper_2405_12520_amd import scenarios as S
    t0 = time.time()
    sc = S.city_snapshot(8_000_000, side=400, target_undirected=184_000, hops=24)
    say(f"[bench] 8M city generated in {time.time() - t0:.1f} s: {sc.summary()}")
    return sc


def bench_big(args):
    """Throughput and per-kernel times on the 8M-vehicle city (big_city), in
    the launch shape the tuner picks for it (unless --no-tune)."""
    import torch
    from paper_2405_12520_amd import autotune
    from paper_2405_12520_amd.moss import Simulator
    sc = big_city()
    launch = None
    if not args.no_tune:
        t0 = time.time()
        launch = autotune.tune(lambda: Simulator(sc), sc, args.warmup, log=say)
        torch.cuda.empty_cache()
        say(f"[bench] 8M city launch shape {launch['launch']} "
            f"({'cached' if launch['cached'] else 'searched'} in {time.time() - t0:.1f} s)")
    sim = Simulator(sc)
    autotune.apply(sim, launch)
    used = fit_graphs(sim, args.steps)
    sim.step(args.warmup)
    ms, dc = timed_steps(sim, args.steps)
    veh_steps = int(dc[:, 6].sum())
    kms = sim.step_timed(20)
    n_act = sim.n_active
    sim.close()
    del sim
    torch.cuda.empty_cache()
    per = {k: v / 20 for k, v in kms.items() if v > 0}
    frac = {k: round(ALGO_BYTES[k] * n_act / (per[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
            for k in ALGO_BYTES}
    say(f"[bench] 8M city: {veh_steps / (ms / 1e3):.4g} vehicle-steps/s, per-kernel ms "
        f"{ {k: round(v, 4) for k, v in per.items()} }")
    return dict(value=round(veh_steps / (ms / 1e3), 1), unit="vehicle-steps/s",
                ms_per_step=round(ms / args.steps, 5), vehicles=int(sc.n_veh),
                lanes=int(sc.n_lanes), kernel_ms={k: round(v, 5) for k, v in per.items()},
                hbm_frac=frac, launch=used)


def junction_city(sc):
    """The city snapshot rebuilt with junction internal lanes: a connector
    lane per movement through every junction, routes through the
    connectors, the turn-lane bias and the yield rule at conflicting
    movements."""
    from paper_2405_12520_amd import junctions as J
    t0 = time.time()
    jsc = J.with_junction_lanes(sc)
    jl = jsc.meta["junction_lanes"]
    say(f"[bench] junction lanes built in {time.time() - t0:.1f} s: {jsc.summary()}, "
        f"{jl['connectors']} connectors, {jl['connector_lanes']} connector lanes")
    return jsc


def bench_junctions(sc, launch, args):
    """The 2M city with junction internal lanes (the update variant with lane
    successors, the turn bias and the yield rule, plus the yield-flag kernel),
    in the launch shape tuned for the snapshot."""
    import torch
    from paper_2405_12520_amd.moss import Simulator
    jsc = junction_city(sc)
    sim = Simulator(jsc)
    sim.set_launch(**{k: v for k, v in launch.items() if k != "graph_steps"})
    used = fit_graphs(sim, args.steps)
    sim.step(args.warmup)
    ms, dc = timed_steps(sim, args.steps)
    veh_steps = int(dc[:, 6].sum())
    kms = sim.step_timed(20)
    n_act = sim.n_active
    _, _, err = sim.counters()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    if err:
        raise RuntimeError(f"junction-lane city: device error word {err}")
    per = {k: v / 20 for k, v in kms.items() if v > 0}
    frac = {k: round(ALGO_BYTES[k] * n_act / (per[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
            for k in ALGO_BYTES}
    jl = jsc.meta["junction_lanes"]
    say(f"[bench] junction-lane city: {veh_steps / (ms / 1e3):.4g} vehicle-steps/s, "
        f"per-kernel ms { {k: round(v, 4) for k, v in per.items()} }")
    return dict(value=round(veh_steps / (ms / 1e3), 1), unit="vehicle-steps/s",
                ms_per_step=round(ms / args.steps, 5), vehicles=int(jsc.n_veh),
                active_vehicles=int(n_act), lanes=int(jsc.n_lanes),
                connector_lanes=int(jl["connector_lanes"]),
                kernel_ms={k: round(v, 5) for k, v in per.items()}, hbm_frac=frac, launch=used)


def bench_batch(args):
    """Disjoint union of independent grid scenarios (4x4 .. 16x16, 1k..50k
    vehicles each, departures over 1800 s) stepped as one network through the
    captured step graphs; timed after a warm-up into the departure period."""
    import torch
    from paper_2405_12520_amd import scenarios as S
    from paper_2405_12520_amd.moss import Simulator
    t0 = time.time()
    sc = S.batch(args.batch_scenarios)
    say(f"[bench] batch generated in {time.time() - t0:.1f} s: {sc.summary()}")
    # launch shape: tuned on a second copy at the same point of the run
    from paper_2405_12520_amd import autotune
    t0 = time.time()
    rec = autotune.tune(lambda: Simulator(sc), sc, 600, log=say)
    torch.cuda.empty_cache()
    say(f"[bench] batch launch shape {rec['launch']} ({'cached' if rec['cached'] else 'searched'}"
        f" in {time.time() - t0:.1f} s)")
    sim = Simulator(sc)
    autotune.apply(sim, rec)
    used = fit_graphs(sim, args.steps)
    sim.step(600)
    ms, dc = timed_steps(sim, args.steps)
    veh_steps = int(dc[:, 6].sum())
    # per-kernel durations over the next 20 steps (HIP events on the
    # simulator's stream) and the roofline of the dominant per-vehicle kernel
    n0 = sim.n_active
    kms = sim.step_timed(20)
    n_act = 0.5 * (n0 + sim.n_active)
    sim.close()
    torch.cuda.empty_cache()
    per = {k: v / 20 for k, v in kms.items() if v > 0}
    dom = max(ALGO_BYTES, key=lambda k: per[k])
    achieved = ALGO_BYTES[dom] * n_act / (per[dom] * 1e-3) / 1e9
    say(f"[bench] batch: {veh_steps / (ms / 1e3):.4g} vehicle-steps/s, per-kernel ms "
        f"{ {k: round(v, 4) for k, v in per.items()} }")
    return dict(value=round(veh_steps / (ms / 1e3), 1), unit="vehicle-steps/s",
                ms_per_step=round(ms / args.steps, 5), scenarios=int(sc.n_scen),
                vehicles_total=int(sc.n_veh), active_mean=round(veh_steps / args.steps, 1),
                window="steps 600..600+K of 1800", lanes=int(sc.n_lanes),
                launch=used, launch_tuned_ms_per_step=rec["ms_per_step"],
                kernel_ms={k: round(v, 5) for k, v in per.items()},
                roofline=dict(bound="hbm", kernel=dom, achieved=round(achieved, 1),
                              peak=HBM_PEAK_GBS, unit="GB/s",
                              frac=round(achieved / HBM_PEAK_GBS, 4),
                              algo_bytes_per_vehicle=ALGO_BYTES[dom],
                              active_vehicles=round(n_act, 1)))


def bench_small(args):
    """The two small workloads over their full hour (3600 steps): the single
    signalised intersection (200 vehicles departing over 600 s) and the
    10 x 10 grid (20,000 vehicles departing over the hour), on the GPU and
    with the oracle on all the host threads OpenMP is given.  Both are
    latency-bound on the GPU (a few thousand vehicles at most): steps per
    second is the figure that matters there."""
    import torch
    from paper_2405_12520_amd import scenarios as S
    from paper_2405_12520_amd.moss import Simulator
    out = {}
    for name, sc in (("c1_intersection", S.intersection()), ("c2_grid", S.grid(10, 20000))):
        sim = Simulator(sc)
        ms, dc = timed_steps(sim, 3600)
        vs = int(dc[:, 6].sum())
        sim.close()
        del sim
        torch.cuda.empty_cache()
        r = dict(steps=3600, vehicles=int(sc.n_veh), vehicle_steps=vs,
                 gpu=dict(ms=round(ms, 2), steps_per_s=round(3600 / (ms / 1e3), 1),
                          vehicle_steps_per_s=round(vs / (ms / 1e3), 1)))
        if not args.no_cpu:
            from oracle import OracleSim, max_threads
            o = OracleSim(sc)
            o.set_threads(max_threads())
            t0 = time.perf_counter()
            o.step(3600)
            dt = time.perf_counter() - t0
            r["cpu_oracle"] = dict(s=round(dt, 3), steps_per_s=round(3600 / dt, 1),
                                   vehicle_steps_per_s=round(vs / dt, 1),
                                   threads=int(max_threads()))
        say(f"[bench] {name}: {r}")
        out[name] = r
    return out


def bench_demand(args):
    """The city with its travel demand (2M gravity-model trips over 400 zones,
    departures over one hour, shortest-path routes), the whole hour (3600
    steps) in IDM mode and with the learned closure: throughput over the
    run and its macroscopic outputs (mean speed over all vehicle-steps,
    trips, mean trip time)."""
    import torch
    from paper_2405_12520_amd import closure
    from paper_2405_12520_amd import scenarios as S
    from paper_2405_12520_amd.moss import Simulator
    t0 = time.time()
    sc = S.city_demand()
    say(f"[bench] city demand generated in {time.time() - t0:.1f} s: {sc.summary()}")
    theta, norm = closure.load(closure.DEFAULT_PATH)
    out = dict(vehicles=int(sc.n_veh), steps=args.demand_steps,
               departures="uniform over steps 0..3599", zones=400)
    for mode in ("idm", "mlp"):
        sim = Simulator(sc if mode == "idm" else sc.with_params(mlp=dict(theta=theta, norm=norm)))
        sim.set_launch(xcd_remap=1)
        ms, dc = timed_steps(sim, args.demand_steps)
        c, sv, err = sim.counters()
        vs, arrived, ttime = int(c[:, 6].sum()), int(c[:, 2].sum()), int(c[:, 3].sum())
        r = dict(value=round(vs / (ms / 1e3), 1), unit="vehicle-steps/s",
                 ms_per_step=round(ms / args.demand_steps, 5), vehicle_steps=vs,
                 active_end=int(sim.n_active), trips=arrived,
                 mean_trip_time_s=round(ttime / max(arrived, 1), 2),
                 mean_speed_mps=round(float(sv.sum()) / max(vs, 1), 4),
                 insert_failures=int(c[:, 1].sum()), lane_changes=int(c[:, 5].sum()),
                 error_word=int(err))
        if mode == "mlp":
            n_eval, n_fb = int(c[:, 7].sum()), int(c[:, 8].sum())
            r["rms_accel_error_vs_idm"] = round(float(np.sqrt(sim.mlp_error().sum() /
                                                              max(n_eval, 1))), 5)
            r["fallback_rate"] = round(n_fb / max(vs, 1), 5)
        sim.close()
        del sim
        torch.cuda.empty_cache()
        say(f"[bench] city demand {mode}: {r}")
        out[mode] = r
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--vehicles", type=int, default=2_000_000)
    ap.add_argument("--cpu-steps", type=int, default=20,
                    help="steps of the single-thread oracle baseline")
    ap.add_argument("--cpu-steps-mt", type=int, default=60,
                    help="steps of the all-threads oracle baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-only", action="store_true",
                    help="run warmup + timed steps only (for rocprofv3)")
    ap.add_argument("--no-mlp", action="store_true")
    ap.add_argument("--mlp", action="store_true",
                    help="with --profile-only: step the city snapshot with the learned closure")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch", action="store_true",
                    help="with --profile-only: step the batch of grids (--batch-scenarios) "
                         "instead of the city snapshot; give --warmup 600 to reach the "
                         "departure period")
    ap.add_argument("--big", action="store_true",
                    help="with --profile-only: step the 8M-vehicle city instead of the "
                         "2M snapshot")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default launch shape instead of tuning it (profiling runs "
                         "never tune)")
    ap.add_argument("--launch", default="", metavar="JSON",
                    help='launch shape to use, e.g. \'{"xcd_remap": 1}\' (fields of moss_launch)')
    ap.add_argument("--no-demand", action="store_true",
                    help="skip the city's hour with its travel demand (IDM and closure)")
    ap.add_argument("--demand-steps", type=int, default=3600)
    ap.add_argument("--no-small", action="store_true",
                    help="skip the intersection and 10x10 grid hours")
    ap.add_argument("--no-big", action="store_true",
                    help="skip the 8M-vehicle city (beyond the Infinity Cache)")
    ap.add_argument("--junctions", action="store_true",
                    help="with --profile-only: step the 2M city built with junction internal "
                         "lanes instead of the snapshot")
    ap.add_argument("--no-junctions", action="store_true",
                    help="skip the 2M city built with junction internal lanes")
    ap.add_argument("--batch-scenarios", type=int, default=256)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="also copy a device buffer of this size once (calibrates the HBM "
                         "byte counters of a profiler run against a known transfer)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the simulator "
              "partitions no network across GPUs", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2405_12520_amd import scenarios as S
    from paper_2405_12520_amd.moss import Simulator

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_probe:
        src = torch.empty(args.copy_probe // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        say(f"[bench] copy probe: {args.copy_probe} bytes read and written")
        del src, dst
    if args.profile_only and (args.batch or args.big):
        if args.batch:
            sc = S.batch(args.batch_scenarios)
            say(f"[bench] batch generated: {sc.summary()}")
        else:
            sc = big_city()
        sim = Simulator(sc)
        if args.launch:
            sim.set_launch(**json.loads(args.launch))
        sim.step(args.warmup)
        sim.step(args.steps)
        torch.cuda.synchronize()
        _, _, err = sim.counters()
        say(f"[bench] {sc.name}: {args.warmup} + {args.steps} steps, {sim.n_active} active, "
            f"error word {err}")
        sim.close()
        if err:
            sys.exit(3)
        return
    say(f"[bench] generating city snapshot with {args.vehicles} vehicles")
    t0 = time.time()
    sc = S.city_snapshot(args.vehicles)
    say(f"[bench] generated in {time.time() - t0:.1f} s: {sc.summary()}")
    if args.profile_only and args.junctions:
        sc = junction_city(sc)
    if args.mlp:
        from paper_2405_12520_amd import closure
        theta, norm = closure.load(closure.DEFAULT_PATH)
        sc = sc.with_params(mlp=dict(theta=theta, norm=norm))
    launch = None
    if args.launch:
        from paper_2405_12520_amd import autotune
        launch = dict(launch=json.loads(args.launch), cached=True, ms_per_step=None)
    elif not (args.no_tune or args.profile_only):
        # launch shape tuned on a second copy at the same point of the run
        from paper_2405_12520_amd import autotune
        t0 = time.time()
        launch = autotune.tune(lambda: Simulator(sc), sc, args.warmup, log=say)
        torch.cuda.empty_cache()
        say(f"[bench] launch shape {launch['launch']} "
            f"({'cached' if launch['cached'] else 'searched'} in {time.time() - t0:.1f} s)")
    sim = Simulator(sc)
    if launch:
        autotune.apply(sim, launch)
    used = fit_graphs(sim, args.steps)
    stream = sim.stream
    say("[bench] created; warmup")
    sim.step(args.warmup)
    torch.cuda.synchronize()
    c0, _, _ = sim.counters()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    sim.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    c1, _, err = sim.counters()
    if err:
        print(f"device error word {err}", file=sys.stderr)
        sys.exit(3)
    veh_steps = int(c1[:, 6].sum() - c0[:, 6].sum())
    value = veh_steps / (ms / 1e3)
    say(f"[bench] {args.steps} steps in {ms:.2f} ms -> {value:.4g} vehicle-steps/s")
    if args.profile_only:
        return

    # per-kernel durations with HIP events on the simulator's stream
    kms = sim.step_timed(args.steps)
    n_act = sim.n_active
    per_launch = {k: v / args.steps for k, v in kms.items() if v > 0}
    dom = max(ALGO_BYTES, key=lambda k: per_launch[k])
    algo = ALGO_BYTES[dom] * n_act
    achieved = algo / (per_launch[dom] / 1e3) / 1e9
    traffic = load_traffic(dom)
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=None if traffic is None else round(traffic / per_launch[dom] / 1e6, 1),
                    kernel=dom, kernel_ms=round(per_launch[dom], 5),
                    algo_bytes_per_launch=int(algo),
                    traffic_bytes_per_launch=None if traffic is None else int(traffic),
                    kernel_ms_all={k: round(v, 5) for k, v in per_launch.items()})
    # whole-step fraction: algorithmic bytes of one step over the timed ms per step
    step_bytes = sum(ALGO_BYTES.values()) * n_act + STEP_LANE_BYTES * sc.n_lanes
    step_gbs = step_bytes / (ms / args.steps * 1e-3) / 1e9
    roofline["step"] = dict(algo_bytes=int(step_bytes), achieved=round(step_gbs, 1),
                            frac=round(step_gbs / HBM_PEAK_GBS, 4))
    say(f"[bench] per-kernel ms: {roofline['kernel_ms_all']}")
    sim.close()
    del sim
    torch.cuda.empty_cache()

    extras = {}
    if not args.no_mlp:
        extras["mlp"] = bench_mlp(sc, args)
    if not args.no_batch:
        extras["batch"] = bench_batch(args)
    if not args.no_big:
        extras["city8M"] = bench_big(args)
    if not args.no_junctions:
        extras["city_junction_lanes"] = bench_junctions(sc, used, args)
    if not args.no_demand:
        extras["city_demand"] = bench_demand(args)
    if not args.no_small:
        extras.update(bench_small(args))
    cpu = None if args.no_cpu else cpu_baseline(sc, args.cpu_steps, args.cpu_steps_mt)
    out = dict(metric=METRIC, value=round(value, 1), unit="vehicle-steps/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=round(ms / args.steps, 5),
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
               data="synthetic",
               config=dict(workload="city-scale synthetic network, 2M vehicles pre-placed, "
                                    "IDM car-following + randomised MOBIL, dt = 1 s",
                           vehicles=int(sc.n_veh), lanes=int(sc.n_lanes), roads=int(sc.n_roads),
                           nodes=int(sc.n_nodes), active_vehicles=int(n_act),
                           launch=used),
               roofline=roofline, cpu_baseline=cpu, **extras)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
