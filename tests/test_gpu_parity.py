"""HIP simulator vs CPU oracle, element by element, through the C ABI.

Both sides start from the same seeded scenario and are compared after every
step (or every few steps on long runs): ids, lanes and route cursors must be
identical, and so must the lane-change decisions, leaders and target-lane
neighbours of the step; positions and speeds must agree within 1e-5
relative.  Both sides evaluate the same FP32 expressions in the same order,
so in practice they agree to the bit; a decision mismatch is only excused
when the oracle's MOBIL margin is within 8 ulp of the threshold (a tie).
"""
import sys

import numpy as np
import pytest

from paper_2405_12520_amd import scenarios as S

pytestmark = pytest.mark.gpu

RTOL = 1e-5
ATOL = 1e-5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sim_cls():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_12520_amd.moss import Simulator
    return Simulator


def _oracle(sc):
    from oracle import OracleSim
    return OracleSim(sc)


def compare_state(g, o, where):
    assert g["id"].shape == o["id"].shape, (where, g["id"].shape, o["id"].shape)
    assert np.array_equal(g["id"], o["id"]), where
    assert np.array_equal(g["lane"], o["lane"]), where
    if "cursor" in g:
        assert np.array_equal(g["cursor"], o["cursor"]), where
    for f in ("s", "v", "a"):
        np.testing.assert_allclose(g[f], o[f], rtol=RTOL, atol=ATOL, err_msg=f"{where} {f}")
    return int(sum(np.count_nonzero(g[f].view(np.uint32) != o[f].view(np.uint32))
                   for f in ("s", "v", "a")))


def compare_debug(g, o, where):
    assert np.array_equal(g["id"], o["id"]), where
    ties = np.abs(o["margin"]) <= 8 * np.spacing(np.maximum(np.abs(o["margin"]), 1.0),
                                                    dtype=np.float32)
    lc_g, lc_o = g["flags"] & 3, o["flags"] & 3
    bad = (lc_g != lc_o) & ~ties
    assert not bad.any(), (where, np.flatnonzero(bad)[:5])
    same = lc_g == lc_o
    assert np.array_equal(g["leader"][same], o["leader"][same]), where
    assert np.array_equal(g["flags"][same], o["flags"][same]), where
    assert np.array_equal(g["t_leader"], o["t_leader"]), where
    assert np.array_equal(g["t_follower"], o["t_follower"]), where
    return int(np.count_nonzero(lc_g != lc_o))


def run_pair(sim_cls, sc, steps, every=1, debug=True):
    g = sim_cls(sc, debug=debug)
    o = _oracle(sc)
    compare_state(g.state(), o.state(), f"{sc.name} t=0")
    nbits = 0
    done = 0
    while done < steps:
        k = min(every, steps - done)
        g.step(k)
        o.step(k)
        done += k
        where = f"{sc.name} t={done}"
        nbits += compare_state(g.state(), o.state(), where)
        if debug and k == 1:
            compare_debug(g.debug(), o.debug(), where)
    cg, svg, err = g.counters()
    co, svo = o.counters()
    assert err == 0
    assert np.array_equal(cg, co), (cg, co)
    np.testing.assert_array_equal(svg, svo)
    g.close()
    return nbits


@pytest.mark.parametrize("seed", range(8))
def test_toy_per_step(sim_cls, seed):
    sc = S.toy(seed, n_placed=50, n_pending=25, horizon=40)
    _say("toy", seed)
    assert run_pair(sim_cls, sc, 80) == 0


def test_toy_many_lanes_dense(sim_cls):
    sc = S.toy(100, n=4, max_lanes=4, n_placed=300, n_pending=100, horizon=60,
               length_range=(60.0, 200.0))
    _say("toy dense")
    assert run_pair(sim_cls, sc, 120) == 0


def test_intersection_full_run(sim_cls):
    sc = S.intersection()
    _say("intersection")
    assert run_pair(sim_cls, sc, 3600, every=60, debug=False) == 0


def test_intersection_per_step_window(sim_cls):
    sc = S.intersection()
    _say("intersection per-step")
    assert run_pair(sim_cls, sc, 200) == 0


def test_grid_full_run(sim_cls):
    sc = S.grid()
    _say("grid10 full")
    assert run_pair(sim_cls, sc, 3600, every=300, debug=False) == 0


def test_grid_per_step_window(sim_cls):
    sc = S.grid()
    _say("grid10 per-step")
    assert run_pair(sim_cls, sc, 60) == 0


def test_grid_snapshot_p_lc_one(sim_cls):
    sc = S.grid_snapshot(10, 8000).with_params(p_lc=1.0)
    _say("grid snapshot p_lc=1")
    assert run_pair(sim_cls, sc, 40) == 0


def test_batch_small(sim_cls):
    sc = S.batch(12, horizon=300, vmin=200, vmax=3000)
    _say("batch 12")
    assert run_pair(sim_cls, sc, 400, every=50, debug=False) == 0


def test_ring_equilibrium_gpu(sim_cls):
    sc = S.ring(40, 1000.0, 10.073723, v0=14.0)
    _say("ring")
    assert run_pair(sim_cls, sc, 300, every=30) == 0


def test_empty_and_pending_only(sim_cls):
    net = S.corridor([200.0, 200.0], 2)
    _say("edge: no vehicles")
    sc = S.with_vehicles("empty", net, [])
    g = sim_cls(sc)
    g.step(5)
    assert g.state()["id"].shape[0] == 0
    g.close()
    _say("edge: pending only")
    vs = [dict(id=i, route=[0, 1], depart=i // 3) for i in range(30)]
    sc = S.with_vehicles("pending", net, vs)
    assert run_pair(sim_cls, sc, 200, every=1) == 0


def test_city_snapshot_full_size(sim_cls):
    """The benchmark workload at full size (2M vehicles on the city network),
    every row compared after each of the first steps."""
    sc = S.city_snapshot()
    _say("city 2M")
    g = sim_cls(sc, debug=True)
    o = _oracle(sc)
    for k in range(3):
        g.step(1)
        o.step(1)
        where = f"city t={k + 1}"
        assert compare_state(g.state(), o.state(), where) == 0
        compare_debug(g.debug(), o.debug(), where)
    cg, svg, err = g.counters()
    co, svo = o.counters()
    assert err == 0 and np.array_equal(cg, co)
    g.close()


def test_city_snapshot_long_run_bench_launch(sim_cls):
    """The benchmark workload at full size in the benchmark's launch shape
    (XCD-contiguous tiles, 16-step graph replays, the kernels without debug
    records): after 80 and 160 steps the whole state and the counters equal
    the oracle's, bit for bit."""
    sc = S.city_snapshot()
    _say("city 2M, 160 steps in the benchmark's launch shape")
    g = sim_cls(sc)
    g.set_launch(xcd_remap=1)
    o = _oracle(sc)
    for k in range(2):
        g.step(80)
        o.step(80)
        where = f"city t={80 * (k + 1)}"
        assert compare_state(g.state(), o.state(), where) == 0
        _say(where)
    cg, svg, err = g.counters()
    co, svo = o.counters()
    assert err == 0 and np.array_equal(cg, co)
    np.testing.assert_array_equal(svg, svo)
    g.close()


def test_city_8M_bench_launch(sim_cls):
    """The largest city the benchmark times (city network tiled 2 x 2: 8M
    vehicles on 482k lanes, past the on-die caches) in the launch shape the
    tuner picks for it (the default: tiles in index order): one 16-step graph
    replay, then 3 direct steps, the whole state and the counters equal to
    the oracle's bit for bit."""
    sc = S.city_snapshot(8_000_000, side=400, target_undirected=184_000, hops=24)
    _say("city 8M, 19 steps in the default launch shape")
    g = sim_cls(sc)
    o = _oracle(sc)
    for k in (16, 3):
        g.step(k)
        o.step(k)
        where = f"city8M t={o.t}"
        assert compare_state(g.state(), o.state(), where) == 0
        _say(where)
    cg, svg, err = g.counters()
    co, svo = o.counters()
    assert err == 0 and np.array_equal(cg, co)
    np.testing.assert_array_equal(svg, svo)
    g.close()


def test_checkpoint_resume(sim_cls):
    """Grid with departures over the hour, stopped at step 120: the pending
    list equals the vehicles that have not entered in the oracle's run (found
    by collecting every id ever active, step by step), and a new simulator
    created from the checkpoint runs 120 more steps into the same state as
    the uninterrupted run and as the oracle resumed from it, bit for bit; its
    counters are the difference of the original run's."""
    from oracle import OracleSim
    sc = S.grid()
    _say("checkpoint at 120, resume")
    g = sim_cls(sc)
    g.step(120)
    ck = g.checkpoint()
    assert ck["t"] == 120
    o = OracleSim(sc)
    seen = set(sc.veh_id[sc.placed == 1].tolist())
    for _ in range(120):
        o.step(1)
        seen |= set(o.state()["id"].tolist())
    pend = np.array(sorted(set(sc.veh_id.tolist()) - seen), np.uint32)
    assert len(pend) > 0
    assert np.array_equal(np.sort(ck["pending"]), pend)
    assert compare_state(ck["state"], o.state(), "grid t=120") == 0
    c1, _, _ = g.counters()
    g.step(120)
    c2, _, err = g.counters()
    full = g.state()
    g.close()
    assert err == 0
    rs = S.resume(sc, ck)
    b = sim_cls(rs)
    b.step(120)
    res = b.state()
    cb, _, errb = b.counters()
    b.close()
    assert errb == 0
    assert compare_state(res, full, "resumed vs uninterrupted t=240") == 0
    assert np.array_equal(cb, c2 - c1)
    r = OracleSim(rs)
    r.step(120)
    assert compare_state(res, r.state(), "resumed vs oracle t=240") == 0


def test_read_pending_capacity(sim_cls):
    """moss_read_pending refuses a buffer shorter than the pending list
    (MOSS_ENOMEM, count reported, nothing written), lists everything at the
    start of a run with departures, and nothing once all vehicles are
    placed."""
    import ctypes as C
    from paper_2405_12520_amd.moss import MOSS_ENOMEM, MossError, load, moss_read_pending
    sc = S.grid()
    g = sim_cls(sc)
    n = C.c_int32(-1)
    buf = np.full(4, 7, np.uint32)
    rc = load().moss_read_pending(C.c_void_p(g.h), 3, buf.ctypes.data_as(C.c_void_p),
                                  C.byref(n))
    assert rc == MOSS_ENOMEM and n.value == sc.n_veh and np.all(buf == 7)
    with pytest.raises(MossError):
        moss_read_pending(g.h, 3)
    assert np.array_equal(np.sort(g.pending()), np.sort(sc.veh_id))
    g.close()
    g = sim_cls(S.city_snapshot(20_000, side=40, target_undirected=1_800, hops=8))
    assert g.pending().shape == (0,)
    g.close()


def test_batch_full_size_long_run(sim_cls):
    """The 256-grid batch at full size (3.1M vehicles, departures spread over
    the run) in a tuned launch shape: insertions through the per-queue-lane
    rows and counters per scenario, 300 steps, state and counters bit for
    bit at steps 150 and 300."""
    sc = S.batch(256)
    _say("batch 256, 300 steps")
    g = sim_cls(sc)
    g.set_launch(xcd_remap=1)
    o = _oracle(sc)
    for k in range(2):
        g.step(150)
        o.step(150)
        where = f"batch t={150 * (k + 1)}"
        assert compare_state(g.state(), o.state(), where) == 0
        _say(where, g.n_active)
    cg, svg, err = g.counters()
    co, svo = o.counters()
    assert err == 0 and np.array_equal(cg, co)
    np.testing.assert_array_equal(svg, svo)
    g.close()


def test_graph_replay_matches_direct_steps(sim_cls):
    """Steps enqueued through the captured step graphs (16 at a time) give
    the same bits as steps launched one by one, replay after replay."""
    sc = S.grid(10, 6000, horizon=600)
    _say("graph vs direct")
    a = sim_cls(sc)
    b = sim_cls(sc)
    for _ in range(6):
        a.step(32)
        for _ in range(32):
            b.step(1)
        sa, sb = a.state(), b.state()
        for f in sa:
            assert np.array_equal(sa[f], sb[f]), f
    a.close()
    b.close()


@pytest.mark.parametrize("name", ["grid", "intersection"])
def test_timed_steps_match_graph_steps(sim_cls, name):
    """moss_step_timed (direct launches between events, 64 steps per
    synchronisation) computes the same steps as moss_step and reports every
    step kernel with a non-negative time: 0 for the yield-flag kernel of a
    network without junction lanes, and 0 for the lane-count block reduction
    of a network of one scan block (the intersection's 16 lanes).  Both have
    departures, so the update's launch carries the insertion workgroups."""
    from paper_2405_12520_amd.moss import kernel_names
    sc = S.grid(10, 6000, horizon=600) if name == "grid" else S.intersection()
    _say(f"timed vs graph steps: {name}")
    a = sim_cls(sc)
    b = sim_cls(sc)
    a.step(150)
    kms = b.step_timed(150)
    assert list(kms) == kernel_names()
    assert all(v >= 0.0 for v in kms.values()), kms
    assert kms["k_update"] > 0.0 and kms["k_merge"] > 0.0
    assert kms["k_yield"] == 0.0
    assert (kms["k_scan_reduce"] == 0.0) == (name == "intersection")
    sa, sb = a.state(), b.state()
    assert a.t == b.t == 150
    for f in sa:
        assert np.array_equal(sa[f], sb[f]), f
    ca, va, ea = a.counters()
    cb, vb, eb = b.counters()
    assert ea == 0 and eb == 0
    assert np.array_equal(ca, cb)
    np.testing.assert_array_equal(va, vb)
    a.close()
    b.close()


def test_device_reads_are_ordered_before_later_steps(sim_cls):
    """Device-pointer reads of the state and of the trace are complete when
    they return, so a step enqueued right after them cannot change what they
    copied (a device-to-device copy left unordered with the simulator's
    stream was overwritten by the next step's kernels).  2M vehicles, so
    that the copies take long enough for a race to show."""
    import torch
    sc = S.city_snapshot()
    _say("device reads vs later steps")
    g = sim_cls(sc, trace=True)
    for k in range(4):
        g.step(1)
        host = g.state(cursor=False)
        hf, hy = g.trace(device=False)
        dev = g.state_device()
        df, dy = g.trace(device=True)
        g.step(1)                       # enqueued at once: must not touch the copies
        torch.cuda.synchronize()
        for f in ("id", "lane", "s", "v", "a"):
            assert np.array_equal(dev[f].cpu().numpy().view(np.uint32),
                                  host[f].view(np.uint32)), (k, f)
        assert np.array_equal(df.cpu().numpy().view(np.uint32), hf.view(np.uint32)), k
        assert np.array_equal(dy.cpu().numpy().view(np.uint32), hy.view(np.uint32)), k
    g.close()


def _long_lanes():
    """Corridor whose lanes overflow the merge kernel's LDS tile (768 old or
    new rows, 160 joiners per 512-row chunk): lane 0 holds 900 vehicles
    (merged one lane per thread), and lanes 1 and 2 (100 and 700 vehicles)
    both start in the second chunk (rows 512..1023), which then only fits
    the tile as two groups of whole lanes.  Lane 0 is dense and lane 1
    sparse, so lane changes bring joiners into both groups."""
    net = S.corridor([7000.0, 5400.0, 300.0], 2)
    vehicles = []
    k = 0

    def put(lane, road, count, gap, v):
        nonlocal k
        for i in range(count):
            vehicles.append(dict(id=k, route=list(range(road, 3)), lane=lane,
                                 s=5.0 + gap * i, v=v, v0=12.0 + (k % 7)))
            k += 1
    put(0, 0, 900, 7.5, 2.0)
    put(1, 0, 100, 60.0, 8.0)
    put(2, 1, 700, 7.5, 1.0)
    put(3, 1, 40, 100.0, 8.0)
    return S.with_vehicles("long_lanes", net, vehicles)


def test_lanes_beyond_the_merge_tile(sim_cls):
    sc = _long_lanes()
    o = _oracle(sc)
    st = o.state()
    size = np.bincount(st["lane"], minlength=sc.n_lanes)
    start = np.concatenate([[0], np.cumsum(size)])[:-1]
    assert size.max() > 768                                   # a lane alone over the tile
    owned = [l for l in range(sc.n_lanes) if 512 <= start[l] < 1024]
    assert sum(size[l] for l in owned) > 768                  # a chunk of two groups
    _say("long lanes")
    assert run_pair(sim_cls, sc, 40) == 0
