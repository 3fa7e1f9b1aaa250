"""Learned car-following closure on the GPU vs the FP64 references.

Network evaluation and gradients come from the project's HIP kernels through
the C ABI; references are oracle/mlp.py (numpy, FP64) and the C oracle's
network forward.  Tolerances follow from bfloat16 activations with FP32
accumulation: outputs within 1e-2 absolute, gradients within 1e-4 relative
in FP32 mode and 2e-2 in bfloat16 mode (norm-wise).
"""
import sys

import numpy as np
import pytest

from paper_2405_12520_amd import scenarios as S
from oracle import mlp as M

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _features(rng, n):
    f = np.empty((n, 8), np.float32)
    f[:, 0] = rng.uniform(-2, 300, n)
    f[:, 1] = rng.uniform(0, 18, n)
    f[:, 2] = np.clip(f[:, 1] + rng.normal(0, 2, n), 0, 20)
    f[:, 3] = rng.uniform(8, 17, n)
    f[:, 4] = np.where(rng.random(n) < 0.3, rng.uniform(0, 300, n), 300.0)
    f[:, 5] = rng.uniform(-9, 2, n)
    f[:, 6] = rng.uniform(0, 300, n)
    f[:, 7] = rng.choice([11.11, 13.89, 16.67], n)
    return f


def _norm_for(f):
    ft = f.astype(np.float64).copy()
    for q in M.LOG_INPUTS:
        ft[:, q] = np.log(np.maximum(ft[:, q], 0.5))
    mean = ft.mean(0)
    inv = 1.0 / np.maximum(ft.std(0), 1e-3)
    lo = np.full(8, -1e9, np.float32)
    hi = np.full(8, 1e9, np.float32)
    return np.concatenate([mean, inv, lo, hi]).astype(np.float32)


def test_predict_matches_oracle_forward(torch_dev):
    torch = torch_dev
    from paper_2405_12520_amd import moss
    from oracle import mlp_forward
    rng = np.random.default_rng(0)
    f = _features(rng, 1000)
    nrm = _norm_for(f)
    p = {k: np.array(v, np.float64) for k, v in M.unpack(M.init_params(7)).items()}
    p["b1"] = rng.uniform(-0.3, 0.3, M.N_H)
    p["b2"] = rng.uniform(-0.3, 0.3, M.N_H)
    p["b3"] = np.array([0.3])
    th = M.pack(p).astype(np.float32)
    _say("mlp predict")
    out = moss.mlp_predict(torch.from_numpy(f).cuda(), torch.from_numpy(th).cuda(),
                           torch.from_numpy(nrm).cuda()).cpu().numpy()
    z = M.normalise(f, nrm)
    ref = np.array([mlp_forward(th, z[i]) for i in range(f.shape[0])])
    err = np.abs(out - ref)
    assert err.max() < 1e-2, err.max()
    assert np.median(err) < 2e-3


@pytest.mark.parametrize("bf16", [False, True])
def test_gradient_matches_fp64_reference(torch_dev, bf16):
    torch = torch_dev
    from paper_2405_12520_amd import moss
    rng = np.random.default_rng(1)
    n = 2048
    f = _features(rng, n)
    nrm = _norm_for(f)
    lab = rng.normal(0, 1.5, n).astype(np.float32)
    th = M.init_params(11)
    _say("mlp grad bf16" if bf16 else "mlp grad fp32")
    loss, g = moss.mlp_grad(torch.from_numpy(f).cuda(), torch.from_numpy(lab).cuda(),
                            torch.from_numpy(th).cuda(), torch.from_numpy(nrm).cuda(), bf16=bf16)
    g = g.cpu().numpy().astype(np.float64)
    z = M.normalise(f, nrm)
    ref_loss, ref = M.loss_and_grad(th.astype(np.float64), z, lab, bf16_mode=bf16)
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    tol = 2e-2 if bf16 else 1e-4
    assert rel < tol, rel
    assert abs(float(loss.item()) - ref_loss) <= tol * ref_loss
    # the largest components individually
    big = np.argsort(-np.abs(ref))[:200]
    np.testing.assert_allclose(g[big], ref[big], rtol=5 * tol, atol=tol * np.abs(ref).max())


def test_adam_matches_reference(torch_dev):
    torch = torch_dev
    from paper_2405_12520_amd import moss
    rng = np.random.default_rng(2)
    th = M.init_params(3)
    m = rng.normal(0, 1e-3, M.N_PARAMS).astype(np.float32)
    v = rng.uniform(0, 1e-5, M.N_PARAMS).astype(np.float32)
    g = rng.normal(0, 1e-2, M.N_PARAMS).astype(np.float32)
    T = [torch.from_numpy(x.copy()).cuda() for x in (th, m, v, g)]
    moss.mlp_adam(T[0], T[1], T[2], T[3], step=5, lr=1e-3)
    # the ABI takes the hyperparameters as float32: the reference uses those values
    f32 = lambda x: float(np.float32(x))
    ref_t, ref_m, ref_v = M.adam(th.astype(np.float64), m.astype(np.float64),
                                 v.astype(np.float64), g.astype(np.float64), 5, lr=f32(1e-3),
                                 b1=f32(0.9), b2=f32(0.999), eps=f32(1e-8))
    np.testing.assert_allclose(T[0].cpu().numpy(), ref_t, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(T[1].cpu().numpy(), ref_m, rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(T[2].cpu().numpy(), ref_v, rtol=1e-5, atol=1e-12)


def test_gpu_training_fits_smooth_target(torch_dev):
    torch = torch_dev
    from paper_2405_12520_amd import moss
    rng = np.random.default_rng(4)
    n = 8192
    f = _features(rng, n)
    nrm = _norm_for(f)
    z = M.normalise(f, nrm)
    lab = (np.tanh(z[:, 0]) - 0.5 * z[:, 1] * z[:, 2]).astype(np.float32)
    F = torch.from_numpy(f).cuda()
    Y = torch.from_numpy(lab).cuda()
    N = torch.from_numpy(nrm).cuda()
    th = torch.from_numpy(M.init_params(4)).cuda()
    m = torch.zeros_like(th)
    v = torch.zeros_like(th)
    gen = torch.Generator(device="cuda").manual_seed(0)
    _say("mlp training")
    l0 = float(moss.mlp_grad(F, Y, th, N)[0].item())
    for step in range(1, 401):
        idx = torch.randint(0, n, (1024,), device="cuda", generator=gen, dtype=torch.int32)
        loss, g = moss.mlp_grad(F, Y, th, N, idx=idx)
        moss.mlp_adam(th, m, v, g, step, lr=3e-3)
    l1 = float(moss.mlp_grad(F, Y, th, N)[0].item())
    assert l1 < 0.1 * l0, (l0, l1)


# --------------------------------------------------------- simulator mode --

def _snapshot_from(sc, st, t):
    """Scenario whose vehicles are the given state's rows, all pre-placed."""
    pos = {int(i): k for k, i in enumerate(sc.veh_id)}
    order = [pos[int(i)] for i in st["id"]]
    routes = [sc.route_roads[sc.route_off[k]:sc.route_off[k + 1]] for k in order]
    off = np.zeros(len(routes) + 1, np.int64)
    off[1:] = np.cumsum([len(r) for r in routes])
    flat = np.concatenate(routes).astype(np.int32) if routes else np.zeros(0, np.int32)
    n = len(order)
    import dataclasses
    p = dict(sc.params)
    p["t0"] = int(t)
    return dataclasses.replace(
        sc, veh_id=st["id"].astype(np.uint32), depart=sc.depart[order], v0=sc.v0[order],
        route_off=off, route_roads=flat, placed=np.ones(n, np.uint8),
        lane=st["lane"].astype(np.int32), s=st["s"].astype(np.float32),
        v=st["v"].astype(np.float32), a=st["a"].astype(np.float32),
        cursor=st["cursor"].astype(np.int32), params=p)


def _mlp_cfg():
    """Closure weights for the network-mode parity cases: seeded He-style
    layers with non-zero hidden biases (a dropped bias term shows) and an
    output layer scaled by 12 with bias 1.0, so that on the 10 x 10 grid
    about 4% of the evaluated outputs fall above a_max and 0.5% below
    -b_max and the output limits bind."""
    p = {k: np.array(v, np.float64) for k, v in M.unpack(M.init_params(21)).items()}
    rng = np.random.default_rng(22)
    p["b1"] = rng.uniform(-0.3, 0.3, M.N_H)
    p["b2"] = rng.uniform(-0.3, 0.3, M.N_H)
    p["w3"] = 12.0 * p["w3"]
    p["b3"] = np.array([1.0])
    th = M.pack(p).astype(np.float32)
    mean = np.array([3.5, 8, 8, 13, 5.0, 0, 4.5, 14], np.float32)
    inv = 1.0 / np.array([1.5, 5, 5, 2, 1.0, 2, 1.2, 2], np.float32)
    lo = np.array([-10, 0, 0, 0, 0, -10, 0, 0], np.float32)
    hi = np.array([250, 25, 25, 25, 300, 3, 300, 20], np.float32)
    return dict(theta=th, norm=np.concatenate([mean, inv, lo, hi]).astype(np.float32))


def test_trace_labels_equal_oracle_accelerations(torch_dev):
    """With the trace on (IDM mode) the recorded labels are the IDM
    accelerations of the step, bit for bit the oracle's."""
    from paper_2405_12520_amd.moss import Simulator
    from oracle import OracleSim
    sc = S.grid_snapshot(10, 6000)
    _say("trace labels")
    g = Simulator(sc, trace=True)
    o = OracleSim(sc)
    for _ in range(3):
        ids_before = g.state()["id"]
        g.step(1)
        o.step(1)
        f, y = g.trace(device=False)
        st = o.state()
        a_by_id = dict(zip(st["id"].tolist(), st["a"].tolist()))
        assert f.shape == (ids_before.shape[0], 8)
        got = np.array([a_by_id.get(int(i), np.nan) for i in ids_before], np.float32)
        keep = ~np.isnan(got)
        assert keep.mean() > 0.99
        assert np.array_equal(y[keep].view(np.uint32), got[keep].view(np.uint32))
        assert np.all(f[:, 0] <= sc.params["d_look"]) and np.all(f[:, 6] <= sc.params["d_look"])
    g.close()


def check_network_step(gs, o, sc, theta, norm, label, list_max=400):
    """One network-mode step of the GPU (state gs) against the oracle o,
    which has just run the same step from the same start.  Element by
    element, for every vehicle:

    - network evaluated: the GPU's acceleration lies within 1e-3 of an
      output the oracle admits for that vehicle's inputs (its own first;
      others only where a hidden activation's FP32 error interval holds a
      bfloat16 rounding boundary, see orc_mlp_candidates).  A vehicle that
      needs another candidate than the oracle's own is excused and listed
      with its tie;
    - IDM (outside the envelope): the acceleration bit for bit;
    - lane and route cursor identical, except for a vehicle whose own
      acceleration differs and which crossed a road end on one side only
      (its position on the far side within the resulting difference);
    - position and speed within 1e-3 plus the largest acceleration
      difference in its lane (a clamped follower inherits its leader's).
    Returns the number of excused vehicles."""
    from oracle import mlp_candidates
    st = o.state()
    dbg = o.debug()
    f, use = o.mlp_inputs()
    p = sc.params
    assert gs["id"].shape == st["id"].shape, label
    assert np.array_equal(np.sort(gs["id"]), np.sort(st["id"])), label
    og = np.argsort(gs["id"], kind="stable")
    oo = np.argsort(st["id"], kind="stable")
    ids = st["id"][oo]
    G = {k: gs[k][og] for k in ("lane", "cursor", "s", "v", "a")}
    O = {k: st[k][oo] for k in ("lane", "cursor", "s", "v", "a")}
    # the network's use per vehicle, from the oracle's own inputs
    ev_ids = dbg["id"][use == 1]
    out, cnt, info = mlp_candidates(theta, norm, f[use == 1], -p["b_max"], p["a_max"])
    pos = np.searchsorted(ids, ev_ids)
    assert np.array_equal(ids[pos], ev_ids), label
    evaluated = np.zeros(len(ids), bool)
    evaluated[pos] = True
    ag, ao = G["a"].astype(np.float64), O["a"].astype(np.float64)
    da = np.abs(ag - ao)
    # IDM vehicles: bit for bit
    idm = ~evaluated
    assert np.array_equal(G["a"][idm].view(np.uint32), O["a"][idm].view(np.uint32)), label
    # evaluated: within 1e-3 of an admissible output
    dbest = np.nanmin(np.abs(out - ag[pos][:, None]), axis=1)
    worst = int(np.argmax(dbest))
    assert dbest.max() < 1e-3, (label, float(dbest.max()), int(ev_ids[worst]), out[worst, :8],
                                float(ag[pos][worst]), info[worst])
    exc = np.flatnonzero(da[pos] >= 1e-3)
    lines = ["%s: %d of %d evaluated vehicles excused (output of an admissible rounding, not "
             "the oracle's own; max |da| to the nearest admissible output %.2e)"
             % (label, len(exc), len(pos), float(dbest.max()))]
    for k in exc[:list_max]:
        lines.append("  id %d: |da| %.4f, ties layer1 %d layer2 %d, input pairs %d, first tied "
                     "unit %s, admissible %s" % (
                         ev_ids[k], da[pos][k], info[k, 0], info[k, 1], info[k, 2],
                         ("L%d.%d" % (1 + info[k, 3] // 64, info[k, 3] % 64))
                         if info[k, 3] >= 0 else "-",
                         np.round(out[k, :min(cnt[k], 6)], 4).tolist()))
    print("\n".join(lines), flush=True)
    # lanes and cursors
    mis = (G["lane"] != O["lane"]) | (G["cursor"] != O["cursor"])
    for k in np.flatnonzero(mis):
        assert da[k] > 0, (label, "lane/cursor differ with identical acceleration", int(ids[k]))
        far = min(float(G["s"][k]), float(O["s"][k]))
        assert far <= 0.5 * da[k] * p["dt"] ** 2 + 1e-3, (label, int(ids[k]), far, da[k])
    # positions and speeds in lanes, with the lane's largest acceleration difference
    same = ~mis
    lane = O["lane"][same]
    mx = np.zeros(int(max(O["lane"].max(), G["lane"].max())) + 1)
    np.maximum.at(mx, O["lane"], da)
    bound = 1e-3 + mx[lane] * p["dt"]
    ds = np.abs(G["s"][same].astype(np.float64) - O["s"][same])
    dv = np.abs(G["v"][same].astype(np.float64) - O["v"][same])
    assert (ds <= 0.5 * bound * p["dt"] + 1e-3).all(), (label, float(ds.max()))
    assert (dv <= bound).all(), (label, float(dv.max()))
    return len(exc)


def test_mlp_mode_step_parity(torch_dev):
    """MLP mode, one step at a time from identical states (re-synchronised
    from the oracle after each step), every vehicle checked element by
    element (check_network_step); counters of network use identical."""
    from paper_2405_12520_amd.moss import Simulator
    from oracle import OracleSim
    base = S.grid_snapshot(10, 8000)
    cfg = _mlp_cfg()
    sc = base.with_params(mlp=cfg)
    o = OracleSim(sc)
    st = o.state()
    _say("mlp mode parity")
    for k in range(4):
        snap = _snapshot_from(sc, st, o.t)
        g = Simulator(snap)
        g.step(1)
        gs = g.state()
        cg, _, err = g.counters()
        g.close()
        o.step(1)
        co, _ = o.counters()
        assert err == 0
        check_network_step(gs, o, sc, cfg["theta"], cfg["norm"], f"grid step {k}")
        if k == 0:
            # the step exercises both output limits
            f, use = o.mlp_inputs()
            y, _ = M.forward(cfg["theta"], M.normalise(f[use == 1], cfg["norm"]))
            assert (y > sc.params["a_max"]).sum() > 0 and (y < -sc.params["b_max"]).sum() > 0
        st = o.state()
        # evaluations and fallbacks of this step
        ev_o = co[0, 7] - (0 if k == 0 else prev_ev)
        assert cg[0, 7] == ev_o and cg[0, 8] == co[0, 8] - (0 if k == 0 else prev_fb)
        prev_ev, prev_fb = co[0, 7], co[0, 8]


@pytest.mark.parametrize("name", ["departures", "junction_lanes"])
def test_mlp_mode_step_parity_with_departures(torch_dev, name):
    """Network mode on networks with departure queues, so that the update's
    launch carries the insertion workgroups, on a 10 x 10 grid and on a 6 x 6
    grid built with junction internal lanes (the update variant with lane
    successors, the turn bias and the yield rule): from the oracle's state,
    queues and step (a resumed scenario), one GPU step against the oracle's,
    every vehicle checked element by element, insertions and failures
    equal."""
    from paper_2405_12520_amd import junctions as J
    from paper_2405_12520_amd.moss import Simulator
    from oracle import OracleSim
    cfg = _mlp_cfg()
    if name == "departures":
        sc = S.grid(10, 6000, horizon=300).with_params(mlp=cfg)
    else:
        sc = J.with_junction_lanes(S.grid(6, 3000, horizon=300)).with_params(mlp=cfg)
    o = OracleSim(sc)
    o.step(60)
    _say(f"mlp mode parity: {name}")
    for k in range(3):
        tr = o.trips()
        ck = dict(state=o.state(), pending=tr["id"][tr["status"] == 0], t=o.t)
        assert len(ck["pending"]) > 0 and len(ck["state"]["id"]) > 0
        g = Simulator(S.resume(sc, ck))
        g.step(1)
        gs = g.state()
        cg, _, err = g.counters()
        g.close()
        co0, _ = o.counters()
        o.step(1)
        co, _ = o.counters()
        assert err == 0
        assert cg[0, 0] == co[0, 0] - co0[0, 0] and cg[0, 1] == co[0, 1] - co0[0, 1]
        assert cg[0, 0] > 0
        check_network_step(gs, o, sc, cfg["theta"], cfg["norm"], f"{name} step {k}")


def test_mlp_mode_city_full_size(torch_dev):
    """The network-mode workload the benchmark reports (2M-vehicle city, the
    trained closure weights, the benchmark's launch shape), one step from
    the same start on both sides, every vehicle checked element by element
    (check_network_step): accelerations within 1e-3 of an admissible output
    of the closure's definition, IDM vehicles bit for bit, lanes and cursors
    identical but for road-end crossings caused by an acceleration
    difference, network evaluations and fallbacks counted identically.
    Excused vehicles (another admissible rounding than the oracle's own) are
    listed with their tie."""
    from paper_2405_12520_amd import closure
    from paper_2405_12520_amd.moss import Simulator
    from oracle import OracleSim, max_threads
    theta, norm = closure.load(closure.DEFAULT_PATH)
    sc = S.city_snapshot().with_params(mlp=dict(theta=theta, norm=norm))
    _say("mlp mode, 2M city, one step")
    g = Simulator(sc)
    g.set_launch(xcd_remap=1)
    g.step(1)
    gs = g.state()
    cg, _, err = g.counters()
    g.close()
    o = OracleSim(sc)
    o.set_threads(max_threads())
    o.step(1)
    co, _ = o.counters()
    assert err == 0
    n_exc = check_network_step(gs, o, sc, theta, norm, "2M city")
    assert n_exc <= 1e-3 * int(co[0, 7])
    assert cg[0, 7] == co[0, 7] and cg[0, 8] == co[0, 8]
