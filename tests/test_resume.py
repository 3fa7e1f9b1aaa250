"""Checkpoint and resume: a run continued in a new simulator from the state
rows, the ids still waiting and the step index equals the uninterrupted run.

A step reads only the vehicle state and the departure queues (Sec. III-A),
so nothing else has to be carried over; counters restart at zero, and the
resumed run's counters equal the difference of the original run's.
"""
import numpy as np

from paper_2405_12520_amd import scenarios as S
from oracle import OracleSim


def _inserted_ids_stepwise(sim, sc, steps):
    """Steps one at a time and collects every id ever active: a vehicle shows
    up in the state after the step that inserts it and cannot arrive in that
    step, so this is exactly the set of vehicles that have entered."""
    seen = set(sc.veh_id[sc.placed == 1].tolist())
    seen |= set(sim.state()["id"].tolist())
    for _ in range(steps):
        sim.step(1)
        seen |= set(sim.state()["id"].tolist())
    return seen


def pending_after(sc, steps):
    o = OracleSim(sc)
    seen = _inserted_ids_stepwise(o, sc, steps)
    pend = np.array(sorted(set(sc.veh_id.tolist()) - seen), np.uint32)
    return o, pend


def _same_state(x, y):
    """Every field equal, floats bit for bit."""
    assert x.keys() == y.keys()
    for k in x:
        assert x[k].dtype == y[k].dtype, k
        bits = (lambda z: z.view(np.uint32)) if x[k].dtype == np.float32 else (lambda z: z)
        assert np.array_equal(bits(x[k]), bits(y[k])), k


def test_resume_builds_the_same_vehicles_at_step_zero():
    sc = S.toy(3, n_placed=50, n_pending=25, horizon=40)
    o = OracleSim(sc)
    ck = dict(state=o.state(), pending=sc.veh_id[sc.placed == 0], t=0)
    r = S.resume(sc, ck)
    assert r.n_veh == sc.n_veh and int(r.placed.sum()) == int(sc.placed.sum())
    a, b = OracleSim(sc), OracleSim(r)
    a.step(60)
    b.step(60)
    _same_state(a.state(), b.state())


def test_resume_mid_run_oracle():
    """Grid with departures over the hour: stopped at step 120 (vehicles have
    entered, arrived and still wait), resumed, 120 more steps."""
    sc = S.grid()
    o, pend = pending_after(sc, 120)
    c1, _ = o.counters()
    assert c1[0, 2] > 0 and len(pend) > 0      # arrivals happened, vehicles still wait
    ck = dict(state=o.state(), pending=pend, t=o.t)
    o.step(120)
    c2, _ = o.counters()
    r = OracleSim(S.resume(sc, ck))
    assert r.t == 120
    r.step(120)
    _same_state(o.state(), r.state())
    cr, _ = r.counters()
    assert np.array_equal(cr, c2 - c1)


def test_checkpoint_file_round_trip(tmp_path):
    """A checkpoint saved to disk and loaded back resumes into the same run."""
    sc = S.grid()
    o, pend = pending_after(sc, 40)
    ck = dict(state=o.state(), pending=pend, t=o.t)
    path = str(tmp_path / "ck.npz")
    S.save_checkpoint(path, ck)
    back = S.load_checkpoint(path)
    assert back["t"] == 40 and np.array_equal(back["pending"], pend)
    _same_state(ck["state"], back["state"])
    a, b = OracleSim(S.resume(sc, ck)), OracleSim(S.resume(sc, back))
    a.step(30)
    b.step(30)
    _same_state(a.state(), b.state())


def test_resume_rejects_unknown_ids():
    sc = S.toy(1, n_placed=10, n_pending=5, horizon=20)
    o = OracleSim(sc)
    bad = np.array([sc.veh_id.max() + 7], np.uint32)
    try:
        S.resume(sc, dict(state=o.state(), pending=bad, t=0))
    except ValueError:
        return
    raise AssertionError("unknown id accepted")
