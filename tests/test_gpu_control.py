"""Runtime control on the GPU vs the oracle: the same signal phases and speed
limits given to both between steps leave identical states (bit for bit), on
a grid under max-pressure control and under random speed-limit changes."""
import sys

import numpy as np
import pytest

from paper_2405_12520_amd import scenarios as S

pytestmark = pytest.mark.gpu


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


def _same(g, o, where):
    a, b = g.state(), o.state()
    for f in ("id", "lane", "cursor"):
        assert np.array_equal(a[f], b[f]), (where, f)
    for f in ("s", "v", "a"):
        assert np.array_equal(a[f].view(np.uint32), b[f].view(np.uint32)), (where, f)


def test_max_pressure_control_parity(sim_cls):
    from oracle import OracleSim
    from paper_2405_12520_amd.control import MaxPressure
    sc = S.grid(10, 12000, horizon=900)
    _say("max pressure")
    g = sim_cls(sc)
    o = OracleSim(sc)
    ctl = MaxPressure(sc, period=10)
    switched = 0
    for k in range(60):
        before = ctl.phase.copy()
        ctl.run(g, 10, also=o)
        switched += int((ctl.phase != before).sum())
        if k % 6 == 5:
            _same(g, o, f"t={10 * (k + 1)}")
    _same(g, o, "end")
    assert switched > 0
    g.close()


def test_speed_limit_changes_parity(sim_cls):
    from oracle import OracleSim
    sc = S.grid(10, 8000, horizon=600)
    _say("speed limits")
    g = sim_cls(sc)
    o = OracleSim(sc)
    rng = np.random.default_rng(3)
    for k in range(8):
        lanes = rng.choice(sc.n_lanes, 200, replace=False).astype(np.int32)
        vl = rng.choice([5.0, 8.33, 11.11, 16.67], 200).astype(np.float32)
        g.set_lane_vlim(lanes, vl)
        o.set_lane_vlim(lanes, vl)
        g.step(40)
        o.step(40)
        _same(g, o, f"t={40 * (k + 1)}")
    g.close()


def test_control_rejects_bad_arguments(sim_cls):
    from paper_2405_12520_amd.moss import MossError
    sc = S.intersection()
    g = sim_cls(sc)
    g.step(100)
    st = g.state()
    with pytest.raises(MossError):
        g.set_signal_phase([1], [0])          # node 1 has no signal
    with pytest.raises(MossError):
        g.set_signal_phase([0], [-2])
    with pytest.raises(MossError):
        g.set_lane_vlim([sc.n_lanes], [10.0])
    with pytest.raises(MossError):
        g.set_lane_vlim([0], [0.0])
    st2 = g.state()
    for f in st:
        assert np.array_equal(st[f], st2[f])
    g.close()
