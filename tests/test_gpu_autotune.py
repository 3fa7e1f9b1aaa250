"""Launch shapes and the tuner: every shape computes the same states.

The launch shape (steps per graph, update and scatter workgroup counts, XCD
tile order) regroups the work of a step; the state after N steps must be
bit-identical for all of them, on a batched workload (many scenarios, lanes
of every length) and on a pre-placed grid (many update tiles, persistent
update loop)."""
import sys

import numpy as np
import pytest

from paper_2405_12520_amd import scenarios as S

pytestmark = pytest.mark.gpu

SHAPES = [
    dict(graph_steps=16, update_blocks=0, scatter_blocks=0, xcd_remap=0),  # default
    dict(graph_steps=0, update_blocks=0, scatter_blocks=0, xcd_remap=0),   # no graphs
    dict(graph_steps=2, update_blocks=3, scatter_blocks=1, xcd_remap=0),
    dict(graph_steps=32, update_blocks=16, scatter_blocks=5, xcd_remap=1),
    dict(graph_steps=64, update_blocks=0, scatter_blocks=0, xcd_remap=1),
    dict(graph_steps=8, update_blocks=1000, scatter_blocks=4096, xcd_remap=1),
    dict(graph_steps=0, update_blocks=0, scatter_blocks=0, xcd_remap=1),   # serial, direct
]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _run(sc, shape, steps):
    from paper_2405_12520_amd.moss import Simulator
    g = Simulator(sc)
    g.set_launch(**shape)
    assert g.launch() == shape
    g.step(steps)
    st = g.state()
    cnt, sumv, err = g.counters()
    g.close()
    return st, cnt, sumv, err


def _same(a, b):
    sa, ca, va, ea = a
    sb, cb, vb, eb = b
    assert ea == 0 and eb == 0
    for k in ("id", "lane", "s", "v", "a", "cursor"):
        assert sa[k].shape == sb[k].shape, k
        assert np.array_equal(sa[k].view(np.uint32), sb[k].view(np.uint32)), k
    assert np.array_equal(ca, cb)
    # summed speeds are integer sums: the same bits in any order of atomics
    assert np.array_equal(va.view(np.uint64), vb.view(np.uint64))


@pytest.mark.parametrize("name", ["batch", "grid_snapshot"])
def test_every_launch_shape_gives_identical_state(torch_dev, name):
    sc = S.batch(24, horizon=600) if name == "batch" else S.grid_snapshot(10, 15000)
    steps = 200 if name == "batch" else 120
    ref = None
    for shape in SHAPES:
        _say(f"launch shape {name} {shape}")
        out = _run(sc, shape, steps)
        if ref is None:
            ref = out
            assert out[0]["id"].shape[0] > 0
        else:
            _same(ref, out)


def test_step_calls_of_any_length_give_identical_state(torch_dev):
    """A run split into calls of odd and uneven lengths (each call's part
    below the graph length launched step by step, starting from either
    lane-start parity) equals the same run in one call."""
    from paper_2405_12520_amd.moss import Simulator
    sc = S.batch(12, horizon=400)
    splits = [1, 3, 14, 17, 30, 5, 7, 31, 33, 9, 2, 48]
    ref = _run(sc, dict(graph_steps=16, update_blocks=0, scatter_blocks=0, xcd_remap=1),
               sum(splits))
    g = Simulator(sc)
    g.set_launch(xcd_remap=1)
    for n in splits:
        g.step(n)
    out = (g.state(), *g.counters())
    g.close()
    assert ref[0]["id"].shape[0] > 0
    _same(ref, out)


def test_set_launch_rejects_bad_shapes(torch_dev):
    from paper_2405_12520_amd.moss import MossError, Simulator
    g = Simulator(S.toy(3))
    before = g.launch()
    for bad in (dict(graph_steps=3), dict(graph_steps=-2), dict(graph_steps=258),
                dict(update_blocks=-1), dict(scatter_blocks=70000), dict(xcd_remap=2)):
        with pytest.raises(MossError):
            g.set_launch(**bad)
        assert g.launch() == before
    with pytest.raises(ValueError):
        g.set_launch(blocks=4)
    g.close()


def test_tuner_searches_then_reuses_cache(torch_dev, tmp_path, monkeypatch):
    from paper_2405_12520_amd import autotune
    from paper_2405_12520_amd.moss import Simulator
    monkeypatch.setenv("MOSS_TUNE_CACHE", str(tmp_path / "tune.json"))
    monkeypatch.setattr(autotune, "SPACE", {"graph_steps": [32], "xcd_remap": [1]})
    sc = S.batch(8, horizon=300)
    made = []

    def make():
        made.append(1)
        return Simulator(sc)

    _say("tuner search")
    rec = autotune.tune(make, sc, 100, steps=32)
    assert not rec["cached"] and len(made) == 3
    assert set(rec["launch"]) == set(autotune.DEFAULT)
    rec2 = autotune.tune(make, sc, 100)
    assert rec2["cached"] and rec2["launch"] == rec["launch"] and len(made) == 3
    g = Simulator(sc)
    autotune.apply(g, rec2)
    assert g.launch() == rec["launch"]
    g.close()
