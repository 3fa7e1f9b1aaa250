"""HIP simulator against the oracle on the hand-built rule states.

The states of tests/rule_cases.py sit on the boundaries of single rules
(insertion gap, stop-line condition, rear-gap safety, target-lane limit,
overlap clamp, equal-position order).  Both sides run them through the C ABI
and are compared after every step: state bit for bit (ids, lanes, cursors,
s, v, a), decisions and neighbours, and counters.
"""
import numpy as np
import pytest

import rule_cases as RC
from test_gpu_parity import compare_debug, sim_cls  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu

CASES = RC.all_cases()


@pytest.mark.parametrize("name,sc,steps", CASES, ids=[c[0] for c in CASES])
def test_rule_case(sim_cls, name, sc, steps):  # noqa: F811
    from oracle import OracleSim
    print("rule case", name, flush=True)
    g = sim_cls(sc, debug=True)
    o = OracleSim(sc)
    for t in range(steps):
        g.step(1)
        o.step(1)
        a, b = g.state(), o.state()
        assert a["id"].shape == b["id"].shape, (name, t)
        for f in ("id", "lane", "cursor"):
            assert np.array_equal(a[f], b[f]), (name, t, f)
        for f in ("s", "v", "a"):
            assert np.array_equal(a[f].view(np.uint32), b[f].view(np.uint32)), (name, t, f)
        da, db = g.debug(), o.debug()
        compare_debug(da, db, f"{name} t={t}")
        assert np.array_equal(da["flags"], db["flags"]), (name, t)
        assert np.array_equal(da["margin"].view(np.uint32), db["margin"].view(np.uint32))
    cg, svg, err = g.counters()
    co, svo = o.counters()
    assert err == 0
    assert np.array_equal(cg, co), (name, cg, co)
    np.testing.assert_array_equal(svg, svo)
    g.close()
