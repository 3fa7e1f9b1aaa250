"""Host logic of the benchmark that needs no GPU: the graph length chosen
for a timed region (every timed step inside a whole graph replay)."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_graph_length_divides_the_timed_steps():
    b = _bench()
    # the tuned length is kept when it divides the steps (or graphs are off)
    assert b.graph_len_for(3600, 16) == 16
    assert b.graph_len_for(128, 32) == 32
    assert b.graph_len_for(20, 0) == 0
    # otherwise the even divisor nearest to it, the longer one on a tie
    assert b.graph_len_for(20, 16) == 20
    assert b.graph_len_for(200, 16) == 20
    assert b.graph_len_for(50, 16) == 10
    assert b.graph_len_for(12, 8) == 6
    assert b.graph_len_for(12, 9) == 12       # 6 and 12 equally near
    # no even divisor (odd step counts): the tuned length stays
    assert b.graph_len_for(21, 16) == 16
    for steps in range(2, 600, 2):
        for tuned in (2, 16, 32, 64):
            g = b.graph_len_for(steps, tuned)
            assert g % 2 == 0 and 2 <= g <= 256 and steps % g == 0, (steps, tuned, g)
