"""C-ABI checks that need no GPU: the library loads, exports every entry
point declared in include/moss.h, and rejects malformed inputs on the host
(moss_query_workspace runs validation only)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2405_12520_amd import moss, scenarios as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            names |= set(re.findall(r"^\s*(?:int|size_t|const char \*|void)\s*\*?\s*(moss_\w+)\s*\(",
                                    txt, re.M))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = moss.load()
    names = declared_functions()
    assert {"moss_create", "moss_step", "moss_read_state", "moss_destroy"} <= set(names)
    for n in names:
        assert hasattr(L, n), n
    assert set(moss.EXPORTS) == set(names)


def _query(sc, **mut):
    net, sig, veh, prm, keep = moss.marshal(sc)
    for k, v in mut.items():
        obj, field = k.split("__")
        setattr({"net": net, "sig": sig, "veh": veh, "prm": prm}[obj], field, v)
    return moss.moss_query_workspace(net, sig, veh, prm)


def test_workspace_size_scales():
    a = _query(S.grid(4, 100))
    b = _query(S.grid(4, 1000))
    assert 0 < a < b


def _arr(x, dt):
    a = np.ascontiguousarray(x, dtype=dt)
    _arr.keep.append(a)
    return a.ctypes.data_as(C.c_void_p)


_arr.keep = []


@pytest.mark.parametrize("case", ["route_not_chain", "dup_id", "bad_dt", "p_lc", "overlap_ok",
                                  "overlap",
                                  "lane_gap", "reserved_id", "empty_route", "nan_v0"])
def test_validation_errors(case):
    sc = S.toy(3, n_placed=20, n_pending=5)
    if case == "route_not_chain":
        rr = sc.route_roads.copy()
        rr[1] = rr[0]                      # a road never follows itself on this grid
        sc.route_roads = rr
    elif case == "dup_id":
        ids = sc.veh_id.copy()
        ids[1] = ids[0]
        sc.veh_id = ids
    elif case == "reserved_id":
        ids = sc.veh_id.copy()
        ids[0] = 0xFFFFFFFF
        sc.veh_id = ids
    elif case == "bad_dt":
        sc = sc.with_params(dt=0.0)
    elif case == "p_lc":
        sc = sc.with_params(p_lc=1.5)
    elif case == "lane_gap":
        l0 = sc.road_lane0.copy()
        l0[2] += 1
        sc.road_lane0 = l0
    elif case == "empty_route":
        off = sc.route_off.copy()
        off[1] = off[0]
        sc.route_off = off
    elif case == "nan_v0":
        v0 = sc.v0.copy()
        v0[3] = np.nan
        sc.v0 = v0
    elif case == "overlap":
        # placed vehicle b given a's route, lane and position, 1 m ahead of
        # a: less than a vehicle length apart
        pl = np.flatnonzero(sc.placed)
        a, b = int(pl[0]), int(pl[1])
        ra, rb = int(sc.route_off[a]), int(sc.route_off[b])
        k = int(sc.route_off[a + 1]) - ra
        assert int(sc.route_off[b + 1]) - rb == k
        rr, lane, cur, pos = sc.route_roads.copy(), sc.lane.copy(), sc.cursor.copy(), sc.s.copy()
        rr[rb:rb + k] = rr[ra:ra + k]
        lane[b], cur[b], pos[b] = lane[a], cur[a], pos[a] + 1.0
        assert pos[b] < sc.road_length[rr[ra + cur[a]]]
        sc.route_roads, sc.lane, sc.cursor, sc.s = rr, lane, cur, pos
    elif case == "overlap_ok":
        assert _query(sc) > 0
        return
    with pytest.raises(moss.MossError) as ei:
        _query(sc)
    assert ei.value.code == moss.MOSS_EINVAL
    assert moss.moss_last_error() != ""


def test_create_refuses_a_small_workspace_before_touching_the_device():
    """MOSS_ENOMEM when the workspace is smaller than moss_query_workspace
    says; checked on the host, before the pointer is ever used."""
    sc = S.toy(3, n_placed=20, n_pending=5)
    net, sig, veh, prm, keep = moss.marshal(sc)
    need = moss.moss_query_workspace(net, sig, veh, prm)
    out = C.c_void_p()
    rc = moss.load().moss_create(C.byref(net), C.byref(sig), C.byref(veh), C.byref(prm),
                                 C.c_void_p(256), need - 1, None, C.byref(out))
    assert rc == moss.MOSS_ENOMEM
    assert "needed" in moss.moss_last_error()
    assert not out.value


def test_static_gradient_refuses_a_batch_beyond_its_scratch():
    """moss_mlp_grad_static checks the batch size against its static scratch
    on the host, before any device work."""
    L = moss.load()
    fake = C.c_void_p(256)
    n = moss.MLP_STATIC_MAX_SAMPLES + 1
    rc = L.moss_mlp_grad_static(fake, fake, None, n, fake, fake, 1, -9.0, 2.0, fake, None, None)
    assert rc == moss.MOSS_EINVAL
    assert "at most %d" % moss.MLP_STATIC_MAX_SAMPLES in moss.moss_last_error()


def test_step_kernel_names():
    """The step kernels in timing order, read through moss_kernel_name (a
    host table; no GPU needed); out-of-range indices give NULL."""
    from paper_2405_12520_amd import moss
    names = moss.kernel_names()
    assert names == ["k_update", "k_scan_reduce", "k_scan_apply", "k_jscatter", "k_merge",
                     "k_yield"]
    assert moss.load().moss_kernel_name(-1) is None
    assert moss.load().moss_kernel_name(len(names)) is None
