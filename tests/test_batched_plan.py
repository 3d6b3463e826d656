"""Host logic of the batched STGD planner (no GPU call: the planner only reads
the problem table and the tuning cache and builds plain data).  Device
pointers are stand-in addresses that nothing dereferences here."""
import ctypes
import os

import pytest

from paper_1309_0787_amd import otm

pytestmark = pytest.mark.skipif(not os.path.exists(otm.LIB_PATH), reason="libotm.so not built")


def _problem(n, k, aliased=True, base=0x10000):
    ldy = otm.default_ldy(k)
    ya = base
    yb = ya if aliased else base + 0x1000
    yc = ya if aliased else base + 0x2000
    return otm._Problem(ya, yb, yc, base + 0x3000, None, 0, base + 0x4000, base + 0x5000, base + 0x6000,
                        n, k, ldy, 0, 0.5)


def _plan(problems, restarts=2, cache=None, y_dtype=otm.F32, passes=3):
    arr = (otm._Problem * len(problems))(*problems)
    p = otm.SgdParams(k=1, batch=100, passes=passes, y_dtype=y_dtype).c()
    plan = otm._vp()
    st = otm.lib().otm_sgd_batched_plan(arr, len(problems), restarts, ctypes.byref(p),
                                        cache.encode() if cache else None, 0x7000, None, ctypes.byref(plan))
    groups = []
    if st == 0:
        L = otm.lib()
        for g in range(L.otm_plan_groups(plan)):
            vals = [otm._i32() for _ in range(4)]
            assert L.otm_plan_group_info(plan, g, *[ctypes.byref(v) for v in vals]) == 0
            groups.append(tuple(v.value for v in vals))
        assert L.otm_plan_size(plan) > 0
        L.otm_plan_free(plan)
    return st, groups


def test_plan_groups_jobs_by_variant():
    st, groups = _plan([_problem(1000, 16), _problem(5000, 100, aliased=False), _problem(300, 128),
                        _problem(50, 9), _problem(700, 100, aliased=False)], restarts=4)
    assert st == 0
    # (padded k, layout, views, jobs), in variant order
    assert groups == [(16, 0, 1, 8), (112, 0, 3, 8), (128, 0, 1, 4)]


def test_plan_rejects_bad_input():
    assert _plan([_problem(1000, 129)])[0] == -8                 # k beyond capacity
    assert _plan([_problem(1000, 16)], y_dtype=otm.BF16)[0] == -3
    assert _plan([_problem(0, 16)])[0] == -2
    bad = _problem(1000, 16)
    bad.Phi0 = None
    assert _plan([bad])[0] == -1
    assert b"problem 0" in otm.lib().otm_last_error()


def test_tuning_cache_selects_the_layout(tmp_path):
    cache = tmp_path / "tune.txt"
    probs = [_problem(1000, 10), _problem(800, 100, aliased=False)]
    assert [g[1] for g in _plan(probs)[1]] == [0, 0]
    cache.write_text("# comment\nsgd_batched f32 kp=16 views=1 layout=1 us_step=3.0,2.0\n"
                     "sgd_batched f32 kp=112 views=3 layout=0 us_step=3.0,4.0\n")
    assert [(g[0], g[1]) for g in _plan(probs, cache=str(cache))[1]] == [(16, 1), (112, 0)]
    # entries for other shapes, malformed lines and a missing file leave the default
    cache.write_text("sgd_batched f32 kp=32 views=1 layout=1 us_step=3.0,2.0\ngarbage\n")
    assert [g[1] for g in _plan(probs, cache=str(cache))[1]] == [0, 0]
    assert [g[1] for g in _plan(probs, cache=str(tmp_path / "missing.txt"))[1]] == [0, 0]
