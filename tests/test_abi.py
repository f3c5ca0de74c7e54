"""C-ABI contract checks that need no GPU: the library loads, exports every
function ``include/swdb.h`` declares, and rejects bad arguments before any HIP
call."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2412_08308_amd as swdb
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "swdb.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sw_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["sw_db_search", "sw_db_prepare", "sw_db_release", "sw_db_search_ex",
                     "sw_db_search_batch", "sw_workspace_bytes", "sw_strerror", "sw_version"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    L = swdb.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_version_and_errors():
    assert "gfx950" in swdb.version()
    L = swdb.lib()
    for code in (0, -1, -2, -3, -4, -5):
        assert L.sw_strerror(code)
    assert L.sw_strerror(-99) == b"unknown error"


SM = np.zeros((32, 32), dtype=np.int32)


def _call_search(qlen=4, nseq=1, go=10, ge=2, sm=SM, query=1, scores=1):
    L = swdb.lib()
    return L.sw_db_search(ctypes.c_void_p(query), qlen, ctypes.c_void_p(1), ctypes.c_void_p(1),
                          ctypes.c_void_p(1), nseq, sm.ctypes.data if sm is not None else None,
                          go, ge, ctypes.c_void_p(scores), None)


@pytest.mark.parametrize("kw", [dict(qlen=-1), dict(nseq=-5), dict(go=-1), dict(ge=-2),
                                dict(go=32001), dict(sm=None), dict(query=0),
                                dict(scores=0)])
def test_one_shot_rejects_bad_arguments(kw):
    assert _call_search(**kw) == -1


def test_matrix_range_checked():
    bad = SM.copy()
    bad[3, 4] = 128
    assert _call_search(sm=bad) == -1
    bad[3, 4] = -129
    assert _call_search(sm=bad) == -1


def test_empty_database_is_a_no_op():
    assert _call_search(nseq=0) == 0


def test_handle_calls_reject_null():
    L = swdb.lib()
    assert L.sw_db_release(None) == -1
    assert L.sw_db_info(None, None, None, None) == -1
    ql = np.array([10], dtype=np.int32)
    assert L.sw_workspace_bytes(None, 1, ql.ctypes.data, None) == 0
    st = swdb.PlanStats()
    assert L.sw_plan_info(None, 1, ql.ctypes.data, None, ctypes.byref(st)) == -1
    assert L.sw_db_search_ex(None, None, 0, SM.ctypes.data, 1, 1, None, None, 0, None, None) == -1
    assert L.sw_db_search_batch(None, None, None, None, 0, SM.ctypes.data, 1, 1, None, None, 0,
                                None, None) == -1
    assert L.sw_flagged_count(None, None) == -1
    h = ctypes.c_void_p()
    assert L.sw_db_prepare(None, None, None, -1, None, ctypes.byref(h)) == -1
    assert L.sw_db_prepare(None, None, None, 3, None, ctypes.byref(h)) == -1
    assert L.sw_db_prepare(None, None, None, 0, None, None) == -1


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(swdb, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(swdb, "_lib", None)
    with pytest.raises(swdb.SwdbError):
        swdb.lib()


def test_select_variant():
    """8-bit profile entries wherever every s + Go fits the lane type's range."""
    sm = synth.blosum_style_matrix()          # entries -4..11
    assert swdb.select_variant(sm, 10) == 3                                  # packed, [0, 127]
    assert swdb.select_variant(sm, 0) == 2                                   # -4 + 0 < 0
    assert swdb.select_variant(sm, 10, swdb.options(wide_profile=1)) == 2
    assert swdb.select_variant(sm, 10, swdb.options(mode="i32")) == 0
    assert swdb.select_variant(sm, 0, swdb.options(mode="i32")) == 0        # [-128, 127]
    assert swdb.select_variant(sm, 120, swdb.options(mode="i32")) == 1      # 131 > 127
    assert swdb.select_variant(sm, 10, swdb.options(mode="tuned")) == 3
    with pytest.raises(swdb.SwdbError):
        swdb.select_variant(sm, -1)
    with pytest.raises(swdb.SwdbError):
        swdb.select_variant(sm, 10, swdb.options(wide_profile=2))
