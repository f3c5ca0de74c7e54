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
    for required in ["sw_db_search", "sw_db_prepare", "sw_db_prepare_bytes", "sw_db_release", "sw_db_search_ex",
                     "sw_db_search_batch", "sw_workspace_bytes", "sw_search_status", "sw_flagged_count",
                     "sw_strerror", "sw_version"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    L = swdb.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_version_and_errors():
    assert "gfx950" in swdb.version()
    L = swdb.lib()
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
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
    assert L.sw_db_prepare(None, None, None, -1, ctypes.c_void_p(256), 1 << 20, None, ctypes.byref(h)) == -1
    assert L.sw_db_prepare(None, None, None, 3, ctypes.c_void_p(256), 1 << 20, None, ctypes.byref(h)) == -1
    assert L.sw_db_prepare(None, None, None, 0, ctypes.c_void_p(256), 1 << 20, None, None) == -1
    # the workspace: required, 256-byte aligned
    assert L.sw_db_prepare(ctypes.c_void_p(1), ctypes.c_void_p(8), ctypes.c_void_p(8), 3, None, 1 << 20, None,
                           ctypes.byref(h)) == -1
    assert L.sw_db_prepare(ctypes.c_void_p(1), ctypes.c_void_p(8), ctypes.c_void_p(8), 3, ctypes.c_void_p(264),
                           1 << 20, None, ctypes.byref(h)) == -1
    assert L.sw_search_status(None, None, None) == -1
    assert L.sw_search_status_async(None, None, None) == -1
    assert L.sw_status_code(None) == -1


def test_prepare_bytes_bounds_and_monotone():
    """sw_db_prepare_bytes: an upper bound of the exact layout (residues padded
    per 64-subject chunk to its longest member, 1 KiB per 16 columns of a chunk,
    plus metadata), monotone in each argument, 0 on inconsistent input."""
    L = swdb.lib()
    f = L.sw_db_prepare_bytes
    rng = np.random.default_rng(3)
    for _ in range(200):
        nseq = int(rng.integers(1, 3000))
        lens = rng.integers(0, int(rng.choice([5, 60, 400, 5000])), size=nseq)
        total, mx = int(lens.sum()), int(lens.max())
        if mx == 0:
            continue
        s = np.sort(lens)[::-1]
        exact_res = sum(64 * ((int(s[c]) + 15) // 16 * 16) for c in range(0, nseq, 64))
        meta = 12 * nseq
        got = f(total, nseq, mx)
        assert got >= exact_res + meta
        assert got <= exact_res + meta + 64 * 16 * 3 + 1024 * 8 + 960 * ((nseq + 63) // 64) + 64 * mx
        # monotone in every argument (where the arguments stay consistent)
        assert f(total + 1, nseq, mx) >= got
        assert f(total, nseq + 1, mx) >= got
        if mx + 1 <= total:
            assert f(total, nseq, mx + 1) >= got
    assert f(0, 0, 0) > 0                 # an empty database still has a (tiny) layout
    assert f(-1, 5, 3) == 0
    assert f(10, 5, 11) == 0              # longest longer than the total
    assert f(100, 5, 3) == 0              # 5 subjects of at most 3 cannot hold 100
    assert f(5, 0, 0) == 0


def test_prepare_rejects_small_workspace_before_hip():
    """A workspace below the layout's metadata is SW_ENOMEM before any HIP
    call (so on a host without a GPU too)."""
    L = swdb.lib()
    h = ctypes.c_void_p()
    nseq = 1000
    rc = L.sw_db_prepare(ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 21), ctypes.c_void_p(1 << 22), nseq,
                         ctypes.c_void_p(1 << 23), 4096, None, ctypes.byref(h))
    assert rc == -2 and not h.value


def test_status_codes():
    """sw_status_code decodes the status words in priority order."""
    L = swdb.lib()
    for words, code in [((0, 0, 0, 0), 0), ((0, 0, 7, 0), 0), ((1, 0, 0, 0), -5), ((1, 3, 0, 1), -5),
                        ((0, 2, 5, 0), -6), ((0, 2, 0, 1), -6), ((0, 0, 0, 1), -7)]:
        st = swdb.Status(*words)
        assert L.sw_status_code(ctypes.byref(st)) == code
        err = swdb.status_error(np.array(words, dtype=np.int32))
        assert (err is None) == (code == 0)
        if err is not None:
            assert err.code == code


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
