"""Host logic of the single-pair (intra-task) schedule: tiles cover the matrix,
the anti-diagonal count, the workspace bound, argument checks (no GPU)."""
import pytest

import paper_2412_08308_amd as swdb
import synth

@pytest.mark.parametrize("m,n", [(1, 1), (1, 5000), (5000, 1), (2047, 2049), (2048, 512), (20000, 15000)]
                         + synth.DNA_PAIR_SIZES)
def test_pair_plan_covers_matrix(m, n):
    p = swdb.pair_plan(m, n)
    R, K, wc = p["rows"], p["lanes"], p["cols"]
    assert R in (8, 16) and K in (1, 2, 4, 8, 16, 32, 64) and wc % 16 == 0
    assert p["bands"] == -(-m // (K * R)) and p["chunks"] == -(-n // wc)
    assert p["launches"] == p["bands"] + p["chunks"] - 1
    assert p["workspace"] == swdb.pair_workspace_bytes(m, n) > 0
    assert p["est_ms"] > 0


def test_pair_plan_options_fix_the_tiling():
    for R in (8, 16):
        for K in (1, 4, 64):
            for wc in (16, 64, 4096):
                o = swdb.options(pair_rows=R, max_lanes=K, pair_cols=wc)
                p = swdb.pair_plan(3000, 4000, o)
                assert (p["rows"], p["lanes"], p["cols"]) == (R, K, wc)
                assert p["workspace"] == swdb.pair_workspace_bytes(3000, 4000, o)


def test_pair_plan_prefers_short_strips_for_short_pairs():
    """Fewer rows per lane put more lanes on each anti-diagonal: the planner
    takes them when the pair is too short to fill the device otherwise."""
    assert swdb.pair_plan(162_000, 172_000)["rows"] < 32
    assert swdb.pair_plan(10_000, 10_000)["rows"] == 8


def test_pair_workspace_covers_every_tiling():
    """The workspace bound does not depend on the schedule the device picks."""
    import ctypes
    for m, n in [(100, 100), (5000, 70000), (162_000, 172_000)]:
        base = swdb.pair_workspace_bytes(m, n)
        for R in (8, 16):
            for K in (1, 8, 64):
                for wc in (16, 512, 8192):
                    o = swdb.options(pair_rows=R, max_lanes=K, pair_cols=wc)
                    assert swdb.pair_workspace_bytes(m, n, o) >= base
        # larger planner choices on other devices stay within the bound
        for cu in (1, 32, 256, 1024):
            assert swdb.pair_plan(m, n, cu_count=cu)["workspace"] == base


def test_pair_argument_checks():
    with pytest.raises(swdb.SwdbError):
        swdb.pair_plan(-1, 10)
    with pytest.raises(swdb.SwdbError):
        swdb.pair_plan(10, 10, swdb.options(max_lanes=3))       # not a power of two
    with pytest.raises(swdb.SwdbError):
        swdb.pair_plan(10, 10, swdb.options(pair_cols=24))      # not a multiple of 16
    with pytest.raises(swdb.SwdbError):
        swdb.pair_workspace_bytes(1 << 25, 10)
    with pytest.raises(swdb.SwdbError):
        swdb.pair_plan(10, 10, swdb.options(pair_rows=32))
