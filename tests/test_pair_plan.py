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


def _a256(x):
    return (x + 255) // 256 * 256


def _align_extra(m, n, p, block):
    """Workspace past the pair buffers for the alignment schedule p: whole-
    matrix direction words, or checkpoint rows / columns, chunk maxima and one
    block's direction words (8 rows x 64 lanes per band); then the end key and
    walk state."""
    nb, nc, wc = p["bands"], p["chunks"], p["cols"]
    cols = nc * wc
    if block == 0 and m * n <= 1 << 35:
        return _a256(nb * 64 * cols * 4) + 512
    B = block or 65536
    gb, gc = -(-B // 512), -(-B // wc)
    return (_a256((nb - 1) // gb * cols * 8) + _a256((nc - 1) // gc * nb * 512 * 8) + _a256(nc * 4)
            + _a256(gb * 64 * gc * wc * 4) + 512)


@pytest.mark.parametrize("m,n", [(3000, 4000), (162_000, 172_000), (1_000_000, 1_000_000), (7_000_000, 5_000_000)])
def test_align_workspace_covers_every_tiling(m, n):
    """sw_align_workspace_bytes bounds the alignment layout of every chunk width
    the device's planner may pick (any CU count, any explicit width), for
    whole-matrix codes and for blocks."""
    for block in (0, 512, 700, 65536):
        for wc in (0, 16, 512, 8192, 65536):
            o = swdb.options(align_block=block, pair_cols=wc)
            need = swdb.align_workspace_bytes(m, n, o)
            for cu in (1, 32, 256, 1024):
                p = swdb.pair_plan(m, n, swdb.options(pair_rows=8, max_lanes=64, pair_cols=wc), cu_count=cu)
                assert (p["rows"], p["lanes"]) == (8, 64)
                assert swdb.pair_workspace_bytes(m, n, o) + 256 + _align_extra(m, n, p, block) <= need, (block, wc, cu)


def test_align_workspace_blocks_beyond_whole_matrix_codes():
    # whole-matrix codes: half a byte per cell; blocks: checkpoints + one block
    assert swdb.align_workspace_bytes(162_000, 172_000) > 162_000 * 172_000 // 2
    assert swdb.align_workspace_bytes(1_000_000, 1_000_000) < 4 << 30
    assert swdb.align_workspace_bytes(7_000_000, 5_000_000) < 24 << 30
    small = swdb.align_workspace_bytes(3000, 4000, swdb.options(align_block=512))
    assert small < swdb.align_workspace_bytes(3000, 4000)
    for bad in (-1, (1 << 24) + 1):
        with pytest.raises(swdb.SwdbError):
            swdb.align_workspace_bytes(100, 100, swdb.options(align_block=bad))
