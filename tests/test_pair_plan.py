"""Host logic of the single-pair (intra-task) schedule: tiles cover the matrix,
the anti-diagonal count, the choice between tiles and the pipelined pass, the
workspace bound, argument checks (no GPU)."""
import pytest

import paper_2412_08308_amd as swdb
import synth

def _skew_chunks(b, n, K, wc):
    """Chunks of band b in the skewed score pass: lane g of band b covers, in
    chunk c, columns [c*wc - b*kr - g, +wc) with kr = K rounded up to 16; the
    first chunk holds the head's column 0, the last the tail's column n - 1."""
    kr = -(-K // 16) * 16
    return range(b * kr // wc, -(-(n + b * kr + K - 1) // wc))


def _skew_launches(m, n, R, K, wc):
    """Anti-diagonals b + c holding at least one tile (band intervals merged)."""
    nb = -(-m // (K * R))
    count, end = 0, -1
    for b in range(nb):
        ch = _skew_chunks(b, n, K, wc)
        lo, hi = b + ch.start, b + ch.stop - 1
        count += max(0, hi - max(lo, end + 1) + 1)
        end = max(end, hi)
    return count


@pytest.mark.parametrize("m,n", [(1, 1), (1, 5000), (5000, 1), (2047, 2049), (2048, 512), (20000, 15000)]
                         + synth.DNA_PAIR_SIZES)
def test_pair_plan_covers_matrix(m, n):
    p = swdb.pair_plan(m, n, swdb.options(pair_mode="tiles"))
    R, K, wc = p["rows"], p["lanes"], p["cols"]
    assert p["flow"] == 0
    assert R in (8, 16) and K in (1, 2, 4, 8, 16, 32, 64) and wc % 16 == 0
    assert p["bands"] == -(-m // (K * R)) and p["chunks"] == -(-n // wc)
    assert p["launches"] == _skew_launches(m, n, R, K, wc)
    assert p["workspace"] == swdb.pair_workspace_bytes(m, n) > 0
    assert p["est_ms"] > 0


@pytest.mark.parametrize("m,n", [(1, 5000), (2047, 2049), (20000, 15000)] + synth.DNA_PAIR_SIZES)
def test_pipelined_plan(m, n):
    """The pipelined pass: bands of 64 lanes x R rows in one launch, on at most
    16 waves per CU (8 beyond 6 rows per lane), chosen only where the scores
    fit its 24-bit words (max(SM) x min(m, n) < 2^24)."""
    for R in (4, 6, 8, 10, 12, 16):
        o = swdb.options(pair_mode="flow", pair_rows=R, pair_sm_max=1)
        p = swdb.pair_plan(m, n, o)
        assert p["flow"] == 1 and p["rows"] == R and p["lanes"] == 64 and p["launches"] == 1
        assert p["bands"] == -(-(-(-m // R)) // 64)
        assert p["workspace"] == swdb.pair_workspace_bytes(m, n) > 0
        # workgroups of W waves, one per CU: W band profiles fit the CU's LDS,
        # the registers allow W / 4 waves per SIMD, and the waves reach every
        # band (in rounds when there are more bands than waves)
        for eb in (1, 2):
            q = swdb.pair_plan(m, n, swdb.options(pair_mode="flow", pair_rows=R, pair_sm_max=1,
                                                  pair_entry_bytes=eb))
            W, G = q["group_waves"], q["groups"]
            stride = next(x for x in (4, 8, 16, 32) if R * eb <= x)
            assert 1 <= W <= (16 if R <= 6 else 8) and W * 33 * 64 * stride <= 160 * 1024
            assert 1 <= G <= 256 and G == min(-(-q["bands"] // W), 256)
    # scores that do not fit 24 bits: the pipelined pass is refused or not chosen
    big = swdb.options(pair_mode="flow", pair_sm_max=127)
    if 127 * min(m, n) >= 1 << 24:
        with pytest.raises(swdb.SwdbError):
            swdb.pair_plan(m, n, big)
        assert swdb.pair_plan(m, n, swdb.options(pair_sm_max=127))["flow"] == 0
    else:
        assert swdb.pair_plan(m, n, big)["flow"] == 1
    # the planner compares both and keeps the cheaper estimate
    auto = swdb.pair_plan(m, n, swdb.options(pair_sm_max=1))
    tiles = swdb.pair_plan(m, n, swdb.options(pair_mode="tiles"))
    assert auto["est_ms"] <= tiles["est_ms"] + 1e-9


def test_pipelined_rounds_follow_the_grid_cap():
    o = swdb.options(pair_mode="flow", pair_rows=4, pair_sm_max=1, grid_limit=2)
    p = swdb.pair_plan(20_000, 3_000, o)
    assert p["flow"] == 1 and p["bands"] == 79 and p["groups"] <= 2


def test_pipelined_shape_keeps_simds_even():
    """Up to one band per SIMD (1,024 on 256 CUs) the planner gives each band
    a SIMD of its own; the paper's DNA pairs all take the pipelined pass."""
    o = swdb.options(pair_sm_max=1, pair_entry_bytes=1)
    for m, n in [(162_000, 172_000), (543_000, 536_000), (1_000_000, 1_000_000)]:
        p = swdb.pair_plan(m, n, o)
        assert p["flow"] == 1 and p["bands"] <= 1024 and p["group_waves"] <= 4
        assert p["est_ms"] < swdb.pair_plan(m, n, swdb.options(pair_mode="tiles"))["est_ms"]
    with pytest.raises(swdb.SwdbError):
        swdb.pair_plan(10, 10, swdb.options(pair_entry_bytes=3))
    # the workgroup shape: one wave per CU up to a band per CU, forced shapes kept
    o = swdb.options(pair_mode="flow", pair_rows=4, pair_sm_max=1, pair_entry_bytes=1)
    assert swdb.pair_plan(50_000, 50_000, o)["group_waves"] == 1
    for W in (1, 2, 4, 8, 16):
        q = swdb.pair_plan(70_001, 2_000, swdb.options(pair_mode="flow", pair_rows=4, pair_sm_max=1,
                                                       pair_entry_bytes=1, pair_group_waves=W))
        assert q["group_waves"] == W and q["groups"] == min(-(-q["bands"] // W), 256)
    for bad in (3, 32, -1):
        with pytest.raises(swdb.SwdbError):
            swdb.pair_plan(1000, 1000, swdb.options(pair_mode="flow", pair_group_waves=bad))


@pytest.mark.parametrize("n,K,wc", [(1, 1, 16), (5, 64, 16), (100, 2, 16), (1000, 64, 64), (777, 16, 48),
                                    (4096, 8, 512), (33, 32, 16)])
def test_skewed_tiles_cover_each_row_block_once(n, K, wc):
    """Every lane's chunks of the skewed tiling cover columns 0..n-1 of its row
    block exactly once, and the launch count matches the planner's for forced
    tilings."""
    for b in range(6):
        for g in range(K):
            seen = []
            for c in _skew_chunks(b, n, K, wc):
                lo = c * wc - b * (-(-K // 16) * 16) - g
                seen.extend(j for j in range(lo, lo + wc) if 0 <= j < n)
            assert seen == list(range(n)), (b, g)
    for R in (8, 16):
        m = 6 * K * R
        o = swdb.options(pair_rows=R, max_lanes=K, pair_cols=wc, pair_mode="tiles")
        assert swdb.pair_plan(m, n, o)["launches"] == _skew_launches(m, n, R, K, wc)


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
    tiles = swdb.options(pair_mode="tiles")
    assert swdb.pair_plan(162_000, 172_000, tiles)["rows"] < 32
    assert swdb.pair_plan(10_000, 10_000, tiles)["rows"] == 8
    # the pipelined pass takes the fewest rows per lane on short pairs
    dna = swdb.options(pair_sm_max=1)
    assert swdb.pair_plan(162_000, 172_000, dna)["rows"] == 4
    assert swdb.pair_plan(1_000_000, 1_000_000, dna)["rows"] >= 8


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
    with pytest.raises(swdb.SwdbError):
        swdb.pair_plan(10, 10, swdb.options(pair_rows=4))       # 4 rows: pipelined pass only
    with pytest.raises(swdb.SwdbError):
        swdb.pair_plan(10, 10, swdb.options(pair_mode=3))
    with pytest.raises(swdb.SwdbError):
        swdb.pair_plan(10, 10, swdb.options(pair_mode="flow", pair_rows=7))
    with pytest.raises(swdb.SwdbError):
        swdb.pair_plan(10, 10, swdb.options(pair_sm_max=128))


def _a256(x):
    return (x + 255) // 256 * 256


def _align_extra(m, n, p, block, o):
    """Workspace past the pair buffers for the alignment schedule p: whole-
    matrix direction words, or checkpoint rows / columns, chunk maxima and the
    direction words of four blocks (8 rows x 64 lanes per band; the walk's
    block and the three neighbours computed beside it, each neighbour with a
    set of pair buffers, here at their bound); then the end key and walk state."""
    nb, nc, wc = p["bands"], p["chunks"], p["cols"]
    cols = nc * wc
    if block == 0 and m * n <= 1 << 35:
        return _a256(nb * 64 * cols * 4) + 512
    B = block or 65536
    gb, gc = -(-B // 512), -(-B // wc)
    dirs = _a256(gb * 64 * gc * wc * 4)
    return (_a256((nb - 1) // gb * cols * 8) + _a256((nc - 1) // gc * nb * 512 * 8) + _a256(nc * 4)
            + 4 * dirs + 3 * _a256(swdb.pair_workspace_bytes(m, n, o)) + 512)


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
                assert swdb.pair_workspace_bytes(m, n, o) + 256 + _align_extra(m, n, p, block, o) <= need, (block, wc, cu)


def test_align_workspace_blocks_beyond_whole_matrix_codes():
    # whole-matrix codes: half a byte per cell; blocks: checkpoints and the
    # codes of four 65,536 x 65,536 blocks (2 GiB each), far below the
    # half-byte-per-cell codes of the whole matrix (500 GB at 1M x 1M)
    assert swdb.align_workspace_bytes(162_000, 172_000) > 162_000 * 172_000 // 2
    assert swdb.align_workspace_bytes(1_000_000, 1_000_000) < 11 << 30
    assert swdb.align_workspace_bytes(7_000_000, 5_000_000) < 24 << 30
    small = swdb.align_workspace_bytes(3000, 4000, swdb.options(align_block=512))
    assert small < swdb.align_workspace_bytes(3000, 4000)
    for bad in (-1, (1 << 24) + 1):
        with pytest.raises(swdb.SwdbError):
            swdb.align_workspace_bytes(100, 100, swdb.options(align_block=bad))


def test_pair_plan_cache_keys_every_option():
    """Plans are cached per (lengths, device size, forced options): repeated
    calls agree, and a forced option never returns another call's plan."""
    m, n = 543_000, 536_000
    base = swdb.pair_plan(m, n, cu_count=256)
    assert swdb.pair_plan(m, n, cu_count=256) == base
    for R in (8, 16):
        for K in (16, 64):
            for wc in (128, 1024):
                p = swdb.pair_plan(m, n, swdb.options(pair_rows=R, max_lanes=K, pair_cols=wc), cu_count=256)
                assert (p["rows"], p["lanes"], p["cols"]) == (R, K, wc)
    assert swdb.pair_plan(m, n, cu_count=256) == base
    small = swdb.pair_plan(m, n, cu_count=32)
    assert small["est_ms"] > base["est_ms"]        # fewer compute units: a slower plan
    assert swdb.pair_plan(m, n, cu_count=256) == base


def test_pair_plan_every_option_gives_a_plan_or_an_error():
    """Every combination of the pair knobs either plans (a positive tiling or
    a pipelined shape with a finite estimate) or is rejected with an error,
    never a zero plan.  (The alignment also plans internally with row counts
    only the pipelined pass has, which this call rejects outside the pipelined
    mode; the GPU alignment test that forces the tiles covers that route.)"""
    import math
    for m, n in [(1, 1), (3000, 4000), (70_001, 2_000)]:
        for mode in ("auto", "tiles", "flow"):
            for R in (0, 4, 6, 8, 10, 12, 16, 24):
                for K in (0, 1, 8, 64):
                    for wc in (0, 16, 8192):
                        o = swdb.options(pair_mode=mode, pair_rows=R, max_lanes=K, pair_cols=wc, pair_sm_max=1)
                        try:
                            p = swdb.pair_plan(m, n, o)
                        except swdb.SwdbError:
                            continue
                        assert p["rows"] > 0 and p["lanes"] > 0 and math.isfinite(p["est_ms"])
                        assert p["flow"] or (p["cols"] > 0 and p["chunks"] > 0 and p["bands"] > 0)
                        if R and not p["flow"]:
                            assert p["rows"] == R
