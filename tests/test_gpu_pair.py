"""Single long pair (intra-task, anti-diagonal tile launches) against the CPU
oracle (GPU required).  Scores are integers: the bar is equality.  Homologous
pairs make the optimal alignment cross many tile boundaries (rows, columns
and corners); explicit tilings force every lane-group width and chunk width,
including single-lane bands and 16-column chunks."""
import numpy as np
import pytest

import synth
from gpuhelp import announce, have_gpu, oracle_pair

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

DNA = (synth.dna_matrix(synth.DNA_MATCH, synth.DNA_MISMATCH), synth.DNA_GAP_OPEN, synth.DNA_GAP_EXTEND)


def _gpu_pair(a, b, sm, go, ge, **kw):
    import torch
    import paper_2412_08308_amd as swdb
    opt = swdb.options(**kw) if kw else None
    qa = torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint8)).cuda()
    qb = torch.from_numpy(np.ascontiguousarray(b, dtype=np.uint8)).cuda()
    out = swdb.pair_score(qa, qb, sm, go, ge, opt=opt)
    torch.cuda.synchronize()
    return int(out.cpu().item())


@pytest.mark.parametrize("m,n", [(1, 1), (1, 3000), (3000, 1), (31, 33), (2047, 2049), (2048, 512),
                                 (4000, 6000), (9000, 7000)])
def test_dna_pairs(m, n):
    a, b = synth.dna_pair(m, n, seed=m + 7 * n)
    sm, go, ge = DNA
    exp = oracle_pair(a, b, sm, go, ge)
    announce(f"pair m={m} n={n}")
    assert _gpu_pair(a, b, sm, go, ge) == exp


@pytest.mark.parametrize("R", [8, 16])
@pytest.mark.parametrize("K", [1, 2, 8, 64])
@pytest.mark.parametrize("wc", [16, 64, 512])
def test_tilings(R, K, wc):
    a, b = synth.dna_pair(3000, 3500, seed=5, identity=0.7, indel_rate=0.02)
    sm, go, ge = DNA
    exp = oracle_pair(a, b, sm, go, ge)
    announce(f"pair tiling R={R} K={K} cols={wc}")
    assert _gpu_pair(a, b, sm, go, ge, pair_rows=R, max_lanes=K, pair_cols=wc) == exp


@pytest.mark.parametrize("m,n", [(1, 700), (700, 1), (7, 3), (600, 20), (20, 600), (513, 17), (17, 513),
                                 (1100, 1030)])
@pytest.mark.parametrize("R,K,wc", [(8, 1, 16), (8, 64, 16), (16, 64, 32), (16, 4, 48), (8, 16, 128)])
def test_skewed_tile_edges(m, n, R, K, wc):
    """Skewed tiles at the matrix's edges: sequences shorter than a band or a
    chunk, very unequal lengths, chunks narrower than the band-to-band skew
    (K = 64 with 16 columns: several chunks of a band lie wholly left of
    column 0), and lane groups below 16 (the skew is rounded up to 16)."""
    a, b = synth.dna_pair(m, n, seed=3 * m + n, identity=0.8, indel_rate=0.03)
    sm, go, ge = DNA
    exp = oracle_pair(a, b, sm, go, ge)
    announce(f"pair skewed edges m={m} n={n} R={R} K={K} cols={wc}")
    assert _gpu_pair(a, b, sm, go, ge, pair_rows=R, max_lanes=K, pair_cols=wc) == exp


@pytest.mark.parametrize("go,ge", [(10, 2), (0, 3), (3, 5), (120, 1)])
def test_protein_pairs_profile_widths(go, ge):
    # (10, 2) and (0, 3): 8-bit profile entries; (120, 1): 16-bit (11 + 120 > 127)
    rng = np.random.default_rng(go * 31 + ge)
    sm = synth.blosum_style_matrix()
    a = synth.residues(rng, 2500)
    b = synth.mutate(rng, a, 0.6)
    exp = oracle_pair(a, b, sm, go, ge)
    announce(f"protein pair go={go} ge={ge}")
    for R in (8, 16):
        assert _gpu_pair(a, b, sm, go, ge, pair_rows=R, max_lanes=16, pair_cols=256) == exp
    assert _gpu_pair(a, b, sm, go, ge) == exp


def test_empty_and_swapped():
    sm, go, ge = DNA
    a, b = synth.dna_pair(1500, 2500, seed=3)
    announce("pair empty / swapped")
    assert _gpu_pair(a[:0], b, sm, go, ge) == 0
    assert _gpu_pair(a, b[:0], sm, go, ge) == 0
    # the score is symmetric in the roles of the two sequences for a symmetric matrix
    assert _gpu_pair(a, b, sm, go, ge) == _gpu_pair(b, a, sm, go, ge) == oracle_pair(a, b, sm, go, ge)


def test_large_identity_closed_form():
    """A sequence against itself scores its length times the match score (no
    alignment can do better: every base contributes at most one match); at a
    size far beyond what the oracle finishes, across thousands of tiles."""
    sm, go, ge = DNA
    rng = np.random.default_rng(21)
    a = synth.residues(rng, 300_000, synth.DNA_FREQS)
    announce("pair 300k self")
    assert _gpu_pair(a, a, sm, go, ge) == 300_000
    # a substring of it scores its own length
    assert _gpu_pair(a, a[123_456:223_456], sm, go, ge) == 100_000


def test_large_tilings_agree():
    """The paper's smallest DNA pair size (162K x 172K, 28G cells): every tiling
    gives the planner's score."""
    sm, go, ge = DNA
    a, b = synth.dna_pair(162_000, 172_000, seed=1)
    announce("pair 162k x 172k")
    ref = _gpu_pair(a, b, sm, go, ge)
    assert ref > 0.2 * 162_000          # a long homologous alignment (about 0.3 per base)
    for R, K, wc in ((16, 16, 256), (16, 64, 4096), (8, 64, 512), (16, 32, 1024)):
        assert _gpu_pair(a, b, sm, go, ge, pair_rows=R, max_lanes=K, pair_cols=wc) == ref


FLOW_ROWS = [4, 6, 8, 10, 12, 16]


@pytest.mark.parametrize("R", FLOW_ROWS)
@pytest.mark.parametrize("m,n", [(1, 1), (1, 700), (700, 1), (5, 16), (17, 15), (63, 64), (257, 300),
                                 (1000, 1500), (2900, 3500)])
def test_flow_pass(R, m, n):
    """The pipelined pass (one launch, bands hand their bottom rows to the
    band below through tagged words): sequences shorter than a band, the
    pipeline fill and drain, bands past the query's end, every R."""
    a, b = synth.dna_pair(m, n, seed=11 * m + n, identity=0.8, indel_rate=0.03)
    sm, go, ge = DNA
    exp = oracle_pair(a, b, sm, go, ge)
    announce(f"flow pass m={m} n={n} R={R}")
    assert _gpu_pair(a, b, sm, go, ge, pair_mode=2, pair_rows=R) == exp


@pytest.mark.parametrize("R", [4, 16])
def test_flow_pass_rounds(R):
    """More bands than wavefronts: waves take bands w, w + waves, ... in
    rounds (a cap of one or two workgroups), the last band ragged."""
    a, b = synth.dna_pair(5000, 3000, seed=31, identity=0.75, indel_rate=0.02)
    sm, go, ge = DNA
    exp = oracle_pair(a, b, sm, go, ge)
    for grid in (1, 2):
        announce(f"flow pass rounds R={R} grid={grid}")
        assert _gpu_pair(a, b, sm, go, ge, pair_mode=2, pair_rows=R, grid_limit=grid) == exp


@pytest.mark.parametrize("m,n,R,grid,W", [(70_001, 2_000, 4, 0, 0), (70_001, 2_000, 16, 0, 0), (30_000, 1_500, 6, 3, 0),
                                           (30_000, 1_500, 12, 5, 0), (9_000, 700, 8, 1, 0), (70_001, 2_000, 4, 0, 1),
                                           (70_001, 2_000, 4, 0, 2), (70_001, 2_000, 6, 0, 8), (9_000, 700, 4, 1, 16),
                                           (30_000, 1_500, 16, 2, 4)])
def test_flow_pass_workgroup_shapes(m, n, R, grid, W):
    """Workgroups of several waves, each wave a band of its own with its own
    LDS profile: the shapes the planner picks for a few hundred bands and
    under a workgroup cap (rounds, waves left without a band)."""
    import paper_2412_08308_amd as swdb
    a, b = synth.dna_pair(m, n, seed=m + R, identity=0.8, indel_rate=0.01)
    sm, go, ge = DNA
    exp = oracle_pair(a, b, sm, go, ge)
    p = swdb.pair_plan(m, n, swdb.options(pair_mode=2, pair_rows=R, grid_limit=grid, pair_sm_max=1,
                                          pair_entry_bytes=1, pair_group_waves=W))
    announce(f"flow shapes m={m} n={n} R={R} grid={grid} W={W}: {p['groups']} x {p['group_waves']} waves")
    assert p["flow"] == 1 and p["group_waves"] >= 1 and (W == 0 or p["group_waves"] == W)
    assert _gpu_pair(a, b, sm, go, ge, pair_mode=2, pair_rows=R, grid_limit=grid, pair_group_waves=W) == exp


@pytest.mark.parametrize("go,ge", [(10, 2), (120, 1)])
def test_flow_pass_protein(go, ge):
    """Protein pairs through the pipelined pass with both profile widths
    (8-bit entries for (10, 2), 16-bit for (120, 1)), and a substring pair
    whose alignment crosses many bands."""
    rng = np.random.default_rng(go + 7 * ge)
    sm = synth.blosum_style_matrix()
    a = synth.residues(rng, 3100)
    b = np.concatenate([synth.residues(rng, 300), synth.mutate(rng, a[100:2900], 0.7), synth.residues(rng, 200)])
    exp = oracle_pair(a, b, sm, go, ge)
    for R in (4, 8, 12):
        announce(f"flow protein go={go} ge={ge} R={R}")
        assert _gpu_pair(a, b, sm, go, ge, pair_mode=2, pair_rows=R) == exp
        assert _gpu_pair(b, a, sm, go, ge, pair_mode=2, pair_rows=R) == exp


def test_flow_pass_refused_when_scores_do_not_fit():
    """Scores that could reach 2^24 are not packed into the handoff words:
    the pipelined pass is refused, the planner keeps the tiles."""
    import torch
    import paper_2412_08308_amd as swdb
    sm = np.full((32, 32), -1, dtype=np.int32)
    np.fill_diagonal(sm, 127)
    m = n = 140_000                                   # 127 * 140,000 > 2^24
    qa = torch.zeros(m, dtype=torch.uint8, device="cuda")
    qb = torch.zeros(n, dtype=torch.uint8, device="cuda")
    announce("flow refused")
    with pytest.raises(swdb.SwdbError):
        swdb.pair_score(qa, qb, sm, 5, 2, opt=swdb.options(pair_mode=2))
    assert swdb.pair_plan(m, n, swdb.options(pair_sm_max=127))["flow"] == 0


def test_flow_large_closed_form():
    """300,000 bases against themselves and a 100,000-base substring through
    the pipelined pass (1,172 bands of 4 rows x 64 lanes, two per SIMD)."""
    sm, go, ge = DNA
    rng = np.random.default_rng(21)
    a = synth.residues(rng, 300_000, synth.DNA_FREQS)
    for R in (4, 16):
        announce(f"flow 300k self R={R}")
        assert _gpu_pair(a, a, sm, go, ge, pair_mode=2, pair_rows=R) == 300_000
        assert _gpu_pair(a, a[123_456:223_456], sm, go, ge, pair_mode=2, pair_rows=R) == 100_000
