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
