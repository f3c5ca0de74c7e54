"""Alignment of one pair (direction-code pass + traceback walk) against the
oracle's traceback (GPU required).  Equality of the whole result: score,
begin and end positions, and every operation -- the tie-breaks are part of
the definition (see oracle.align)."""
import numpy as np
import pytest

import oracle
import synth
from gpuhelp import announce, have_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

DNA = (synth.dna_matrix(synth.DNA_MATCH, synth.DNA_MISMATCH), synth.DNA_GAP_OPEN, synth.DNA_GAP_EXTEND)


def _gpu_align(a, b, sm, go, ge, **kw):
    import torch
    import paper_2412_08308_amd as swdb
    qa = torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint8)).cuda()
    qb = torch.from_numpy(np.ascontiguousarray(b, dtype=np.uint8)).cuda()
    return swdb.align_pair(qa, qb, sm, go, ge, opt=swdb.options(**kw) if kw else None)


@pytest.mark.parametrize("m,n", [(1, 1), (1, 50), (50, 1), (31, 33), (300, 400), (1000, 1500), (2000, 2000)])
def test_dna_alignments(m, n):
    a, b = synth.dna_pair(m, n, seed=3 * m + n, identity=0.75, indel_rate=0.02)
    sm, go, ge = DNA
    announce(f"align m={m} n={n}")
    assert _gpu_align(a, b, sm, go, ge) == oracle.align(a, b, sm, go, ge)


@pytest.mark.parametrize("mode", ["tiles", "flow"])
def test_score_pass_either_way(mode):
    """With whole-matrix codes the score comes from the tile pass or the
    pipelined pass (the planner's choice, forced here), the codes from the
    tiles: the alignment is the oracle's either way."""
    sm, go, ge = DNA
    for m, n, seed in [(2000, 2300, 5), (700, 5000, 6), (4100, 900, 7)]:
        a, b = synth.dna_pair(m, n, seed=seed, identity=0.8, indel_rate=0.02)
        announce(f"align m={m} n={n} score pass {mode}")
        assert _gpu_align(a, b, sm, go, ge, pair_mode=mode) == oracle.align(a, b, sm, go, ge)
    rng = np.random.default_rng(61)
    psm = synth.blosum_style_matrix()
    a = synth.residues(rng, 900)
    b = np.concatenate([synth.residues(rng, 200), synth.mutate(rng, a[100:700], 0.6), synth.residues(rng, 150)])
    announce(f"align protein score pass {mode}")
    assert _gpu_align(a, b, psm, 10, 2, pair_mode=mode) == oracle.align(a, b, psm, 10, 2)


@pytest.mark.parametrize("rows", [4, 8])
def test_pipelined_code_pass_rows(rows):
    """The pipelined code pass with its row count fixed: 8 rows per lane fill
    a direction word, 4 rows one half of it; row counts just past a band
    (256 rows at 4, 512 at 8) and narrow or wide pairs."""
    sm, go, ge = DNA
    for m, n, seed in [(257, 900, 11), (513, 700, 12), (2001, 2300, 13), (77, 3000, 14), (4103, 900, 15)]:
        a, b = synth.dna_pair(m, n, seed=seed, identity=0.8, indel_rate=0.02)
        announce(f"align m={m} n={n} code pass rows={rows}")
        assert _gpu_align(a, b, sm, go, ge, pair_mode="flow", pair_rows=rows) == oracle.align(a, b, sm, go, ge)


@pytest.mark.parametrize("go,ge", [(10, 2), (0, 3), (4, 4), (120, 1)])
def test_protein_alignments(go, ge):
    # (120, 1): 16-bit profile entries; the others 8-bit
    rng = np.random.default_rng(go + 17 * ge)
    sm = synth.blosum_style_matrix()
    a = synth.residues(rng, 600)
    b = np.concatenate([synth.residues(rng, 100), synth.mutate(rng, a[150:500], 0.6), synth.residues(rng, 80)])
    announce(f"align protein go={go} ge={ge}")
    assert _gpu_align(a, b, sm, go, ge) == oracle.align(a, b, sm, go, ge)


@pytest.mark.parametrize("seed", range(6))
def test_tie_heavy_alignments(seed):
    """Two-letter sequences with free gaps: many optimal alignments; the rules
    pick one."""
    rng = np.random.default_rng(100 + seed)
    a = rng.integers(0, 2, int(rng.integers(50, 300))).astype(np.uint8)
    b = rng.integers(0, 2, int(rng.integers(50, 300))).astype(np.uint8)
    sm = synth.dna_matrix(1, -1)
    go, ge = int(rng.integers(0, 2)), int(rng.integers(0, 2))
    announce(f"align ties seed={seed}")
    assert _gpu_align(a, b, sm, go, ge) == oracle.align(a, b, sm, go, ge)


@pytest.mark.parametrize("wc", [16, 64, 512])
def test_chunk_widths(wc):
    a, b = synth.dna_pair(1500, 1700, seed=9, identity=0.7, indel_rate=0.03)
    sm, go, ge = DNA
    announce(f"align cols={wc}")
    assert _gpu_align(a, b, sm, go, ge, pair_cols=wc) == oracle.align(a, b, sm, go, ge)


def test_empty_and_zero():
    sm, go, ge = DNA
    a = np.zeros(40, np.uint8)
    b = np.full(30, 1, np.uint8)                     # all mismatches: score 0
    empty = {"score": 0, "q_begin": 0, "s_begin": 0, "q_end": 0, "s_end": 0, "ops": ""}
    announce("align empty")
    assert _gpu_align(a, b, sm, go, ge) == empty == oracle.align(a, b, sm, go, ge)
    assert _gpu_align(a[:0], b, sm, go, ge) == empty


def test_large_self_alignment():
    """A 50,000-base sequence against itself: the whole diagonal (closed form),
    2.5e9 cells of direction codes and a 50,000-step walk."""
    sm, go, ge = DNA
    rng = np.random.default_rng(5)
    a = synth.residues(rng, 50_000, synth.DNA_FREQS)
    announce("align 50k self")
    r = _gpu_align(a, a, sm, go, ge)
    assert r == {"score": 50_000, "q_begin": 1, "s_begin": 1, "q_end": 50_000, "s_end": 50_000, "ops": "M" * 50_000}


def test_alignment_beyond_2_32_cells():
    """1e10 cells (5 GB of direction codes, byte offsets past 2^32): a
    100,000-base sequence against its suffix from position 501 -- the whole
    suffix matches on one diagonal (closed form: begin 501 / 1, 99,500 pairs)."""
    sm, go, ge = DNA
    rng = np.random.default_rng(6)
    a = synth.residues(rng, 100_000, synth.DNA_FREQS)
    announce("align 100k vs suffix")
    r = _gpu_align(a, a[500:], sm, go, ge)
    assert r == {"score": 99_500, "q_begin": 501, "s_begin": 1, "q_end": 100_000, "s_end": 99_500,
                 "ops": "M" * 99_500}


# Blocked traceback: the score pass keeps checkpoint rows and columns, and the
# direction codes are recomputed one block at a time along the walk.  Small
# forced blocks put block edges (rows, columns, corners) across the paths;
# the result must equal the oracle's exactly, as with whole-matrix codes.
@pytest.mark.parametrize("block,wc", [(512, 0), (700, 64), (1024, 16), (1536, 512)])
@pytest.mark.parametrize("m,n", [(2000, 2000), (1300, 3100), (3100, 900)])
def test_blocked_dna_alignments(block, wc, m, n):
    a, b = synth.dna_pair(m, n, seed=m + 7 * n + block, identity=0.72, indel_rate=0.03)
    sm, go, ge = DNA
    announce(f"align blocked block={block} cols={wc} m={m} n={n}")
    assert _gpu_align(a, b, sm, go, ge, align_block=block, pair_cols=wc) == oracle.align(a, b, sm, go, ge)


@pytest.mark.parametrize("go,ge", [(10, 2), (0, 3), (120, 1)])
def test_blocked_protein_alignments(go, ge):
    rng = np.random.default_rng(3 * go + ge)
    sm = synth.blosum_style_matrix()
    a = synth.residues(rng, 1800)
    b = np.concatenate([synth.residues(rng, 300), synth.mutate(rng, a[200:1600], 0.55), synth.residues(rng, 200)])
    announce(f"align blocked protein go={go} ge={ge}")
    assert _gpu_align(a, b, sm, go, ge, align_block=512, pair_cols=64) == oracle.align(a, b, sm, go, ge)


@pytest.mark.parametrize("seed", range(4))
def test_blocked_tie_heavy(seed):
    rng = np.random.default_rng(200 + seed)
    a = rng.integers(0, 2, int(rng.integers(600, 1400))).astype(np.uint8)
    b = rng.integers(0, 2, int(rng.integers(600, 1400))).astype(np.uint8)
    sm = synth.dna_matrix(1, -1)
    go, ge = int(rng.integers(0, 2)), int(rng.integers(0, 2))
    announce(f"align blocked ties seed={seed}")
    assert _gpu_align(a, b, sm, go, ge, align_block=512, pair_cols=16) == oracle.align(a, b, sm, go, ge)


def test_blocked_empty_and_zero():
    sm, go, ge = DNA
    empty = {"score": 0, "q_begin": 0, "s_begin": 0, "q_end": 0, "s_end": 0, "ops": ""}
    a = np.zeros(700, np.uint8)
    b = np.full(900, 1, np.uint8)
    announce("align blocked empty")
    assert _gpu_align(a, b, sm, go, ge, align_block=512) == empty
    assert _gpu_align(a[:0], b, sm, go, ge, align_block=512) == empty


def test_blocked_large_suffix():
    """120,000 x 119,000 cells in 16,384-side blocks: the suffix matches on
    one diagonal across 8 x 8 blocks (closed form)."""
    sm, go, ge = DNA
    rng = np.random.default_rng(8)
    a = synth.residues(rng, 120_000, synth.DNA_FREQS)
    announce("align blocked 120k vs suffix")
    r = _gpu_align(a, a[1000:], sm, go, ge, align_block=16384)
    assert r == {"score": 119_000, "q_begin": 1001, "s_begin": 1, "q_end": 120_000, "s_end": 119_000,
                 "ops": "M" * 119_000}


@pytest.mark.parametrize("seed", range(24))
def test_random_alignments(seed):
    """Seeded sweep: sizes, signed matrices (symmetric or not), gap penalties,
    whole-matrix or blocked codes and chunk widths drawn together; the whole
    alignment must equal the oracle's."""
    rng = np.random.default_rng(500 + seed)
    m, n = int(rng.integers(1, 2600)), int(rng.integers(1, 2600))
    if seed % 3 == 0:
        sm = rng.integers(-128, 128, size=(32, 32)).astype(np.int32)
        a = rng.integers(0, 32, m).astype(np.uint8)
        b = rng.integers(0, 32, n).astype(np.uint8)
    elif seed % 3 == 1:
        sm, a = synth.blosum_style_matrix(), synth.residues(rng, m)
        lo = int(rng.integers(0, m))
        b = np.concatenate([synth.residues(rng, int(rng.integers(0, 400))),
                            synth.mutate(rng, a[lo:], float(rng.uniform(0.4, 0.95)))])[:max(n, 1)]
    else:
        sm = synth.dna_matrix(int(rng.integers(1, 6)), -int(rng.integers(1, 6)))
        a, b = synth.dna_pair(m, n, seed=seed, identity=float(rng.uniform(0.5, 0.95)), indel_rate=0.03)
    go, ge = int(rng.integers(0, 40)), int(rng.integers(0, 8))
    kw = dict(align_block=int(rng.choice([0, 512, 1100])), pair_cols=int(rng.choice([0, 16, 48, 256])))
    announce(f"align random seed={seed} m={len(a)} n={len(b)} go={go} ge={ge} {kw}")
    assert _gpu_align(a, b, sm, go, ge, **kw) == oracle.align(a, b, sm, go, ge)
