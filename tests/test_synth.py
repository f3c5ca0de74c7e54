"""The seeded input generator: determinism and the stated distributions."""
import numpy as np

import synth


def test_deterministic():
    a = synth.workload("q64_vs_2k")
    b = synth.workload("q64_vs_2k")
    assert np.array_equal(a.db.residues, b.db.residues)
    assert np.array_equal(a.queries[0], b.queries[0])
    c = synth.workload("q64_vs_2k", seed=1)
    assert not np.array_equal(a.db.residues, c.db.residues)


def test_q64_vs_2k_shape():
    w = synth.workload("q64_vs_2k")
    assert len(w.queries) == 1 and len(w.queries[0]) == 64
    assert w.db.nseq == 2000
    assert w.db.lengths.min() >= 32 and w.db.lengths.max() <= 512
    assert w.gap_open == 10 and w.gap_extend == 2
    assert w.db.residues.max() < 20


def test_lognormal_law():
    w = synth.workload("q567_vs_200k", scale=0.1)
    L = w.db.lengths
    assert L.min() >= 10 and L.max() <= 35000
    assert abs(np.median(L) - 300) < 10
    assert 355 < L.mean() < 395


def test_residue_frequencies():
    rng = np.random.default_rng(0)
    x = synth.residues(rng, 400_000)
    obs = np.bincount(x, minlength=20) / len(x)
    chi2 = len(x) * np.sum((obs - synth.BACKGROUND) ** 2 / synth.BACKGROUND)
    assert chi2 < 60          # 19 dof; p ~ 1e-5 threshold


def test_matrix_properties():
    sm = synth.blosum_style_matrix()
    assert sm.shape == (32, 32) and sm.dtype == np.int32
    core = sm[:20, :20]
    assert np.array_equal(core, core.T)
    d = np.diag(core)
    assert d.min() >= 4 and d.max() <= 11
    off = core[~np.eye(20, dtype=bool)]
    assert off.min() >= -4 and off.max() <= 3
    assert synth.BACKGROUND @ core @ synth.BACKGROUND < 0
    assert np.all(sm[20:, :] == synth.PAD_SCORE)


def test_query_lengths_c3():
    L = synth.c3_query_lengths()
    assert len(L) == 20 and L[0] == 144 and L[-1] == 5478
    assert all(b > a for a, b in zip(L, L[1:]))


def test_mutate_identity():
    rng = np.random.default_rng(1)
    src = synth.residues(rng, 5000)
    h = synth.mutate(rng, src, 0.9, indel_rate=0.0)
    assert len(h) == len(src)
    ident = np.mean(h == src)
    assert 0.88 < ident < 0.95   # kept 90% + chance matches among substitutions


def test_planted_small():
    w = synth.planted(scale=0.01, qlen=800)
    assert len(w.queries) == 1 and len(w.queries[0]) == 800
    assert w.db.lengths.max() >= 10_000
    assert len(w.extra["hom_ids"]) == 20


def test_ncbi_loader():
    text = "   A  R\nA  4 -1\nR -1  5\n"
    m = synth.load_ncbi_matrix(text, alphabet="AR")
    assert m[0, 0] == 4 and m[0, 1] == -1 and m[1, 1] == 5 and m[5, 5] == synth.PAD_SCORE
