"""Packed 16-bit lanes with exact int32 rescoring on the planted-overflow
workload: long subjects and near-homologs of an 8,000-residue query, whose
true scores exceed the 16-bit range (GPU required)."""
import numpy as np
import pytest

import synth
from gpuhelp import announce, gpu_db, gpu_scores, have_gpu, mismatch_report, oracle_scores

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]


def _flagged(gdb, q, sm, go, ge):
    import torch
    import paper_2412_08308_amd as swdb
    opt = swdb.options(mode="i16")
    ws = gdb.alloc_workspace([len(q)], opt)
    gdb.search(torch.from_numpy(q).cuda(), sm, go, ge, opt=opt, workspace=ws)
    torch.cuda.synchronize()
    return gdb.flagged_count(ws)


def test_planted_reduced_scale_every_subject():
    w = synth.planted(scale=0.02)
    q = w.queries[0]
    exp = oracle_scores(w.db, q, w.matrix, w.gap_open, w.gap_extend)
    assert int(np.sum(exp >= 32767)) > 0, "the workload must overflow 16 bits"
    gdb = gpu_db(w.db)
    try:
        for mode in ("i16", "auto", "i32"):
            announce(f"planted reduced mode={mode}")
            got = gpu_scores(gdb, q, w.matrix, w.gap_open, w.gap_extend, mode=mode)
            assert np.array_equal(got, exp), f"{mode}: " + mismatch_report(got, exp)
        assert _flagged(gdb, q, w.matrix, w.gap_open, w.gap_extend) == int(np.sum(exp >= 32767))
    finally:
        gdb.release()


def test_planted_full_scale_sampled():
    w = synth.workload("q8000_planted_vs_200k")
    q = w.queries[0]
    rng = np.random.default_rng(31)
    hom, lng = w.extra["hom_ids"], w.extra["long_ids"]
    ids = np.unique(np.concatenate([rng.choice(hom, 48, replace=False), rng.choice(lng, 12, replace=False),
                                    rng.choice(w.db.nseq, 100, replace=False)]))
    exp = oracle_scores(w.db, q, w.matrix, w.gap_open, w.gap_extend, ids=ids)
    assert np.sum(exp >= 32767) > 0
    gdb = gpu_db(w.db)
    try:
        for mode in ("auto", "i32"):
            announce(f"planted full mode={mode}")
            got = gpu_scores(gdb, q, w.matrix, w.gap_open, w.gap_extend, mode=mode)[ids]
            assert np.array_equal(got, exp), f"{mode}: " + mismatch_report(got, exp, ids)
        # the control query of the same database cannot overflow
        ctrl = w.extra["control_query"]
        assert _flagged(gdb, ctrl, w.matrix, w.gap_open, w.gap_extend) == 0
    finally:
        gdb.release()


def _pass_crossing_case(P: int, seed: int):
    """A query of P 64-lane rescore passes (1,536 rows each) and near-homologs
    of query windows that straddle pass boundaries (one window spans several
    when P >= 4), inside random flanks, plus random subjects."""
    rng = np.random.default_rng(seed)
    m = 1536 * P - 77
    q = synth.residues(rng, m)
    seqs = []
    for k in range(1, P):
        b = 1536 * k
        lo = max(0, b - int(rng.integers(200, 1200)))
        hi = min(m, b + int(rng.integers(200, 1200)))
        h = synth.mutate(rng, q[lo:hi], float(rng.uniform(0.7, 0.95)))
        seqs.append(np.concatenate([synth.residues(rng, int(rng.integers(0, 300))), h,
                                    synth.residues(rng, int(rng.integers(0, 300)))]))
    if P >= 4:
        seqs.append(synth.mutate(rng, q[1536 - 300:1536 * 3 + 300], 0.8))
    seqs += [synth.residues(rng, int(n)) for n in rng.integers(10, 600, size=40)]
    order = rng.permutation(len(seqs))
    return q, synth.Database.from_list([seqs[i] for i in order])


@pytest.mark.parametrize("P", [2, 5, 10])
@pytest.mark.parametrize("scale,go,ge,variant", [(8, 32, 6, 3), (11, 40, 8, 2)])
def test_rescore_passes_across_wavefronts(P, scale, go, ge, variant):
    # The rescore splits a subject's query rows into 64-lane passes over the
    # wavefronts of a workgroup (at most 8, so P = 10 reuses boundary
    # buffers); homologs whose best alignment crosses pass boundaries catch a
    # wrong hand-over.  Scaled matrices push their scores past 32,767.
    import paper_2412_08308_amd as swdb
    sm = synth.blosum_style_matrix() * scale
    assert swdb.select_variant(sm, go) == variant
    q, db = _pass_crossing_case(P, seed=100 + P)
    exp = oracle_scores(db, q, sm, go, ge)
    n_over = int(np.sum(exp >= 32767))
    assert n_over >= P - 1
    gdb = gpu_db(db)
    try:
        for mode in ("i16", "auto", "i32"):
            announce(f"rescore passes P={P} m={len(q)} scale={scale} mode={mode}")
            got = gpu_scores(gdb, q, sm, go, ge, mode=mode)
            assert np.array_equal(got, exp), f"{mode}: " + mismatch_report(got, exp)
        assert _flagged(gdb, q, sm, go, ge) == n_over
    finally:
        gdb.release()
