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
