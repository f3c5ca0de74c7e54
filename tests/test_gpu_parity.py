"""Bit-exact parity of the HIP path against the CPU oracle (GPU required).

Scores are integers, so the bar is equality.  Inputs are seeded and synthetic;
shapes cover several work items, ragged tails of every tiling (16-column
blocks, 64-subject chunks, R-row blocks, K-lane passes) and the degenerate
cases of the recurrence.
"""
import numpy as np
import pytest

import synth
from gpuhelp import (announce, gpu_batch, gpu_db, gpu_scores, have_gpu, mismatch_report,
                     oracle_scores, overflow_matrix, overflow_sequence)

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

# "w": the same lanes with 16-bit profile entries (the default takes 8-bit
# entries whenever every s + Go fits)
MODES = ["i32", "i32w", "i16", "i16w", "auto"]


def _check(db, q, sm, go, ge, modes=MODES, ids=None, **kw):
    exp = oracle_scores(db, q, sm, go, ge, ids=ids)
    gdb = gpu_db(db)
    try:
        for mode in modes:
            announce(f"mode={mode} m={len(q)} nseq={db.nseq} go={go} ge={ge} {kw}")
            got = gpu_scores(gdb, q, sm, go, ge, mode=mode, **kw)
            if ids is not None:
                got = got[np.asarray(ids)]
            assert np.array_equal(got, exp), f"{mode}: " + mismatch_report(got, exp, ids)
    finally:
        gdb.release()


def test_q64_vs_2k_all_modes():
    w = synth.workload("q64_vs_2k")
    _check(w.db, w.queries[0], w.matrix, w.gap_open, w.gap_extend)


def test_one_shot_entry_point():
    import torch
    import paper_2412_08308_amd as swdb
    w = synth.workload("q64_vs_2k", scale=0.1)
    exp = oracle_scores(w.db, w.queries[0], w.matrix, 10, 2)
    announce("sw_db_search one-shot")
    res = torch.from_numpy(w.db.residues).cuda()
    off = torch.from_numpy(w.db.offsets).cuda()
    ln = torch.from_numpy(w.db.lengths).cuda()
    q = torch.from_numpy(w.queries[0]).cuda()
    got = swdb.search(q, res, off, ln, w.matrix, 10, 2).cpu().numpy()
    assert np.array_equal(got, exp), mismatch_report(got, exp)


@pytest.mark.parametrize("m", [0, 1, 15, 16, 17, 31, 32, 33, 47, 64, 65, 100, 257])
def test_query_lengths(m):
    rng = np.random.default_rng(1000 + m)
    lens = [0, 1, 2, 15, 16, 17, 31, 32, 33, 63, 64, 65, 127, 128, 129, 300, 511, 700]
    lens = lens * 5 + rng.integers(0, 400, size=110).tolist()
    q, db = synth.random_case(rng, m, lens)
    _check(db, q, synth.blosum_style_matrix(), 10, 2)


@pytest.mark.parametrize("nseq", [1, 2, 63, 64, 65, 127, 128, 129, 257])
def test_chunk_edges(nseq):
    rng = np.random.default_rng(2000 + nseq)
    q, db = synth.random_case(rng, 90, rng.integers(1, 200, size=nseq).tolist())
    _check(db, q, synth.blosum_style_matrix(), 10, 2)


def test_asymmetric_random_matrix():
    rng = np.random.default_rng(7)
    sm = synth.random_matrix(rng, -5, 5)
    q, db = synth.random_case(rng, 150, rng.integers(0, 300, size=400).tolist(), alpha=32)
    _check(db, q, sm, 7, 3)


@pytest.mark.parametrize("go,ge", [(3, 5), (4, 4), (10, 0), (0, 0), (0, 3), (32000, 32000), (200, 50)])
def test_gap_penalty_regimes(go, ge):
    rng = np.random.default_rng(go * 131 + ge)
    q, db = synth.random_case(rng, 120, rng.integers(0, 260, size=300).tolist())
    _check(db, q, synth.blosum_style_matrix(), go, ge)


def test_extreme_matrix_values():
    rng = np.random.default_rng(8)
    sm = synth.random_matrix(rng, -128, 127)
    q, db = synth.random_case(rng, 70, rng.integers(0, 150, size=200).tolist(), alpha=32)
    _check(db, q, sm, 20, 3)


def test_long_subjects_and_lane_groups():
    # a few long subjects force multi-lane groups (K up to 64) and many passes
    rng = np.random.default_rng(9)
    lens = [35000, 12000, 5000, 4097, 2049, 1000] + rng.integers(10, 400, size=300).tolist()
    q, db = synth.random_case(rng, 567, lens)
    _check(db, q, synth.blosum_style_matrix(), 10, 2)


@pytest.mark.parametrize("kw", [dict(max_lanes=1), dict(max_lanes=2), dict(max_lanes=8),
                                dict(lane_cells=2000), dict(lane_cells=1 << 24),
                                dict(waves=1), dict(waves=3), dict(waves=8), dict(lds_limit=1024),
                                dict(grid_limit=1)])
def test_plan_knobs_do_not_change_scores(kw):
    rng = np.random.default_rng(10)
    lens = [3000, 1500, 800] + rng.integers(10, 600, size=500).tolist()
    q, db = synth.random_case(rng, 333, lens)
    _check(db, q, synth.blosum_style_matrix(), 10, 2, **kw)


def test_long_query_global_profile():
    # profile larger than the LDS budget: read from global memory
    rng = np.random.default_rng(11)
    q, db = synth.random_case(rng, 3000, rng.integers(10, 500, size=200).tolist())
    _check(db, q, synth.blosum_style_matrix(), 10, 2)


@pytest.mark.parametrize("m,lds", [(1537, 0), (1537, 131072), (3073, 0), (6200, 0)])
def test_self_paired_items(m, lds):
    # Packed lanes with both halves on one subject's rows (the longest items
    # of long queries): 1537 rows = 65 row blocks, one pass whose high halves
    # hold a single block (LDS or global profile); 3073 = 129 blocks, two
    # passes; 6200 = 259 blocks, three passes.  Homologs of query windows
    # across the half boundary (row 1536) and the pass boundary (row 3072),
    # ragged subject lengths around the 16-column blocks and the 128-column
    # pipeline depth.
    import paper_2412_08308_amd as swdb
    rng = np.random.default_rng(m + lds)
    q = synth.residues(rng, m)
    seqs = [synth.residues(rng, n) for n in (1, 5, 15, 16, 17, 63, 64, 65, 127, 128, 129, 500, 2000, 9000)]
    for lo, hi in ((1300, 1800), (2900, 3300), (100, 6000)):
        if hi <= m:
            seqs.append(synth.mutate(rng, q[lo:hi], 0.8))
    seqs += [synth.residues(rng, int(n)) for n in rng.integers(10, 700, size=120)]
    db = synth.Database.from_list([seqs[i] for i in rng.permutation(len(seqs))])
    plan = swdb.Database.describe(db.lengths)
    try:
        for mode, spl in (("auto", 2), ("i32", 1)):
            items = plan.plan_items([m], swdb.options(mode=mode, lds_limit=lds))
            n_self = int(np.sum((items[:, 3] >> 25) & 1))
            assert (n_self > 0) == (spl == 2), (mode, n_self)
    finally:
        plan.release()
    _check(db, q, synth.blosum_style_matrix(), 10, 2, modes=["i16", "i16w", "auto"], lds_limit=lds)


@pytest.mark.parametrize("top,low", [(127, -128), (117, -10)])
def test_int16_overflow_boundary(top, low):
    # (127, -128): 16-bit profile entries; (117, -10) with Go = 10: every
    # s + Go in [0, 127], so the packed lanes take 8-bit entries
    import paper_2412_08308_amd as swdb
    sm = overflow_matrix(top, low)
    assert swdb.select_variant(sm, 10) == (3 if low == -10 else 2)
    seqs, targets = [], [32766, 32767, 32768, 40000, 32000, 1000]
    for t in targets:
        seqs.append(overflow_sequence(t, top))
    rng = np.random.default_rng(12)
    # the query holds every constructed subject as a substring (a run of code 0
    # followed by a run of code 1), so each subject scores its diagonal sum
    q = np.concatenate([np.zeros(400, np.uint8), np.ones(300, np.uint8),
                        rng.integers(2, 20, size=50).astype(np.uint8)])
    subj = seqs + [rng.integers(0, 20, size=int(n)).astype(np.uint8)
                   for n in rng.integers(10, 300, size=150)]
    db = synth.Database.from_list(subj)
    exp = oracle_scores(db, q, sm, 10, 2)
    assert list(exp[:6]) == targets
    _check(db, q, sm, 10, 2)
    # the 16-bit pass flags exactly the subjects whose true score is >= 32767
    import torch
    gdb = gpu_db(db)
    try:
        opt = swdb.options(mode="i16")
        ws = gdb.alloc_workspace([len(q)], opt)
        announce("int16 flag count")
        gdb.search(torch.from_numpy(q).cuda(), sm, 10, 2, opt=opt, workspace=ws)
        torch.cuda.synchronize()
        assert gdb.flagged_count(ws) == int(np.sum(exp >= 32767))
    finally:
        gdb.release()


def test_batch_rows_equal_single_queries():
    rng = np.random.default_rng(13)
    sm = synth.blosum_style_matrix()
    _, db = synth.random_case(rng, 1, rng.integers(0, 700, size=700).tolist())
    qs = [synth.residues(rng, int(m)) for m in [144, 0, 17, 600, 1, 2500, 333]]
    gdb = gpu_db(db)
    try:
        for mode in MODES:
            announce(f"batch mode={mode}")
            got = gpu_batch(gdb, qs, sm, 10, 2, mode=mode)
            for k, q in enumerate(qs):
                exp = oracle_scores(db, q, sm, 10, 2)
                assert np.array_equal(got[k], exp), f"{mode} query {k}: " + mismatch_report(got[k], exp)
            # order of queries in the batch does not matter
            perm = [6, 3, 0, 5, 1, 4, 2]
            got2 = gpu_batch(gdb, [qs[i] for i in perm], sm, 10, 2, mode=mode)
            assert np.array_equal(got2, got[perm])
    finally:
        gdb.release()


def test_bad_residue_rejected():
    import paper_2412_08308_amd as swdb
    db = synth.Database.from_list([np.array([1, 2, 40, 3], dtype=np.uint8)])
    announce("bad residue code")
    with pytest.raises(swdb.SwdbError) as ei:
        gpu_db(db)
    assert ei.value.code == -5


def test_q567_vs_200k_sampled():
    """Full 200,000-subject database in the benchmark's launch configuration;
    every subject of three length strata checked by the oracle one by one."""
    w = synth.workload("q567_vs_200k")
    order = np.argsort(-w.db.lengths, kind="stable")
    rng = np.random.default_rng(14)
    ids = np.unique(np.concatenate([order[:200], order[-100:],
                                    rng.choice(w.db.nseq, size=700, replace=False)]))
    _check(w.db, w.queries[0], w.matrix, w.gap_open, w.gap_extend, modes=["i32", "auto"], ids=ids)


@pytest.mark.parametrize("mode", ["auto", "i32", "tuned"])
def test_sliced_launches(mode):
    """A search cut into many persistent launches (slice_mcells) equals the
    oracle: single queries, a batch, a tuned table with several launch groups,
    and 16-bit overflows rescored per launch."""
    import paper_2412_08308_amd as swdb
    rng = np.random.default_rng(19)
    sm = synth.blosum_style_matrix()
    lens = rng.integers(0, 900, size=1200).tolist() + [0, 1, 6000, 12000]
    _, db = synth.random_case(rng, 1, lens)
    qs = [synth.residues(rng, int(m)) for m in [300, 0, 17, 1500, 4000, 64]]
    gdb = gpu_db(db)
    try:
        if mode == "tuned":
            gdb.set_tuning([{"qlen": 100, "mode": 2, "waves": 8, "lane_cells": 24576},
                            {"qlen": 2000, "mode": 1, "waves": 4, "lane_cells": 49152},
                            {"qlen": 9000, "mode": 2, "waves": 4, "lane_cells": 98304}])
        for mc in (1, 40):
            announce(f"sliced batch mode={mode} slice_mcells={mc}")
            got = gpu_batch(gdb, qs, sm, 10, 2, mode=mode, slice_mcells=mc)
            for k, q in enumerate(qs):
                exp = oracle_scores(db, q, sm, 10, 2)
                assert np.array_equal(got[k], exp), f"{mode} {mc} query {k}: " + mismatch_report(got[k], exp)
            assert gdb.plan_info([len(q) for q in qs], swdb.options(mode=mode, slice_mcells=mc))["launches"] > 1
    finally:
        gdb.release()
    # overflows rescored inside sliced launches
    sm2 = overflow_matrix(127, -10)
    subj = [overflow_sequence(t, 127) for t in (32766, 32767, 40000)] * 3
    subj += [rng.integers(2, 20, size=int(n)).astype(np.uint8) for n in rng.integers(10, 300, size=200)]
    db2 = synth.Database.from_list(subj)
    q2 = np.concatenate([np.zeros(400, np.uint8), np.ones(300, np.uint8)])
    if mode != "tuned":
        announce(f"sliced overflow mode={mode}")
        gdb2 = gpu_db(db2)
        try:
            got = gpu_scores(gdb2, q2, sm2, 10, 2, mode=mode, slice_mcells=1)
            exp = oracle_scores(db2, q2, sm2, 10, 2)
            assert np.array_equal(got, exp), mismatch_report(got, exp)
        finally:
            gdb2.release()


@pytest.mark.parametrize("mode", ["auto", "i32", "tuned"])
def test_sliced_search_launch_by_launch(mode):
    """A sliced search enqueued one launch per call (slice_begin, slice_count
    = 1) on one workspace equals the oracle, and its status words add up over
    the calls as in one call (the flagged count of planted 16-bit overflows)."""
    import torch
    import paper_2412_08308_amd as swdb
    rng = np.random.default_rng(23)
    sm = synth.blosum_style_matrix()
    lens = rng.integers(0, 900, size=900).tolist() + [0, 3, 5000]
    _, db = synth.random_case(rng, 1, lens)
    qs = [synth.residues(rng, int(m)) for m in [700, 0, 33, 2500]]
    gdb = gpu_db(db)
    try:
        if mode == "tuned":
            gdb.set_tuning([{"qlen": 100, "mode": 2, "waves": 8, "lane_cells": 24576},
                            {"qlen": 9000, "mode": 1, "waves": 4, "lane_cells": 49152}])
        lens_q = [len(q) for q in qs]
        kw = dict(mode=mode, slice_mcells=2)
        n = gdb.plan_info(lens_q, swdb.options(**kw))["launches"]
        assert n > 3
        qts = [torch.from_numpy(q).cuda() for q in qs]
        cat = torch.cat(qts)
        offs = np.concatenate([[0], np.cumsum(lens_q[:-1])]).astype(np.int64)
        ws = gdb.alloc_workspace(lens_q, swdb.options(**kw))
        out = torch.full((len(qs), db.nseq), -7, dtype=torch.int32, device="cuda")
        announce(f"launch-by-launch search mode={mode}: {n} launches")
        for k in range(n):
            gdb.search_batch((cat, offs, lens_q), sm, 10, 2, opt=swdb.options(**kw, slice_begin=k, slice_count=1),
                             out=out, workspace=ws, check=False)
        gdb.status(ws, raise_on_error=True)
        got = out.cpu().numpy().astype(np.int64)
        for k, q in enumerate(qs):
            exp = oracle_scores(db, q, sm, 10, 2)
            assert np.array_equal(got[k], exp), f"{mode} query {k}: " + mismatch_report(got[k], exp)
        with pytest.raises(swdb.SwdbError):
            gdb.search_batch((cat, offs, lens_q), sm, 10, 2, opt=swdb.options(**kw, slice_begin=n), out=out,
                             workspace=ws, check=False)
    finally:
        gdb.release()
    if mode == "tuned":
        return
    sm2 = overflow_matrix(127, -10)
    subj = [overflow_sequence(t, 127) for t in (32766, 32767, 40000)] * 4
    subj += [rng.integers(2, 20, size=int(x)).astype(np.uint8) for x in rng.integers(10, 300, size=300)]
    db2 = synth.Database.from_list(subj)
    q2 = np.concatenate([np.zeros(400, np.uint8), np.ones(300, np.uint8)])
    gdb2 = gpu_db(db2)
    try:
        kw = dict(mode=mode, slice_mcells=1)
        n = gdb2.plan_info([len(q2)], swdb.options(**kw))["launches"]
        assert n > 2
        ws = gdb2.alloc_workspace([len(q2)], swdb.options(**kw))
        out = torch.full((1, db2.nseq), -7, dtype=torch.int32, device="cuda")
        qt = torch.from_numpy(q2).cuda()
        announce(f"launch-by-launch overflow mode={mode}: {n} launches")
        for k in range(n):
            gdb2.search_batch([qt], sm2, 10, 2, opt=swdb.options(**kw, slice_begin=k, slice_count=1), out=out,
                              workspace=ws, check=False)
        st = gdb2.status(ws, raise_on_error=True)
        got = out.cpu().numpy()[0].astype(np.int64)
        exp = oracle_scores(db2, q2, sm2, 10, 2)
        assert np.array_equal(got, exp), mismatch_report(got, exp)
        if mode == "auto":
            assert st["flagged"] == int(np.sum(exp >= 32767)) > 0
    finally:
        gdb2.release()
