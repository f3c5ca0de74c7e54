"""Autotuner and tuned-mode searches (GPU required): whatever schedule the
tuner picks, scores stay exact; the cache reproduces the table."""
import numpy as np
import pytest

import synth
from gpuhelp import announce, gpu_batch, gpu_db, have_gpu, oracle_scores

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]


def test_autotune_then_tuned_batch(tmp_path):
    import paper_2412_08308_amd as swdb
    from paper_2412_08308_amd import autotune
    rng = np.random.default_rng(51)
    sm = synth.blosum_style_matrix()
    db = synth.make_db(rng, synth.lognormal_lengths(rng, 2500, 300, 0.668, 10, 35_000))
    gdb = gpu_db(db)
    try:
        announce("autotune bins 100, 700")
        cache = str(tmp_path / "tune.json")
        t1 = autotune.tuned(gdb, [100, 700], sm, 10, 2, cache_path=cache)
        assert [e["qlen"] for e in t1] == [100, 700]
        assert all(e["mode"] in (swdb.MODE_AUTO, swdb.MODE_I16, swdb.MODE_I32) and e["gcups"] > 0 for e in t1)
        gdb.set_tuning([])
        # second call: same table from the cache, no measurement
        gdb.autotune = None
        t2 = autotune.tuned(gdb, [100, 700], sm, 10, 2, cache_path=cache)
        assert t2 == t1 and gdb.get_tuning() == t1
        del gdb.autotune
        qs = [synth.residues(rng, m) for m in (50, 300, 700, 1500)]
        announce("tuned batch")
        got = gpu_batch(gdb, qs, sm, 10, 2, mode="tuned")
        for k, q in enumerate(qs):
            assert np.array_equal(got[k], oracle_scores(db, q, sm, 10, 2)), f"query {k}"
    finally:
        gdb.release()


def test_autotune_batch_as_a_unit():
    """sw_autotune_batch times schedules on the batch itself and returns one;
    the batch searched with it (and with the strict lane-group rule it may
    pick) equals the oracle, and nothing is installed on the handle."""
    import torch
    import paper_2412_08308_amd as swdb
    rng = np.random.default_rng(52)
    sm = synth.blosum_style_matrix()
    db = synth.make_db(rng, synth.lognormal_lengths(rng, 3000, 300, 0.668, 10, 20_000))
    gdb = gpu_db(db)
    try:
        qs = [synth.residues(rng, m) for m in (40, 300, 900, 2200, 64)]
        qts = [torch.from_numpy(q).cuda() for q in qs]
        announce("autotune batch of 5")
        opt, rec = gdb.autotune_batch(qts, sm, 10, 2)
        assert rec["gcups"] > 0 and rec["qlen"] == 2200 and gdb.get_tuning() == []
        exp = [oracle_scores(db, q, sm, 10, 2) for q in qs]
        for o in (opt, swdb.options(strict_groups=1), swdb.options(mode="i32", strict_groups=1)):
            announce(f"batch with mode={o.mode} waves={o.waves} lane_cells={o.lane_cells} strict={o.strict_groups}")
            got = gdb.search_batch(qts, sm, 10, 2, opt=o).cpu().numpy()
            for k in range(len(qs)):
                assert np.array_equal(got[k], exp[k]), f"query {k}"
    finally:
        gdb.release()
