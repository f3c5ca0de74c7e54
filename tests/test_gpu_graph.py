"""Captured batched search (HIP graph): every replay equals the eager search,
with eager work and synchronisations between replays (GPU required)."""
import numpy as np
import pytest

import synth
from gpuhelp import announce, gpu_batch, gpu_db, have_gpu, oracle_scores

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]


@pytest.mark.parametrize("mode", ["auto", "i32"])
def test_graph_replays_equal_eager(mode):
    import torch
    import paper_2412_08308_amd as swdb
    rng = np.random.default_rng(41)
    sm = synth.blosum_style_matrix()
    lens = synth.lognormal_lengths(rng, 1500, 300, 0.668, 10, 35_000)
    db = synth.make_db(rng, lens)
    qlens = [144, 567, 1200, 60]
    qs = [synth.residues(rng, m) for m in qlens]
    gdb = gpu_db(db)
    try:
        opt = swdb.options(mode=mode)
        eager = gpu_batch(gdb, qs, sm, 10, 2, mode=mode)
        cat = torch.from_numpy(np.concatenate(qs)).cuda()
        offs = np.concatenate([[0], np.cumsum(qlens[:-1])])
        announce(f"graph capture mode={mode}")
        g = gdb.capture((cat, offs, qlens), sm, 10, 2, opt=opt)
        for rep in range(4):
            g.out.fill_(-1)
            announce(f"graph replay {rep}")
            g.launch()
            torch.cuda.synchronize()
            assert np.array_equal(g.out.cpu().numpy(), eager), f"replay {rep}"
            # unrelated eager work between replays
            gpu_batch(gdb, [qs[1]], sm, 10, 2, mode=mode)
        # new residues of the same lengths, written into the captured buffer
        qs2 = [synth.residues(rng, m) for m in qlens]
        g.queries.copy_(torch.from_numpy(np.concatenate(qs2)).cuda())
        g.launch()
        torch.cuda.synchronize()
        got = g.out.cpu().numpy()
        for k, q in enumerate(qs2):
            assert np.array_equal(got[k], oracle_scores(db, q, sm, 10, 2)), f"query {k} after rewrite"
        g.destroy()
    finally:
        gdb.release()
