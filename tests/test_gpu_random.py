"""Seeded random sweep of the search against the oracle (GPU required):
database shapes, query sets, substitution matrices (symmetric or not, in the
full signed 8-bit range, or scaled so that 16-bit lanes overflow), gap
penalties, modes and planner options drawn together, so that combinations no
single-knob test reaches are exercised (self-paired items with overflow flags,
batches mixing LDS and global profiles, lane groups with ragged subjects).
Every score must equal the oracle's."""
import numpy as np
import pytest

import oracle
import synth
from gpuhelp import announce, gpu_db, have_gpu, mismatch_report

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

CELL_BUDGET = 60_000_000          # oracle cells per case


def _case(seed):
    rng = np.random.default_rng(1000 + seed)
    kind = seed % 4
    if kind == 0:                                   # random signed matrix
        sm = rng.integers(-128, 128, size=(32, 32)).astype(np.int32)
        if rng.random() < 0.5:
            sm = np.triu(sm) + np.triu(sm, 1).T
    elif kind == 1:                                 # BLOSUM-style
        sm = synth.blosum_style_matrix()
    else:                                           # scaled: scores past 32,767 on homologs
        sm = synth.blosum_style_matrix() * int(rng.choice([6, 8, 11]))
    go = int(rng.integers(0, 60))
    ge = int(rng.integers(0, 12))
    nq = int(rng.integers(1, 5))
    qlens = [int(x) for x in rng.choice([0, 1, 17, 200, 567, 1537, 2100, 3100, 4000], size=nq)]
    qs = [synth.residues(rng, m) for m in qlens]
    budget = CELL_BUDGET // max(1, sum(qlens))
    seqs, total = [], 0
    while total < budget and len(seqs) < 400:
        r = rng.random()
        if r < 0.15 and qlens[0] > 50:              # homolog of a query window
            q = qs[int(rng.integers(0, nq))]
            if len(q) > 50:
                lo = int(rng.integers(0, len(q) - 40))
                s = synth.mutate(rng, q[lo:lo + int(rng.integers(40, len(q) - lo + 1))], float(rng.uniform(0.6, 0.98)))
            else:
                s = synth.residues(rng, 30)
        elif r < 0.25:
            s = synth.residues(rng, int(rng.choice([0, 1, 15, 16, 17, 63, 64, 65, 127, 128, 129])))
        else:
            s = synth.residues(rng, int(min(rng.lognormal(np.log(300), 0.8), 6000)))
        seqs.append(s)
        total += len(s)
    db = synth.Database.from_list(seqs)
    mode = str(rng.choice(["auto", "i16", "i32"]))
    kw = {}
    if rng.random() < 0.5:
        kw = dict(waves=int(rng.choice([0, 1, 2, 4, 8])), lane_cells=int(rng.choice([0, 4096, 20000, 96000])),
                  max_lanes=int(rng.choice([0, 1, 3, 16, 64])), lds_limit=int(rng.choice([0, 8192, 131072])),
                  wide_profile=int(rng.integers(0, 2)))
    return qs, db, sm, go, ge, mode, kw


@pytest.mark.parametrize("seed", range(40))
def test_random_search_cases(seed):
    import torch
    import paper_2412_08308_amd as swdb
    qs, db, sm, go, ge, mode, kw = _case(seed)
    exp = np.stack([oracle.search_db(q, db, sm, go, ge) for q in qs])
    announce(f"random seed={seed} nq={len(qs)} m={[len(q) for q in qs]} nseq={db.nseq} "
             f"go={go} ge={ge} mode={mode} {kw} max={int(exp.max())}")
    gdb = gpu_db(db)
    try:
        opt = swdb.options(mode=mode, **kw)
        qts = [torch.from_numpy(np.ascontiguousarray(q)).cuda() for q in qs]
        got = gdb.search_batch(qts, sm, go, ge, opt=opt)
        torch.cuda.synchronize()
        got = got.cpu().numpy().astype(np.int64)
        for k in range(len(qs)):
            assert np.array_equal(got[k], exp[k]), f"query {k}: " + mismatch_report(got[k], exp[k])
        if len(qs) == 1 or seed % 3 == 0:
            one = gdb.search(qts[0], sm, go, ge, opt=opt)
            torch.cuda.synchronize()
            assert np.array_equal(one.cpu().numpy().astype(np.int64), exp[0])
    finally:
        gdb.release()
