"""sw_pair_score_static (the pair score on the library's static device
scratch, for callers that cannot allocate) against sw_pair_score with a
caller workspace and against the oracle: two calls in a row, the second with
a smaller pair, so the second runs on scratch the first left behind (GPU
required)."""
import numpy as np
import pytest

import synth
from gpuhelp import announce, have_gpu, oracle_pair

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]


def _both(a, b, sm, go, ge, opt=None):
    import torch
    import paper_2412_08308_amd as swdb
    qa, qb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    announce(f"pair_score_static {len(a)} x {len(b)}")
    got_static = int(swdb.pair_score_static(qa, qb, sm, go, ge, opt=opt).cpu().item())
    announce(f"pair_score (workspace) {len(a)} x {len(b)}")
    got_ws = int(swdb.pair_score(qa, qb, sm, go, ge, opt=opt).cpu().item())
    return got_static, got_ws


def test_static_pair_equals_workspace_pair_dna():
    sm = synth.dna_matrix(synth.DNA_MATCH, synth.DNA_MISMATCH)
    go, ge = synth.DNA_GAP_OPEN, synth.DNA_GAP_EXTEND
    for (m, n, seed) in [(4000, 5200, 3), (900, 700, 4)]:        # the second smaller
        a, b = synth.dna_pair(m, n, seed=seed)
        s_static, s_ws = _both(a, b, sm, go, ge)
        exp = oracle_pair(a, b, sm, go, ge)
        assert s_static == s_ws == exp, f"{m}x{n}: static {s_static} workspace {s_ws} oracle {exp}"


def test_static_pair_equals_workspace_pair_protein_and_tilings():
    import paper_2412_08308_amd as swdb
    rng = np.random.default_rng(71)
    sm = synth.blosum_style_matrix()
    q = synth.residues(rng, 1500)
    d = np.concatenate([synth.mutate(rng, q[200:1300], 0.6), synth.residues(rng, 400)])
    exp = oracle_pair(q, d, sm, 10, 2)
    for opt in (swdb.options(pair_rows=8, pair_cols=64), swdb.options(pair_rows=16, pair_cols=256, max_lanes=16)):
        s_static, s_ws = _both(q, d, sm, 10, 2, opt)
        assert s_static == s_ws == exp
    q2, d2 = q[:300], d[:250]                                     # then a smaller pair
    s_static, s_ws = _both(q2, d2, sm, 10, 2)
    assert s_static == s_ws == oracle_pair(q2, d2, sm, 10, 2)


def test_static_pair_too_large_rejected():
    """A pair needing more scratch than the static array is refused with
    SW_ENOMEM and nothing is launched; empty pairs score 0."""
    import torch
    import paper_2412_08308_amd as swdb
    m, n = 420_000, 420_000
    assert swdb.pair_workspace_bytes(m, n) > swdb.STATIC_SCRATCH_BYTES
    qa = torch.zeros(m, dtype=torch.uint8, device="cuda")
    qb = torch.zeros(n, dtype=torch.uint8, device="cuda")
    sm = synth.dna_matrix(1, -3)
    announce("pair_score_static too large")
    with pytest.raises(swdb.SwdbError) as ei:
        swdb.pair_score_static(qa, qb, sm, 5, 2)
    assert ei.value.code == -2
    announce("pair_score_static empty")
    e = torch.empty(0, dtype=torch.uint8, device="cuda")
    assert int(swdb.pair_score_static(e, qb[:10], sm, 5, 2).cpu().item()) == 0
