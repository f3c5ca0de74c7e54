"""Serving loop on the GPU: requests that overlap on the device in batches of
any composition return exactly what each query returns alone."""
import time

import numpy as np
import pytest

import oracle
import synth
from gpuhelp import announce, gpu_db, have_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]


def _workload(n=3000, nq=40, seed=21):
    rng = np.random.default_rng(seed)
    lens = synth.lognormal_lengths(rng, n, 300, 0.668, 10, 35_000)
    db = synth.make_db(rng, lens)
    qlens = synth.lognormal_lengths(rng, nq, 350, 0.75, 50, 5000)
    return db, [synth.residues(rng, int(m)) for m in qlens], rng


@pytest.mark.parametrize("mode", ["auto", "i32"])
def test_serve_results_equal_alone(mode):
    import torch
    from paper_2412_08308_amd.serve import GpuBackend, Server
    db, qs, rng = _workload()
    sm = synth.blosum_style_matrix()
    gdb = gpu_db(db)
    try:
        alone = []
        for q in qs:
            announce(f"alone m={len(q)} mode={mode}")
            alone.append(gdb.search(torch.from_numpy(q).cuda(), sm, 10, 2,
                                    opt=__import__("paper_2412_08308_amd").options(mode=mode)).cpu().numpy())
        torch.cuda.synchronize()
        be = GpuBackend(gdb, sm, 10, 2, mode=mode, n_streams=3)
        # burst queued before the scheduler starts: batches of up to 8 are certain
        announce("serving burst")
        srv = Server(be, max_batch=8)
        futs = [srv.submit(q) for q in qs]
        srv.start()
        got = [f.result(timeout=120) for f in futs]
        srv.stop()
        st = srv.stats()
        assert st["completed"] == len(qs) and st["max_batch"] == 8
        for k, (a, g) in enumerate(zip(alone, got)):
            assert np.array_equal(a, g), f"request {k} differs in a batch"
        # timed arrivals: batches form and overlap as the device allows
        announce("serving timed arrivals")
        with Server(be, max_batch=8) as srv:
            futs = []
            for q in qs:
                futs.append(srv.submit(q))
                time.sleep(float(rng.exponential(0.002)))
            got = [f.result(timeout=120) for f in futs]
        assert srv.stats()["completed"] == len(qs)
        for k, (a, g) in enumerate(zip(alone, got)):
            assert np.array_equal(a, g), f"request {k} differs in the mix"
        for k in (0, 7):
            assert np.array_equal(got[k], oracle.search_db(qs[k], db, sm, 10, 2))
    finally:
        gdb.release()


def test_serve_memory_budget_forces_waiting():
    from paper_2412_08308_amd.serve import GpuBackend, Server
    db, qs, rng = _workload(n=2000, nq=12, seed=22)
    sm = synth.blosum_style_matrix()
    gdb = gpu_db(db)
    try:
        be = GpuBackend(gdb, sm, 10, 2, n_streams=4)
        budget = be.need_bytes([max(len(q) for q in qs)] * 2)
        announce(f"serving with budget {budget}")
        with Server(be, max_batch=8, mem_budget=budget) as srv:
            futs = [srv.submit(q) for q in qs]
            got = [f.result(timeout=120) for f in futs]
        assert srv.stats()["max_bytes_in_use"] <= budget
        for q, g in zip(qs[:3], got[:3]):
            assert np.array_equal(g, oracle.search_db(q, db, sm, 10, 2))
    finally:
        gdb.release()


@pytest.mark.parametrize("mode", ["auto", "i32"])
def test_stepped_long_batches_equal_alone(mode):
    """Searches cut into many launches, the long requests' launches enqueued
    one at a time by the scheduler (slice_begin / slice_count) around short
    requests: every result equals the query searched alone, and the long
    batches really were stepped."""
    import torch
    import paper_2412_08308_amd as swdb
    from paper_2412_08308_amd.serve import GpuBackend, Server
    db, qs, rng = _workload(n=2500, nq=24, seed=23)
    sm = synth.blosum_style_matrix()
    gdb = gpu_db(db)
    try:
        alone = [gdb.search(torch.from_numpy(q).cuda(), sm, 10, 2, opt=swdb.options(mode=mode)).cpu().numpy()
                 for q in qs]
        be = GpuBackend(gdb, sm, 10, 2, mode=mode, n_streams=4, slice_mcells=20)
        calls = []
        adv = be.advance
        be.advance = lambda h: (calls.append(h["next"]), adv(h))
        cells = be.cells([int(np.median([len(q) for q in qs]))])
        # a nominal rate that makes the longer half of the requests long
        announce(f"stepped serving mode={mode}")
        with Server(be, max_batch=4, rate_guess=cells / 0.02, long_s=0.02, long_depth=2) as srv:
            futs = []
            for q in qs:
                futs.append(srv.submit(q))
                time.sleep(float(rng.exponential(0.001)))
            got = [f.result(timeout=120) for f in futs]
        assert srv.stats()["completed"] == len(qs) and srv.stats()["errors"] == 0
        assert len(calls) > 0 and max(calls) > 0, "no batch was enqueued launch by launch"
        for k, (a, g) in enumerate(zip(alone, got)):
            assert np.array_equal(a, g), f"request {k} (m={len(qs[k])}) differs when stepped"
        for k in (0, 5):
            assert np.array_equal(got[k], oracle.search_db(qs[k], db, sm, 10, 2))
    finally:
        gdb.release()
