"""The C-ABI's ownership and error contract on the GPU: the database layout in
a caller-owned (torch-allocated) buffer, its size bound, and errors found on
the device surfaced through the search status (GPU required)."""
import ctypes

import numpy as np
import pytest

import synth
from gpuhelp import announce, have_gpu, mismatch_report, oracle_scores

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]


def _case(seed=61, n=900):
    rng = np.random.default_rng(seed)
    lens = np.concatenate([[0, 1, 15, 16, 17, 2500], rng.integers(1, 700, size=n - 6)]).astype(np.int32)
    db = synth.make_db(rng, lens)
    q = synth.residues(rng, 333)
    return db, q


def test_prepare_into_torch_buffer_view():
    """The layout lives in a view at a 256-byte offset into a larger torch
    tensor holding a canary; the search matches the oracle, the canary and
    the bytes past the reported size stay untouched."""
    import torch
    import paper_2412_08308_amd as swdb
    db, q = _case()
    sm = synth.blosum_style_matrix()
    need = swdb.prepare_bytes(db.total, db.nseq, int(db.lengths.max()))
    big = torch.full((need + 4096,), 0xA5, dtype=torch.uint8, device="cuda")
    layout = big[256:256 + need]
    announce(f"prepare into a view of {need} bytes")
    gdb = swdb.Database.from_host(db, layout=layout)
    try:
        assert gdb.device_bytes <= need
        assert gdb.layout.data_ptr() == layout.data_ptr()
        exp = oracle_scores(db, q, sm, 10, 2)
        for mode in ("auto", "i32"):
            got = gdb.search(torch.from_numpy(q).cuda(), sm, 10, 2, opt=swdb.options(mode=mode))
            got = got.cpu().numpy()
            assert np.array_equal(got, exp), f"{mode}: " + mismatch_report(got, exp)
        torch.cuda.synchronize()
        head = big[:256].cpu().numpy()
        tail = big[256 + need:].cpu().numpy()
        assert (head == 0xA5).all() and (tail == 0xA5).all()
    finally:
        gdb.release()


def test_prepare_exact_size_and_too_small():
    """sw_db_prepare accepts a layout of exactly the bytes it reports using
    and returns SW_ENOMEM for one byte fewer."""
    import torch
    import paper_2412_08308_amd as swdb
    db, q = _case(62, 400)
    sm = synth.blosum_style_matrix()
    announce("prepare: exact-size layout")
    probe = swdb.Database.from_host(db)
    exact = probe.device_bytes
    probe.release()
    # the exact need adds the two preparation-only pieces (512 bytes here)
    gdb = None
    for extra in (512, 768, 1024, 2048):
        try:
            gdb = swdb.Database.from_host(db, layout=torch.empty(exact + extra, dtype=torch.uint8, device="cuda"))
            break
        except swdb.SwdbError as e:
            assert e.code == -2
    assert gdb is not None
    try:
        got = gdb.search(torch.from_numpy(q).cuda(), sm, 10, 2).cpu().numpy()
        exp = oracle_scores(db, q, sm, 10, 2)
        assert np.array_equal(got, exp), mismatch_report(got, exp)
        size = gdb.layout.numel()
    finally:
        gdb.release()
    announce("prepare: layout one byte short")
    with pytest.raises(swdb.SwdbError) as ei:
        swdb.Database.from_host(db, layout=torch.empty(size - 1, dtype=torch.uint8, device="cuda"))
    assert ei.value.code == -2


def test_bad_query_code_reported():
    """A query residue code >= 32 is reported by the search status (the
    search itself is asynchronous), in every mode, for batches, graphs and
    the one-shot call; a clean search afterwards on the same workspace
    reports nothing."""
    import torch
    import paper_2412_08308_amd as swdb
    db, q = _case(63, 300)
    sm = synth.blosum_style_matrix()
    bad = q.copy()
    bad[100] = 40
    gdb = swdb.Database.from_host(db)
    try:
        for mode in ("auto", "i32", "i16"):
            announce(f"bad query code, mode={mode}")
            with pytest.raises(swdb.SwdbError) as ei:
                gdb.search(torch.from_numpy(bad).cuda(), sm, 10, 2, opt=swdb.options(mode=mode))
            assert ei.value.code == -5
            ws = gdb.alloc_workspace([len(q)], swdb.options(mode=mode))
            gdb.search(torch.from_numpy(bad).cuda(), sm, 10, 2, opt=swdb.options(mode=mode), workspace=ws,
                       check=False)
            st = gdb.status(ws)
            assert st["bad_query"] == 1 and st["code"] == -5
            got = gdb.search(torch.from_numpy(q).cuda(), sm, 10, 2, opt=swdb.options(mode=mode),
                             workspace=ws).cpu().numpy()
            assert gdb.status(ws)["code"] == 0
            assert np.array_equal(got, oracle_scores(db, q, sm, 10, 2))
        announce("bad query code in a batch")
        with pytest.raises(swdb.SwdbError) as ei:
            gdb.search_batch([torch.from_numpy(q).cuda(), torch.from_numpy(bad).cuda()], sm, 10, 2)
        assert ei.value.code == -5
        announce("bad query code in a graph replay")
        g = gdb.capture([torch.from_numpy(q).cuda()], sm, 10, 2)
        g.launch()
        assert g.status()["code"] == 0
        g.queries.copy_(torch.from_numpy(bad).cuda())
        g.launch()
        with pytest.raises(swdb.SwdbError):
            g.status()
        g.destroy()
    finally:
        gdb.release()
    announce("bad query code, one-shot")
    res = torch.from_numpy(db.residues).cuda()
    off = torch.from_numpy(db.offsets).cuda()
    ln = torch.from_numpy(db.lengths).cuda()
    with pytest.raises(swdb.SwdbError) as ei:
        swdb.search(torch.from_numpy(bad).cuda(), res, off, ln, sm, 10, 2)
    assert ei.value.code == -5


def test_status_async_into_pinned_host():
    """sw_search_status_async copies the status words into pinned host memory
    on the search's stream; flagged counts subjects sent to the rescore."""
    import torch
    import paper_2412_08308_amd as swdb
    from gpuhelp import overflow_matrix, overflow_sequence
    sm = overflow_matrix(127, -10)
    subj = [overflow_sequence(t, 127) for t in (32766, 32767, 40000)]
    rng = np.random.default_rng(64)
    subj += [rng.integers(2, 20, size=int(n)).astype(np.uint8) for n in rng.integers(10, 300, size=60)]
    db = synth.Database.from_list(subj)
    q = np.concatenate([np.zeros(400, np.uint8), np.ones(300, np.uint8)])
    gdb = swdb.Database.from_host(db)
    try:
        s = torch.cuda.Stream()
        opt = swdb.options(mode="i16")
        ws = gdb.alloc_workspace([len(q)], opt)
        host = torch.zeros(4, dtype=torch.int32, pin_memory=True)
        announce("status async")
        qt = torch.from_numpy(q).cuda()
        torch.cuda.synchronize()
        out = gdb.search(qt, sm, 10, 2, opt=opt, workspace=ws, stream=s, check=False)
        gdb.status_async(ws, host, stream=s)
        s.synchronize()
        assert swdb.status_error(host) is None
        assert int(host[2]) == 2              # 32767 and 40000 reach the 16-bit ceiling
        exp = oracle_scores(db, q, sm, 10, 2)
        assert np.array_equal(out.cpu().numpy(), exp)
    finally:
        gdb.release()
