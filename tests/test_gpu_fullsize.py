"""Every workload at its stated size, every score compared with the CPU oracle
(GPU required).

The oracle's scores of the full workloads take tens of CPU-minutes, so they
are stored as SHA-256 digests by ``tests/golden/make_digests.py`` (which calls
only ``oracle/`` and ``synth/``).  Each GPU row is hashed the same way; a
mismatching row is localised by its 4,096-subject block digests and the
subjects of those blocks are recomputed by the oracle one by one, so the
failure names the subjects and both scores.

* ``q567_vs_200k``: 567-residue query vs 200,000 subjects, the benchmark's
  launch configuration, packed and int32 lanes;
* ``20q_vs_200k``: the 20-query batch (144..5,478 residues) in one persistent
  launch: default, int32, a tuned schedule table (mixed modes, so several
  launch groups) and a HIP-graph replay;
* ``q8000_planted_vs_200k``: the 16-bit overflow workload (1% near-homologs,
  0.5% long subjects) and its 567-residue control query, packed lanes with the
  exact rescore and int32 lanes;
* ``serve_500k``: the first requests of the serving stream through the
  continuous-batching server against the 500,000-subject database.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
import synth
from gpuhelp import announce, have_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU"),
              pytest.mark.timeout(900)]

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "oracle_digests.json")


def _golden():
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_digests", os.path.join(HERE, "golden", "make_digests.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    with open(GOLDEN) as fh:
        data = json.load(fh)
    assert data["oracle_source_sha256"] == mk.oracle_source_sha(), \
        "stored digests come from another oracle source: rerun tests/golden/make_digests.py"
    return data, mk


@pytest.fixture(scope="module")
def golden():
    return _golden()


_W = {}


def _inputs(mk, name):
    if name not in _W:
        _W[name] = mk.workload_inputs(name)
    return _W[name]


def _entry(golden, name):
    data, mk = golden
    assert name in data["workloads"], f"no stored digests for {name}: run tests/golden/make_digests.py {name}"
    e = data["workloads"][name]
    db, qs, sm, go, ge = _inputs(mk, name)
    assert e["config_sha256"] == mk.config_sha(db, qs, sm, go, ge), \
        f"{name}: inputs differ from the ones the digests were made from"
    return e, (db, qs, sm, go, ge), mk


def _compare(tag, got_rows, e, inputs, mk, rows=None):
    """Assert every GPU row equals the oracle's by digest; localise otherwise."""
    db, qs, sm, go, ge = inputs
    rows = range(len(got_rows)) if rows is None else rows
    bad = []
    for k, r in zip(rows, got_rows):
        g = np.ascontiguousarray(np.asarray(r, dtype=np.int64))
        want = e["rows"][k]
        if hashlib.sha256(g.astype("<i4").tobytes()).hexdigest() == want["sha256"]:
            continue
        d = mk.row_digest(np.clip(g, 0, None))
        blocks = [b for b, (x, y) in enumerate(zip(d["blocks"], want["blocks"])) if x != y] or [0]
        ids = np.concatenate([np.arange(b * e["block"], min((b + 1) * e["block"], db.nseq)) for b in blocks[:4]])
        exp = oracle.search_db(qs[k], db, sm, go, ge, ids=ids)
        diff = ids[g[ids] != exp]
        sample = "; ".join(f"subject {int(s)}: gpu {int(g[s])} oracle {int(exp[np.searchsorted(ids, s)])}"
                           for s in diff[:6])
        bad.append(f"row {k} (query {len(qs[k])}): blocks {blocks[:8]} differ; {len(diff)} mismatches in the "
                   f"first {min(len(blocks), 4)} of them; {sample}")
    assert not bad, f"{tag}: " + " | ".join(bad)


def _gpu_db(db):
    import paper_2412_08308_amd as swdb
    return swdb.Database.from_host(db)


def test_q567_vs_200k_full(golden):
    import torch
    import paper_2412_08308_amd as swdb
    e, inp, mk = _entry(golden, "q567_vs_200k")
    db, qs, sm, go, ge = inp
    gdb = _gpu_db(db)
    try:
        q = torch.from_numpy(qs[0]).cuda()
        for mode in ("auto", "i32", "tuned"):
            if mode == "tuned":
                gdb.set_tuning([{"qlen": 400, "mode": 2, "waves": 8, "lane_cells": 49152},
                                {"qlen": 800, "mode": 1, "waves": 4, "lane_cells": 24576}])
            announce(f"q567_vs_200k full, mode={mode}")
            got = gdb.search(q, sm, go, ge, opt=swdb.options(mode=mode)).cpu().numpy()
            _compare(f"q567_vs_200k {mode}", [got], e, inp, mk)
    finally:
        gdb.release()


def test_20q_vs_200k_full(golden):
    """The batched workload at full size in every launch form."""
    import torch
    import paper_2412_08308_amd as swdb
    e, inp, mk = _entry(golden, "20q_vs_200k")
    db, qs, sm, go, ge = inp
    gdb = _gpu_db(db)
    try:
        qts = [torch.from_numpy(x).cuda() for x in qs]
        # a tuned table with both arithmetic modes and several schedules: the
        # batch runs as several persistent launches, one per schedule
        gdb.set_tuning([{"qlen": 300, "mode": 2, "waves": 8, "lane_cells": 49152},
                        {"qlen": 1000, "mode": 1, "waves": 4, "lane_cells": 98304},
                        {"qlen": 2500, "mode": 2, "waves": 4, "lane_cells": 98304},
                        {"qlen": 6000, "mode": 2, "waves": 8, "lane_cells": 196608}])
        for mode in ("auto", "i32", "tuned"):
            announce(f"20q_vs_200k full, mode={mode}")
            got = gdb.search_batch(qts, sm, go, ge, opt=swdb.options(mode=mode)).cpu().numpy()
            _compare(f"20q_vs_200k {mode}", got, e, inp, mk)
        announce("20q_vs_200k full, graph replay")
        cat = torch.cat(qts)
        lens = [len(x) for x in qs]
        offs = np.concatenate([[0], np.cumsum(lens[:-1])])
        g = gdb.capture((cat, offs, lens), sm, go, ge, opt=swdb.options(mode="auto"))
        for rep in range(2):
            g.out.fill_(-7)
            g.launch()
            g.status()
            _compare(f"20q_vs_200k graph replay {rep}", g.out.cpu().numpy(), e, inp, mk)
        g.destroy()
    finally:
        gdb.release()


def test_planted_overflow_full(golden):
    """16-bit lanes overflow on the near-homologs and long subjects: the exact
    int32 rescore must restore every score; int32 lanes agree."""
    import torch
    import paper_2412_08308_amd as swdb
    e, inp, mk = _entry(golden, "q8000_planted_vs_200k")
    db, qs, sm, go, ge = inp
    gdb = _gpu_db(db)
    try:
        for mode in ("auto", "i32"):
            rows = []
            for k, x in enumerate(qs):
                announce(f"planted full, mode={mode}, query {len(x)}")
                opt = swdb.options(mode=mode)
                ws = gdb.alloc_workspace([len(x)], opt)
                rows.append(gdb.search(torch.from_numpy(x).cuda(), sm, go, ge, opt=opt, workspace=ws).cpu().numpy())
                st = gdb.status(ws, raise_on_error=True)
                if mode == "auto":
                    want = int(np.sum(np.asarray(rows[-1]) >= 32767))
                    assert st["flagged"] == want, f"flagged {st['flagged']}, scores >= 32767: {want}"
            _compare(f"planted {mode}", rows, e, inp, mk)
        assert e["rows"][0]["max"] >= 32767 and e["rows"][1]["max"] < 32767
    finally:
        gdb.release()


def test_serve_500k_requests(golden):
    """The serving stream's first requests, submitted to the server among
    others, against the 500,000-subject database: each result equals the
    oracle's row."""
    import paper_2412_08308_amd as swdb
    from paper_2412_08308_amd.serve import GpuBackend, Server
    e, inp, mk = _entry(golden, "serve_500k")
    db, qs, sm, go, ge = inp
    gdb = _gpu_db(db)
    try:
        be = GpuBackend(gdb, sm, go, ge, mode="auto", n_streams=4)
        extra = synth.serve_requests(24)[len(qs):]          # later requests of the same stream
        announce(f"serve_500k: {len(qs)} checked requests among {len(qs) + len(extra)}")
        with Server(be, max_batch=4) as srv:
            futs = []
            for k in range(len(qs)):
                futs.append(srv.submit(qs[k]))
                if k < len(extra):
                    srv.submit(extra[k])
            got = [f.result(timeout=600) for f in futs]
        assert srv.stats()["errors"] == 0
        _compare("serve_500k", got, e, inp, mk)
    finally:
        gdb.release()


def test_pair_162k_x_172k(golden):
    """The paper's smallest DNA pair size, scored by the whole device; the
    score equals the oracle's (stored by the digest script)."""
    import torch
    import paper_2412_08308_amd as swdb
    data, mk = golden
    p = data["pairs"]["dna_162k_x_172k"]
    a, b = synth.dna_pair(p["m"], p["n"], seed=p["seed"])
    sm = synth.dna_matrix(synth.DNA_MATCH, synth.DNA_MISMATCH)
    go, ge = synth.DNA_GAP_OPEN, synth.DNA_GAP_EXTEND
    h = hashlib.sha256()
    for x in (a, b, sm.astype("<i4")):
        h.update(np.ascontiguousarray(x).tobytes())
    h.update(f"{go},{ge}".encode())
    assert h.hexdigest() == p["config_sha256"]
    qa, qb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    for opt in (None, swdb.options(pair_rows=8, pair_cols=128), swdb.options(pair_rows=16, pair_cols=512),
                swdb.options(pair_mode=2, pair_rows=4), swdb.options(pair_mode=2, pair_rows=10)):
        announce(f"pair 162k x 172k {opt and (opt.pair_mode, opt.pair_rows, opt.pair_cols)}")
        got = int(swdb.pair_score(qa, qb, sm, go, ge, opt=opt).cpu().item())
        assert got == p["score"], f"gpu {got} oracle {p['score']}"
