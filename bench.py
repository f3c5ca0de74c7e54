#!/usr/bin/env python3
"""Benchmark of the gfx950 Smith-Waterman / Gotoh protein database search.

Workload (default): one query of 567 residues against 200,000 synthetic subjects
(log-normal lengths, median 300, about 75M residues), BLOSUM62-style matrix,
gap penalties 10 / 2, database resident and prepared in HBM.  A step is one
search call: plan upload, query profile, the persistent search kernel and the
exact int32 rescore of 16-bit overflows.  GCUPS = query length x database
residues / step time (the paper's Section 3.2 definition).

Printed (one JSON line): the headline GCUPS of the default exact mode, the
int32-lane kernel on the same input, a batched 20-query launch, the 16-bit
overflow workload, a Poisson serving run, single long DNA pairs at the
paper's pairwise sizes, alignments (traceback) of the best hits, the
integer-VALU roofline of the search kernel (timed
live with HIP events on its stream), and the CPU oracle timed on a bounded
sample on this host.

Only one GPU is used; ``--gpus N`` with N > 1 exits with a message.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12     # 256 CUs x 4 SIMD16 x 2.4 GHz, lane-ops
PAPER_OPS_PER_CELL = 12                       # the paper's Algorithm 1


class HipEvents:
    """Minimal HIP event API through the process's HIP runtime."""

    def __init__(self):
        self.h = ctypes.CDLL("libamdhip64.so.7")
        self.h.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.h.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.h.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        self.h.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def create(self):
        e = ctypes.c_void_p()
        if self.h.hipEventCreate(ctypes.byref(e)) != 0:
            raise RuntimeError("hipEventCreate failed")
        return e

    def ms(self, a, b) -> float:
        self.h.hipEventSynchronize(b)
        f = ctypes.c_float()
        if self.h.hipEventElapsedTime(ctypes.byref(f), a, b) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(f.value)

    def destroy(self, e):
        self.h.hipEventDestroy(e)


def isa_counts():
    path = os.path.join(ROOT, "paper_2412_08308_amd", "isa_counts.json")
    if not os.path.exists(path):
        from paper_2412_08308_amd import isa_count
        return isa_count.run()
    with open(path) as fh:
        return json.load(fh)


KNOBS = {}
TRAFFIC = os.path.join(ROOT, "profiles", "traffic_k_search_q567_vs_200k.json")

# kernel variant (sw_plan_stats.variant) -> (hot-loop instruction count key of
# isa_count.py, kernel); the count is that of single-lane groups (K = 1), the
# fewest instructions per cell the variant issues
VARIANTS = {
    0: ("i32_p8_lds_k1", "k_search<32,1,false> (int32 lanes, 8-bit profile)"),
    1: ("i32_p16_lds_k1", "k_search<32,2,false> (int32 lanes, 16-bit profile)"),
    2: ("i16_lds_k1", "k_search<24,2,true> (packed 16-bit lanes, 16-bit profile)"),
    3: ("i16_p8_lds_k1", "k_search<24,1,true> (packed 16-bit lanes, 8-bit profile)"),
}


def kernel_fingerprint() -> str:
    """Hash of the sources that decide what the search kernel reads and writes
    (kernels, plan, layout); stored counter readings are used only while it
    matches."""
    import hashlib
    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_2412_08308_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".h", ".hip", ".cpp")) and f not in ("sw_isa_probe.hip", "sw_pair.hip", "sw_k_rescore.hip",
                                                             "sw_pair_flow.hip", "sw_swar8.h"):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def traffic_bytes(mode: str):
    """HBM bytes per search-kernel launch from the committed FETCH_SIZE /
    WRITE_SIZE readings, each scaled by the same counter's reading for a
    device-to-device copy of known size; None if absent or stale."""
    if not os.path.exists(TRAFFIC):
        return None
    with open(TRAFFIC) as fh:
        t = json.load(fh)
    e = t.get("modes", {}).get(mode)
    if not e or t.get("fingerprint") != kernel_fingerprint() or KNOBS.get("lane_cells") or KNOBS.get("waves"):
        return None
    c = t["copy"]
    fetch = e["fetch_kib"] * c["bytes"] / c["fetch_kib"]
    write = e["write_kib"] * c["bytes"] / c["write_kib"]
    return {"bytes": int(fetch + write), "fetch_bytes": int(fetch), "write_bytes": int(write)}


_DIGESTS = {}


def digests():
    """The oracle's digests of the full workloads (tests/golden/oracle_digests.json,
    written by tests/golden/make_digests.py from oracle/ and synth/ only)."""
    if not _DIGESTS:
        path = os.path.join(ROOT, "tests", "golden", "oracle_digests.json")
        if os.path.exists(path):
            with open(path) as fh:
                _DIGESTS.update(json.load(fh))
    return _DIGESTS


def digest_parity(name, rows, first_row=0):
    """Compare GPU score rows (int32, caller's order) with the stored oracle
    digests of workload ``name``: rows and 4,096-subject blocks that differ."""
    import hashlib
    import numpy as np
    e = digests().get("workloads", {}).get(name)
    if e is None:
        return {"status": "no stored digests"}
    bad_rows, bad_blocks, n = 0, 0, 0
    for k, r in enumerate(rows):
        want = e["rows"][first_row + k]
        b = np.ascontiguousarray(np.asarray(r)).astype("<i4")
        n += len(b)
        if hashlib.sha256(b.tobytes()).hexdigest() != want["sha256"]:
            bad_rows += 1
            blk = e["block"]
            bad_blocks += sum(hashlib.sha256(b[i:i + blk].tobytes()).hexdigest()[:16] != want["blocks"][i // blk]
                              for i in range(0, len(b), blk))
    return {"rows": len(rows), "scores": n, "rows_mismatched": bad_rows, "blocks_mismatched": bad_blocks}


def timed_search(gdb, queries, sm, go, ge, mode, steps, warmup, ev, batch=False, extra=None):
    """Run warmup + steps searches; wall time per step and the search kernel's
    own time (HIP events recorded by the library around its launch).  ``extra``:
    option fields set on top of the mode (a tuned schedule)."""
    import torch
    import paper_2412_08308_amd as swdb
    lens = [int(q.numel()) for q in queries]
    kw = {**KNOBS, **(extra or {})}
    base = swdb.options(mode=mode, **kw)
    ws = gdb.alloc_workspace(lens, base)
    out = torch.empty((len(queries), gdb.nseq) if batch else (gdb.nseq,), dtype=torch.int32, device="cuda")
    if batch:
        cat = torch.cat([q.reshape(-1) for q in queries])
        offs = [0]
        for L in lens[:-1]:
            offs.append(offs[-1] + L)
        qarg = (cat, offs, lens)

    def one(opt):
        if batch:
            gdb.search_batch(qarg, sm, go, ge, opt=opt, out=out, workspace=ws, check=False)
        else:
            gdb.search(queries[0], sm, go, ge, opt=opt, out=out, workspace=ws, check=False)

    for _ in range(warmup):
        one(base)
    torch.cuda.synchronize()
    evs = []
    for _ in range(steps):
        o = swdb.options(mode=mode, **kw)
        e = (ev.create(), ev.create(), ev.create())
        o.ev_search_begin, o.ev_search_end, o.ev_rescore_end = e[0].value, e[1].value, e[2].value
        evs.append((o, e))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for o, _ in evs:
        one(o)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    k = [ev.ms(e[0], e[1]) for _, e in evs]
    r = [ev.ms(e[1], e[2]) for _, e in evs]
    for _, e in evs:
        for x in e:
            ev.destroy(x)
    status = gdb.status(ws, raise_on_error=True)     # the last timed search's status words
    flagged = status["flagged"]
    plan = gdb.plan_info(lens, base)
    plan["variant"] = swdb.select_variant(sm, go, base)   # plan_info reports the 16-bit sizing variant
    return dict(wall_ms=wall * 1e3, kernel_ms=sum(k) / len(k), kernel_min_ms=min(k),
                rescore_ms=sum(r) / len(r), flagged=flagged, plan=plan, out=out)


def serving(args, capacity_gcups, mode):
    """Poisson request stream against the 500,000-subject serving database through
    the continuous-batching server; p50/p99 latency and sustained GCUPS."""
    import numpy as np
    import torch

    import paper_2412_08308_amd as swdb
    import synth
    from paper_2412_08308_amd.serve import GpuBackend, Server

    w5 = synth.workload("serve_500k", scale=args.serve_scale)
    gdb = swdb.Database.from_host(w5.db)
    n = args.serve_requests
    qs = synth.serve_requests(n)
    qlens = np.array([len(q) for q in qs])
    # launches of about serve_slice_ms: capacity in cells per ms, over the cells
    # one lane sweeps per lane cell (two subjects per lane in the packed modes)
    per_lane = 1 if mode == "i32" else 2
    slice_mcells = int(capacity_gcups * args.serve_slice_ms / per_lane) if args.serve_slice_ms > 0 else 0
    knobs = dict(KNOBS)
    if args.serve_lane_cells:
        knobs["lane_cells"] = args.serve_lane_cells
    be = GpuBackend(gdb, w5.matrix, w5.gap_open, w5.gap_extend, mode=mode, n_streams=4,
                    slice_mcells=slice_mcells, **knobs)
    rate = capacity_gcups * 1e9
    srv_kw = dict(max_batch=16, rate_guess=rate, long_s=args.serve_long_ms / 1e3, long_depth=args.serve_long_depth)
    with Server(be, **srv_kw) as srv:                    # warm-up: plans, allocator, code
        for f in [srv.submit(q) for q in qs[:8]]:
            f.result()
    torch.cuda.synchronize()
    # each request alone (the server idle when it arrives): its service time
    edges = [int(x) for x in np.percentile(qlens, [100 / 3, 200 / 3])]
    alone = Server(be, **srv_kw).start()
    for q in qs:
        alone.submit(q).result()
    alone.stop()
    alone_cls = alone.stats_by_length(edges)
    mean_m = float(np.mean(qlens))
    # load rho is the utilisation: arrival rate x the mean service time of a
    # request served alone by the same server (options, slices, streams)
    alone_mean_s = float(np.mean(alone.latencies))
    serve_capacity = mean_m * w5.db.total / alone_mean_s / 1e9
    runs, checks = [], []
    for policy in args.serve_policies:
        arng = np.random.default_rng(78)          # the same arrival times for every policy
        for rho in args.serve_rho:
            lam = rho / alone_mean_s
            arrivals = synth.poisson_arrivals(arng, lam, n)
            srv = Server(be, policy=policy, **srv_kw).start()
            futs = []
            t0 = time.perf_counter()
            for k, q in enumerate(qs):
                dt = t0 + arrivals[k] - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
                futs.append(srv.submit(q))
            res = [f.result() for f in futs]
            srv.stop()
            st = srv.stats()
            if args.serve_scale == 1.0:
                # every score of the first requests against the oracle's digests,
                # and a seeded sample of other requests on sampled subjects
                nd = len(digests().get("workloads", {}).get("serve_500k", {}).get("rows", []))
                checks.append(("digest", digest_parity("serve_500k", res[:nd])))
                checks.append(("sample", sample_parity(w5.db, qs, res, w5.matrix, w5.gap_open, w5.gap_extend,
                                                       seed=len(runs))))
            print(f"[bench] serving {policy} rho={rho}: p50 {st['p50_s'] * 1e3:.1f} ms p99 {st['p99_s'] * 1e3:.1f} ms",
                  file=sys.stderr, flush=True)
            cls = srv.stats_by_length(edges)
            offered = lam * mean_m * w5.db.total / 1e9
            runs.append({"policy": policy, "rho": rho, "rate_per_s": round(lam, 2), "requests": n,
                         "offered_gcups": round(offered, 1),
                         "offered_over_search_capacity": round(offered / capacity_gcups, 3),
                         "p50_ms": round(st["p50_s"] * 1e3, 2), "p99_ms": round(st["p99_s"] * 1e3, 2),
                         "sustained_gcups": round(st["sustained_gcups"], 1),
                         "mean_batch": round(st["mean_batch"], 2), "max_batch": st["max_batch"],
                         "by_length": [{"qlen": [c["qlen_lo"], c["qlen_hi"]], "requests": c["requests"],
                                        "p50_ms": round(c["p50_s"] * 1e3, 2), "p99_ms": round(c["p99_s"] * 1e3, 2),
                                        "p99_over_alone_p99": round(c["p99_s"] / a["p99_s"], 2)}
                                       for c, a in zip(cls, alone_cls)]})
    gdb.release()
    parity = None
    if checks:
        dg = [c for k, c in checks if k == "digest" and "rows" in c]
        sp = [c for k, c in checks if k == "sample"]
        parity = {"digest_requests": sum(c["rows"] for c in dg), "digest_rows_mismatched":
                  sum(c["rows_mismatched"] for c in dg),
                  "sampled_requests": sum(c["requests"] for c in sp),
                  "sampled_scores": sum(c["scores"] for c in sp), "sample_mismatches": sum(c["mismatches"] for c in sp)}
    return {"workload": f"{w5.db.nseq} subjects ({w5.db.total} residues); {n} queries log-normal median 350 "
                        "clamped 50-5000; Poisson arrivals at utilisation rho (arrival rate x mean alone "
                        "service time)",
            "capacity_gcups": round(capacity_gcups, 1),
            "alone_mean_ms": round(alone_mean_s * 1e3, 2),
            "alone_capacity_gcups": round(serve_capacity, 1),
            "server": {"slice_mcells": slice_mcells, "slice_ms": args.serve_slice_ms, "long_ms": args.serve_long_ms,
                       "long_depth": args.serve_long_depth, "lane_cells": args.serve_lane_cells,
                       "size_ratio": 4.0, "streams": 4, "max_batch": 16},
            "alone_by_length": [{"qlen": [c["qlen_lo"], c["qlen_hi"]], "requests": c["requests"],
                                 "p50_ms": round(c["p50_s"] * 1e3, 2), "p99_ms": round(c["p99_s"] * 1e3, 2)}
                                for c in alone_cls],
            "runs": runs, "parity": parity}


def sample_parity(db, qs, res, sm, go, ge, seed=0, nreq=6, nsub=64):
    """The oracle on a seeded sample of requests, each on a seeded sample of
    subjects (the longest ones included)."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(900 + seed)
    reqs = rng.choice(len(qs), size=min(nreq, len(qs)), replace=False)
    longest = np.argsort(-db.lengths, kind="stable")[:8]
    bad, n = 0, 0
    for k in reqs:
        ids = np.unique(np.concatenate([longest, rng.choice(db.nseq, nsub, replace=False)]))
        exp = oracle.search_db(qs[k], db, sm, go, ge, ids=ids)
        bad += int(np.sum(np.asarray(res[k])[ids] != exp))
        n += len(ids)
    return {"requests": len(reqs), "scores": n, "mismatches": bad}


def planted(args, ev):
    """Overflow workload: 8,000-residue query vs the 200,000-subject database with long
    subjects and near-homologs planted; 16-bit lanes + int32 rescore vs int32."""
    import torch

    import paper_2412_08308_amd as swdb
    import synth
    w4 = synth.workload("q8000_planted_vs_200k", scale=args.scale)
    gdb = swdb.Database.from_host(w4.db)
    q = torch.from_numpy(w4.queries[0]).cuda()
    cells = len(w4.queries[0]) * w4.db.total
    a = timed_search(gdb, [q], w4.matrix, w4.gap_open, w4.gap_extend, "auto", args.planted_steps, 1, ev)
    b = timed_search(gdb, [q], w4.matrix, w4.gap_open, w4.gap_extend, "i32", args.planted_steps, 1, ev)
    parity = None
    if args.scale == 1.0:
        parity = {"auto": digest_parity("q8000_planted_vs_200k", [a["out"].cpu().numpy()]),
                  "i32": digest_parity("q8000_planted_vs_200k", [b["out"].cpu().numpy()])}
    gdb.release()
    return {"workload": f"query 8000 vs {w4.db.nseq} subjects ({w4.db.total} residues): 0.5% long "
                        "10,000-35,000, 1% near-homologs 30-90% identity",
            "i16_rescore_gcups": round(cells / (a["wall_ms"] / 1e3) / 1e9, 1),
            "i16_search_ms": round(a["kernel_ms"], 2), "rescore_ms": round(a["rescore_ms"], 2),
            "flagged": a["flagged"], "i32_gcups": round(cells / (b["wall_ms"] / 1e3) / 1e9, 1),
            "i32_search_ms": round(b["kernel_ms"], 2), "cells": cells, "parity": parity}


def pairwise(args, ev):
    """Single long DNA pairs at the sizes of the paper's pairwise workload
    (synthetic homologous sequences, +1/-3, gaps 5/2): the whole device on one
    matrix through the planner's pass (one pipelined launch, or anti-diagonal
    tile launches), and the tile launches beside it for comparison.  The
    largest pairs (9T and 35T cells) run once each, with no comparison."""
    import numpy as np
    import torch

    import paper_2412_08308_amd as swdb
    import synth
    sm = synth.dna_matrix(synth.DNA_MATCH, synth.DNA_MISMATCH)
    go, ge = synth.DNA_GAP_OPEN, synth.DNA_GAP_EXTEND
    p8 = int(sm.max()) + go <= 127 and int(sm.min()) + go >= -128   # 8-bit profile entries
    isa = isa_counts()
    runs = []
    for k in args.pair_sizes:
        m, n = synth.DNA_PAIR_SIZES[k]
        a, b = synth.dna_pair(m, n, seed=k)
        qa, qb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
        ws = torch.empty(swdb.pair_workspace_bytes(m, n), dtype=torch.uint8, device="cuda")
        out = torch.empty(1, dtype=torch.int32, device="cuda")
        big = m * n > 2e12
        steps, warm = (1, 0) if big else (args.pair_steps, 1)
        for _ in range(warm):
            swdb.pair_score(qa, qb, sm, go, ge, workspace=ws, out=out)
        torch.cuda.synchronize()
        walls, kers = [], []
        for _ in range(steps):
            o = swdb.options()
            e0, e1 = ev.create(), ev.create()
            o.ev_search_begin, o.ev_search_end = e0.value, e1.value
            t0 = time.perf_counter()
            swdb.pair_score(qa, qb, sm, go, ge, opt=o, workspace=ws, out=out)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
            kers.append(ev.ms(e0, e1))
            ev.destroy(e0)
            ev.destroy(e1)
        wall = sum(walls) / len(walls)
        cu = torch.cuda.get_device_properties(0).multi_processor_count
        plan = swdb.pair_plan(m, n, swdb.options(pair_sm_max=max(int(sm.max()), 1), pair_entry_bytes=1 if p8 else 2),
                              cu_count=cu)
        pass_s = sum(kers) / len(kers) / 1e3          # between the events around the pass's launches
        kind = "flow" if plan["flow"] else "pair"
        ops = isa[f"{kind}_r{plan['rows']}_p{8 if p8 else 16}"]["valu_per_cell"]
        # the anti-diagonal tile launches on the same pair, for comparison
        cmp = None
        if plan["flow"] and not big:
            ot = swdb.options(pair_mode="tiles")
            swdb.pair_score(qa, qb, sm, go, ge, opt=ot, workspace=ws, out=out)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            swdb.pair_score(qa, qb, sm, go, ge, opt=ot, workspace=ws, out=out)
            torch.cuda.synchronize()
            cmp = {"tiles_ms": round((time.perf_counter() - t0) * 1e3, 2), "tiles_score": int(out.cpu().item())}
            swdb.pair_score(qa, qb, sm, go, ge, workspace=ws, out=out)
            torch.cuda.synchronize()
        runs.append({"m": m, "n": n, "cells": m * n, "gcups": round(m * n / wall / 1e9, 1),
                     "ms": round(wall * 1e3, 2), "kernel_ms": round(pass_s * 1e3, 2),
                     "score": int(out.cpu().item()), "steps": steps,
                     "plan": {k2: plan[k2] for k2 in ("flow", "rows", "lanes", "cols", "bands", "chunks", "launches",
                                                      "groups", "group_waves")},
                     "tile_launches": cmp,
                     "model_ms": round(plan["est_ms"], 1), "isa_valu_per_cell": ops,
                     "roofline_frac": round(m * n * ops / pass_s / 1e12 / PEAK_VALU_TOPS, 4)})
        print(f"[bench] pair {m}x{n}: {runs[-1]['gcups']} GCUPS", file=sys.stderr, flush=True)
        del qa, qb, ws
    return {"workload": "one DNA pair per size (paper's pairwise sizes, synthetic 80%-identity homologs, "
                        "+1/-3, gaps 5/2), int32 lanes; the planner's pass: one pipelined launch (flow) or "
                        "anti-diagonal tile launches", "runs": runs}


def alignments(args, w, scores):
    """Traceback of the best hits (the paper's optional step after the score):
    the query against its 16 highest-scoring subjects, one sw_align_pair call
    each (score pass, direction-code pass, walk), one 50,000-base DNA pair
    against a homolog, the paper's smallest DNA pair (162K x 172K, codes for
    the whole matrix) and its 1M x 1M pair (codes recomputed block by block);
    wall time per call.  ``args.align_legs`` selects among top, 50k, 162k, 1m."""
    import numpy as np
    import torch

    import paper_2412_08308_amd as swdb
    import synth
    legs = set(args.align_legs.split(","))
    out = {}
    sm = synth.dna_matrix(synth.DNA_MATCH, synth.DNA_MISMATCH)
    go, ge = synth.DNA_GAP_OPEN, synth.DNA_GAP_EXTEND
    if "top" in legs:
        q = torch.from_numpy(w.queries[0]).cuda()
        top = torch.topk(scores.to(torch.int64), 16).indices.cpu().numpy()
        subs = [torch.from_numpy(np.ascontiguousarray(w.db.subject(int(i)))).cuda() for i in top]
        ws = torch.empty(max(swdb.align_workspace_bytes(len(w.queries[0]), int(s.numel())) for s in subs),
                         dtype=torch.uint8, device="cuda")
        swdb.align_pair(q, subs[0], w.matrix, w.gap_open, w.gap_extend, workspace=ws)      # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = [swdb.align_pair(q, s, w.matrix, w.gap_open, w.gap_extend, workspace=ws) for s in subs]
        dt = time.perf_counter() - t0
        cells = len(w.queries[0]) * sum(int(s.numel()) for s in subs)
        out["top_hits"] = {"alignments": len(subs), "ms_per_alignment": round(dt / len(subs) * 1e3, 2),
                           "cells": cells,
                           "best": {k: res[0][k] for k in ("score", "q_begin", "s_begin", "q_end", "s_end")},
                           "best_ops": len(res[0]["ops"])}
        del ws
    if "50k" in legs:
        a, b = synth.dna_pair(50_000, 50_000, seed=11)
        qa, qb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
        wsd = torch.empty(swdb.align_workspace_bytes(50_000, 50_000), dtype=torch.uint8, device="cuda")
        swdb.align_pair(qa, qb, sm, go, ge, workspace=wsd)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = swdb.align_pair(qa, qb, sm, go, ge, workspace=wsd)
        dt2 = time.perf_counter() - t1
        del wsd
        out["dna_50k"] = {"ms": round(dt2 * 1e3, 1), "gcups_two_passes": round(2 * 50_000 ** 2 / dt2 / 1e9, 1),
                          "score": r["score"], "ops": len(r["ops"])}
    # the paper's smallest pairwise size (the pair of the pairwise leg): 2.8e10
    # cells, 14 GB of direction codes; and its 1M x 1M pair, whose codes for the
    # whole matrix would take 500 GB, recomputed block by block (65536 x 65536)
    # from checkpoints.  The operations are re-scored on the host.
    for leg, k, name in (("162k", 0, "dna_162k_x_172k"), ("1m", 2, "dna_1m_x_1m_blocked")):
        if leg not in legs:
            continue
        m, n = synth.DNA_PAIR_SIZES[k]
        a, b = synth.dna_pair(m, n, seed=k)
        qa, qb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
        wsd = torch.empty(swdb.align_workspace_bytes(m, n), dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        big = swdb.align_pair(qa, qb, sm, go, ge, workspace=wsd)
        dt3 = time.perf_counter() - t2
        out[name] = {"ms": round(dt3 * 1e3, 1), "cells": m * n, "workspace_gb": round(wsd.numel() / 1e9, 2),
                     "score": big["score"], "ops": len(big["ops"]),
                     "begin": [big["q_begin"], big["s_begin"]], "end": [big["q_end"], big["s_end"]],
                     "ops_rescore": ops_score(a, b, big, sm, go, ge)}
        del wsd
    return out


def ops_score(a, b, r, sm, go, ge):
    """Score of an alignment's operations (a gap of length L costs
    go + (L - 1) * ge); equals r["score"] for a consistent alignment."""
    i, j, total, prev = r["q_begin"] - 1, r["s_begin"] - 1, 0, "M"
    for op in r["ops"]:
        if op == "M":
            total += int(sm[a[i], b[j]])
            i, j = i + 1, j + 1
        else:
            total -= ge if op == prev else go
            i, j = (i + 1, j) if op == "I" else (i, j + 1)
        prev = op
    return total


def paper_model(cells, kernel_s, variant):
    """Algorithm 1's 12 operations per cell against the lane-operation peak of
    the kernel's own arithmetic: 39.32 T 32-bit lane-ops/s for int32 lanes,
    twice that for packed 16-bit lanes (each 32-bit lane-op carries two
    16-bit operations)."""
    lanes_per_op = 2 if variant in (2, 3) else 1
    peak = PEAK_VALU_TOPS * lanes_per_op
    achieved = cells * PAPER_OPS_PER_CELL / kernel_s / 1e12
    return {"ops_per_cell": PAPER_OPS_PER_CELL, "achieved": round(achieved, 3), "peak": round(peak, 3),
            "unit": "TOP/s", "frac": round(achieved / peak, 4),
            "peak_gcups": round(peak * 1e3 / PAPER_OPS_PER_CELL, 1),
            "peak_basis": "16-bit lane-ops (two per 32-bit lane)" if lanes_per_op == 2 else "32-bit lane-ops"}


def timed_graph(gdb, queries, sm, go, ge, steps, ev):
    """The batch as a captured HIP graph (sw_graph_create): one warm-up replay,
    then ``steps`` replays timed by wall clock and by HIP events around each
    replay on its stream."""
    import numpy as np
    import torch
    import paper_2412_08308_amd as swdb
    lens = [int(q.numel()) for q in queries]
    cat = torch.cat([q.reshape(-1) for q in queries])
    offs = np.concatenate([[0], np.cumsum(lens[:-1])]).astype(np.int64)
    g = gdb.capture((cat, offs, lens), sm, go, ge, opt=swdb.options(mode="auto", **KNOBS))
    s = torch.cuda.current_stream()
    g.launch()
    g.status()
    pairs = [(ev.create(), ev.create()) for _ in range(steps)]
    h = ev.h
    h.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in pairs:
        h.hipEventRecord(a, ctypes.c_void_p(s.cuda_stream))
        g.launch()
        h.hipEventRecord(b, ctypes.c_void_p(s.cuda_stream))
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    replay = sum(ev.ms(a, b) for a, b in pairs) / steps
    for a, b in pairs:
        ev.destroy(a)
        ev.destroy(b)
    g.status()
    out = g.out.cpu().numpy()
    g.destroy()
    return {"wall_ms": wall * 1e3, "replay_ms": replay, "out": out}


def cpu_baseline(w, seconds: float):
    """The oracle (plain C, int64, threads over subjects) on a random sample of
    the same database, sized for about ``seconds`` of host time."""
    import numpy as np
    import oracle
    q = w.queries[0]
    threads = min(16, len(os.sched_getaffinity(0)))      # the host cores this process may use (at most 16)
    rng = np.random.default_rng(123)
    n = w.db.nseq
    ids = rng.permutation(n)
    take = min(n, max(64, n // 400))
    t0 = time.perf_counter()
    oracle.search_db(q, w.db, w.matrix, w.gap_open, w.gap_extend, ids=ids[:take], threads=threads)
    dt = time.perf_counter() - t0
    rate = len(q) * int(w.db.lengths[ids[:take]].sum()) / max(dt, 1e-9)
    want = int(min(n, take * max(1.0, seconds / max(dt, 1e-3))))
    sel = ids[:want]
    cells = len(q) * int(w.db.lengths[sel].sum())
    t0 = time.perf_counter()
    scores = oracle.search_db(q, w.db, w.matrix, w.gap_open, w.gap_extend, ids=sel, threads=threads)
    dt = time.perf_counter() - t0
    cpu = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                cpu = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return ({"value": round(cells / dt / 1e9, 3), "unit": "GCUPS", "cores": threads, "kind": "oracle",
             "sample": f"query 567 vs {want} of {n} subjects drawn at random ({cells:.3e} cells, {dt:.1f} s)",
             "cpu": cpu, "calibration_gcups": round(rate / 1e9, 3)}, sel, scores)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", default="auto", choices=["auto", "i16", "i32", "tuned"])
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--scale", type=float, default=1.0, help="database scale (1.0 = 200,000 subjects)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-i32", action="store_true")
    ap.add_argument("--lane-cells", type=int, default=0)
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--lds-limit", type=int, default=0)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-planted", action="store_true")
    ap.add_argument("--planted-steps", type=int, default=3)
    ap.add_argument("--no-pair", action="store_true")
    ap.add_argument("--no-align", action="store_true")
    ap.add_argument("--align-legs", default="top,50k,162k,1m",
                    help="alignment cases: top (16 best hits), 50k, 162k, 1m (DNA pairs)")
    ap.add_argument("--pair-sizes", type=int, nargs="+", default=[0, 1, 2, 3, 4],
                    help="indices into the paper's DNA pair sizes (162Kx172K .. 7Mx5M)")
    ap.add_argument("--pair-steps", type=int, default=2)
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-rho", type=float, nargs="+", default=[0.5, 0.8])
    ap.add_argument("--serve-scale", type=float, default=1.0)
    ap.add_argument("--serve-policies", nargs="+", default=["edf", "fifo"], choices=["edf", "fifo"])
    ap.add_argument("--serve-slice-ms", type=float, default=6.0,
                    help="device time per persistent launch of a serving batch (0: one launch)")
    ap.add_argument("--serve-long-depth", type=int, default=2,
                    help="launches of long (stepped) batches outstanding at once")
    ap.add_argument("--serve-lane-cells", type=int, default=16384,
                    help="work-item lane-cell target of serving searches (0 = planner)")
    ap.add_argument("--serve-long-ms", type=float, default=20.0,
                    help="estimated device time above which a request is long (keeps a slot for short ones)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="also run one device-to-device copy of MIB MiB (traffic calibration)")
    args = ap.parse_args(argv)
    KNOBS.update(lane_cells=args.lane_cells, waves=args.waves, lds_limit=args.lds_limit)
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only; --gpus {args.gpus} is not supported "
              "(the search shards by database range across GPUs with one score gather, "
              "which is designed but not run here)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2412_08308_amd as swdb
    import synth

    torch.cuda.set_device(0)
    w = synth.workload("q567_vs_200k", scale=args.scale)
    gdb = swdb.Database.from_host(w.db)
    q = torch.from_numpy(w.queries[0]).cuda()
    cells = len(w.queries[0]) * w.db.total
    ev = HipEvents()
    isa = isa_counts()

    tuning = None
    if not args.no_tune:
        from paper_2412_08308_amd import autotune
        bins = [200, 400, 567, 800, 1200, 2000, 3500, 6000]
        tuning = autotune.tuned(gdb, bins, w.matrix, w.gap_open, w.gap_extend, cache_path=None)
    elif args.mode == "tuned":
        raise SystemExit("--mode tuned needs the autotuner")
    main_run = timed_search(gdb, [q], w.matrix, w.gap_open, w.gap_extend, args.mode, args.steps, args.warmup, ev)
    tuned_run = None
    if tuning is not None and args.mode != "tuned":
        tuned_run = timed_search(gdb, [q], w.matrix, w.gap_open, w.gap_extend, "tuned", args.steps,
                                 args.warmup, ev)
    i32_run = main_run if args.no_i32 else timed_search(gdb, [q], w.matrix, w.gap_open, w.gap_extend, "i32",
                                                         args.steps, args.warmup, ev)
    if args.copy_probe:
        src = torch.empty(args.copy_probe << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    # parity of every config at its stated size: the stored oracle digests of
    # every score (tests/golden/make_digests.py), plus the oracle run of the
    # CPU-baseline leg compared with the same GPU outputs subject by subject
    parity = None
    outs = {args.mode: main_run["out"].cpu().numpy(), "i32": i32_run["out"].cpu().numpy()}
    if tuned_run is not None:
        outs["tuned"] = tuned_run["out"].cpu().numpy()
    if not args.no_check and args.scale == 1.0:
        parity = {"q567_vs_200k": {m: digest_parity("q567_vs_200k", [o]) for m, o in outs.items()}}

    traffic = traffic_bytes(args.mode)
    variant = main_run["plan"]["variant"]
    key, kname = VARIANTS[variant]
    ops = isa[key]["valu_per_cell"]
    kernel_s = main_run["kernel_ms"] / 1e3
    achieved = cells * ops / kernel_s / 1e12
    i32_key = VARIANTS[i32_run["plan"]["variant"]][0]
    gcups = cells / (main_run["wall_ms"] / 1e3) / 1e9

    batched = None
    if not args.no_batch:
        w3 = synth.workload("20q_vs_200k", scale=args.scale)
        qs = [torch.from_numpy(x).cuda() for x in w3.queries]
        bcells = sum(len(x) for x in w3.queries) * w.db.total
        batched = {"workload": "20 queries 144-5478 vs the same 200,000 subjects, one persistent launch "
                               "per schedule", "cells": bcells}
        bpar = {}
        legs = [("auto", "auto", None), ("i32", "i32", None)]
        if tuning is not None:
            # the batch tuned as a unit (sw_autotune_batch: one schedule timed on
            # this batch), and the per-length tables of the single-query tuner
            t0 = time.perf_counter()
            bopt, brec = gdb.autotune_batch(qs, w3.matrix, w3.gap_open, w3.gap_extend)
            batched["tune_s"] = round(time.perf_counter() - t0, 1)
            batched["tuned_schedule"] = {k: brec[k] for k in ("mode", "waves", "lane_cells", "strict_groups")}
            legs += [("tuned", {0: "auto", 1: "i32", 2: "i16"}[bopt.mode],
                      {"waves": bopt.waves, "lane_cells": bopt.lane_cells, "strict_groups": bopt.strict_groups}),
                     ("tuned_bins", "tuned", None)]
        for bm, bmode, extra in legs:
            b = timed_search(gdb, qs, w3.matrix, w3.gap_open, w3.gap_extend, bmode, args.batch_steps, 1, ev,
                             batch=True, extra=extra)
            batched[bm] = {"gcups": round(bcells / (b["wall_ms"] / 1e3) / 1e9, 1),
                           "ms_per_batch": round(b["wall_ms"], 2), "search_kernel_ms": round(b["kernel_ms"], 2),
                           "flagged": b["flagged"]}
            if args.scale == 1.0:
                bpar[bm] = digest_parity("20q_vs_200k", b["out"].cpu().numpy())
        g = timed_graph(gdb, qs, w3.matrix, w3.gap_open, w3.gap_extend, args.batch_steps, ev)
        batched["graph"] = {"gcups": round(bcells / (g["wall_ms"] / 1e3) / 1e9, 1),
                            "ms_per_batch": round(g["wall_ms"], 2), "replay_ms": round(g["replay_ms"], 2)}
        if args.scale == 1.0:
            bpar["graph"] = digest_parity("20q_vs_200k", g["out"])
        batched["gcups"] = max(v["gcups"] for k, v in batched.items() if isinstance(v, dict) and "gcups" in v)
        if parity is not None and bpar:
            parity["20q_vs_200k"] = bpar

    traceback = None if args.no_align else alignments(args, w, main_run["out"])
    overflow = None if args.no_planted else planted(args, ev)
    pair = None if args.no_pair else pairwise(args, ev)
    latency = None if args.no_serve else serving(args, gcups, args.mode)
    cpu = None
    if not args.no_cpu:
        cpu, sel, exp = cpu_baseline(w, args.cpu_seconds)
        if parity is not None:
            parity["q567_vs_200k"]["cpu_oracle_run"] = {
                "subjects": int(len(sel)),
                "mismatches": {m: int(np.sum(o[sel] != exp)) for m, o in outs.items()}}
    if parity is not None and overflow is not None and overflow.get("parity"):
        parity["q8000_planted_vs_200k"] = overflow["parity"]
    if parity is not None and latency is not None and latency.get("parity"):
        parity["serve_500k"] = latency["parity"]

    rec = {
        "metric": "GCUPS per MI355X (int32 vs packed-int16+batched), bit-exact; p50/p99 query latency",
        "value": round(gcups, 1),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_run["wall_ms"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i16x2+i32" if args.mode != "i32" else "i32",
        "data": "synthetic",
        "config": {"workload": "query 567 vs 200,000 subjects, log-normal lengths median 300 "
                               f"(sum {w.db.total} residues), BLOSUM62-style, gaps 10/2",
                   "mode": args.mode, "cells": cells},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_VALU_TOPS, 3),
                     "unit": "TOP/s", "frac": round(achieved / PEAK_VALU_TOPS, 4),
                     "traffic": (None if traffic is None else traffic["bytes"]),
                     "traffic_detail": traffic,
                     "algorithmic_bytes": int(w.db.total + len(w.queries[0]) + 4 * w.db.nseq),
                     "kernel_fingerprint": kernel_fingerprint(),
                     "kernel": kname,
                     "isa_valu_per_cell": ops, "search_kernel_ms": round(main_run["kernel_ms"], 3),
                     "isa_peak_gcups": round(PEAK_VALU_TOPS * 1e3 / ops, 1),
                     "paper_model": paper_model(cells, kernel_s, variant)},
        "int32": {"gcups": round(cells / (i32_run["wall_ms"] / 1e3) / 1e9, 1),
                  "ms_per_step": round(i32_run["wall_ms"], 3),
                  "search_kernel_ms": round(i32_run["kernel_ms"], 3),
                  "isa_valu_per_cell": isa[i32_key]["valu_per_cell"],
                  "roofline_frac": round(cells * isa[i32_key]["valu_per_cell"] / (i32_run["kernel_ms"] / 1e3)
                                         / 1e12 / PEAK_VALU_TOPS, 4)},
        "i16": {"rescore_ms": round(main_run["rescore_ms"], 3), "flagged": main_run["flagged"]},
        "tuned": None if tuned_run is None else {
            "gcups": round(cells / (tuned_run["wall_ms"] / 1e3) / 1e9, 1),
            "search_kernel_ms": round(tuned_run["kernel_ms"], 3),
            "schedules": [{k: e[k] for k in ("qlen", "mode", "waves", "lane_cells", "gcups")} for e in tuning]},
        "overflow": overflow,
        "batched": batched,
        "pairwise": pair,
        "traceback": traceback,
        "latency": latency,
        "parity": parity,
        "plan": {k: main_run["plan"][k] for k in ("lane_cells", "items", "launches", "grid", "rows")},
        "knobs": {k: v for k, v in KNOBS.items() if v},
        "cpu_baseline": cpu,
    }
    gdb.release()
    print(json.dumps(rec))
    return 0


if __name__ == "__main__":
    sys.exit(main())
