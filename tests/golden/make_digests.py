#!/usr/bin/env python3
"""Write ``tests/golden/oracle_digests.json``: the CPU oracle's scores of the
full-size workloads, stored as SHA-256 digests.

This script calls only ``oracle/`` (the plain C recurrence of the paper's
Section 2.2) and ``synth/`` (the seeded input generators); nothing it stores
comes from the GPU library.  The GPU tests and the benchmark compare the GPU
scores against these digests at the workloads' stated sizes:

* ``q567_vs_200k``: one 567-residue query against 200,000 subjects;
* ``20q_vs_200k``: 20 queries of 144..5,478 residues against that database
  (the paper's Section 4.1 workload shape: 20 queries per search);
* ``q8000_planted_vs_200k``: the 16-bit overflow workload (8,000-residue query,
  long subjects and near-homologs planted) plus its 567-residue control query;
* ``serve_500k``: the first requests of the serving stream
  (``synth.serve_requests``) against the 500,000-subject serving database;
* ``pairs``: the score of the paper's smallest DNA pair size (162K x 172K,
  ``synth.dna_pair``), one plain oracle call.

Every query row is stored as the SHA-256 of its int32 little-endian scores in
the caller's subject order, with a 64-bit digest per block of 4,096 subjects
(so a mismatch can be localised and re-checked with the oracle one subject at a
time), plus its sum, maximum and positive count.  Each workload carries the
SHA-256 of its inputs (``config_sha256``) and the file the SHA-256 of the
oracle's source (``oracle_source_sha256``); consumers refuse stale entries.

Usage: python tests/golden/make_digests.py [workload ...] [--threads N]
(default: everything; entries already present are replaced).  Oracle time on
8 host cores: about 30 s (q567), 26 min (20q), 11 min (planted), 8 min
(serving requests), 3 min (the pair).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth   # noqa: E402

OUT = os.path.join(HERE, "oracle_digests.json")
BLOCK = 4096
SERVE_REQUESTS = 8
PAIR_SIZES = {"dna_162k_x_172k": 0}     # name -> index into synth.DNA_PAIR_SIZES


def oracle_source_sha() -> str:
    with open(os.path.join(ROOT, "oracle", "sw_oracle.c"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def config_sha(db, queries, sm, go, ge) -> str:
    """SHA-256 of every input of a workload (subjects, queries, matrix, gaps)."""
    h = hashlib.sha256()
    for a in (db.lengths.astype("<i4"), db.offsets.astype("<i8"), db.residues.astype(np.uint8),
              np.asarray(sm, dtype="<i4")):
        h.update(np.ascontiguousarray(a).tobytes())
    h.update(f"{int(go)},{int(ge)},{len(queries)}".encode())
    for q in queries:
        h.update(len(q).to_bytes(8, "little"))
        h.update(np.ascontiguousarray(q, dtype=np.uint8).tobytes())
    return h.hexdigest()


def row_digest(scores) -> dict:
    """Digests of one query row of int32 scores (caller's subject order)."""
    s = np.ascontiguousarray(np.asarray(scores, dtype=np.int64))
    if s.size and (s.min() < 0 or s.max() > np.iinfo(np.int32).max):
        raise ValueError("oracle score outside int32")
    b = s.astype("<i4")
    blocks = [hashlib.sha256(b[k:k + BLOCK].tobytes()).hexdigest()[:16] for k in range(0, len(b), BLOCK)]
    return {"sha256": hashlib.sha256(b.tobytes()).hexdigest(), "blocks": blocks,
            "sum": int(s.sum()), "max": int(s.max()) if s.size else 0, "positive": int(np.sum(s > 0))}


def workload_inputs(name: str):
    """(db, queries, matrix, go, ge) of a stored workload."""
    if name == "serve_500k":
        w = synth.workload("serve_500k")
        return w.db, synth.serve_requests(SERVE_REQUESTS), w.matrix, w.gap_open, w.gap_extend
    w = synth.workload(name)
    qs = list(w.queries)
    if name == "q8000_planted_vs_200k":
        qs.append(w.extra["control_query"])
    return w.db, qs, w.matrix, w.gap_open, w.gap_extend


def run_workload(name: str, threads: int) -> dict:
    db, qs, sm, go, ge = workload_inputs(name)
    rows = []
    for k, q in enumerate(qs):
        t0 = time.perf_counter()
        s = oracle.search_db(q, db, sm, go, ge, threads=threads)
        dt = time.perf_counter() - t0
        r = row_digest(s)
        r["qlen"] = int(len(q))
        rows.append(r)
        print(f"{name} query {k} ({len(q)} residues): {dt:.1f} s, max {r['max']}", flush=True)
    return {"nseq": db.nseq, "residues": db.total, "block": BLOCK,
            "config_sha256": config_sha(db, qs, sm, go, ge), "rows": rows}


def run_pair(name: str) -> dict:
    k = PAIR_SIZES[name]
    m, n = synth.DNA_PAIR_SIZES[k]
    a, b = synth.dna_pair(m, n, seed=k)
    sm = synth.dna_matrix(synth.DNA_MATCH, synth.DNA_MISMATCH)
    go, ge = synth.DNA_GAP_OPEN, synth.DNA_GAP_EXTEND
    t0 = time.perf_counter()
    s = oracle.score(a, b, sm, go, ge)
    print(f"{name}: score {s} in {time.perf_counter() - t0:.1f} s", flush=True)
    h = hashlib.sha256()
    for x in (a, b, sm.astype("<i4")):
        h.update(np.ascontiguousarray(x).tobytes())
    h.update(f"{go},{ge}".encode())
    return {"m": m, "n": n, "seed": k, "score": int(s), "config_sha256": h.hexdigest()}


def main(argv=None):
    names = ["q567_vs_200k", "q8000_planted_vs_200k", "serve_500k", "20q_vs_200k"]
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("what", nargs="*", default=names + list(PAIR_SIZES))
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args(argv)
    data = {"workloads": {}, "pairs": {}}
    if os.path.exists(OUT):
        with open(OUT) as fh:
            data = json.load(fh)
    src = oracle_source_sha()
    if data.get("oracle_source_sha256") not in (None, src):
        data = {"workloads": {}, "pairs": {}}       # another oracle: start over
    data["oracle_source_sha256"] = src
    data["generator"] = "tests/golden/make_digests.py"
    for what in args.what:
        if what in PAIR_SIZES:
            data["pairs"][what] = run_pair(what)
        else:
            data["workloads"][what] = run_workload(what, args.threads)
        with open(OUT + ".tmp", "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(OUT + ".tmp", OUT)
    return 0


if __name__ == "__main__":
    sys.exit(main())
