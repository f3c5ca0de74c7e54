"""The stored oracle digests (tests/golden/oracle_digests.json, written by
tests/golden/make_digests.py from oracle/ and synth/ only) belong to this
oracle and these inputs (no GPU needed): the oracle source hash matches, every
workload has its rows and block digests, and one block of the 567-residue
search recomputed here by the oracle hashes to the stored value."""
import hashlib
import importlib.util
import json
import os

import numpy as np

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _mk():
    spec = importlib.util.spec_from_file_location("make_digests", os.path.join(HERE, "golden", "make_digests.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    return mk


def test_digests_match_this_oracle_and_cover_every_workload():
    mk = _mk()
    with open(mk.OUT) as fh:
        data = json.load(fh)
    assert data["oracle_source_sha256"] == mk.oracle_source_sha()
    w = data["workloads"]
    assert {"q567_vs_200k", "20q_vs_200k", "q8000_planted_vs_200k", "serve_500k"} <= set(w)
    assert len(w["20q_vs_200k"]["rows"]) == 20 and len(w["q8000_planted_vs_200k"]["rows"]) == 2
    assert len(w["serve_500k"]["rows"]) == mk.SERVE_REQUESTS
    for name, e in w.items():
        nblocks = -(-e["nseq"] // e["block"])
        for r in e["rows"]:
            assert len(r["blocks"]) == nblocks and len(r["sha256"]) == 64
    # the 16-bit overflow workload overflows; its control query does not
    assert w["q8000_planted_vs_200k"]["rows"][0]["max"] >= 32767 > w["q8000_planted_vs_200k"]["rows"][1]["max"]
    assert data["pairs"]["dna_162k_x_172k"]["score"] > 0


def test_one_block_recomputed_by_the_oracle():
    mk = _mk()
    with open(mk.OUT) as fh:
        e = json.load(fh)["workloads"]["q567_vs_200k"]
    db, qs, sm, go, ge = mk.workload_inputs("q567_vs_200k")
    assert mk.config_sha(db, qs, sm, go, ge) == e["config_sha256"]
    ids = np.arange(e["block"])
    s = oracle.search_db(qs[0], db, sm, go, ge, ids=ids).astype("<i4")
    assert hashlib.sha256(s.tobytes()).hexdigest()[:16] == e["rows"][0]["blocks"][0]
