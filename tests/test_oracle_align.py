"""Pins of the oracle's alignment (traceback) against brute force and hand
examples (no GPU).

What is fixed independently of the oracle's matrices:
  * the score is the brute-force optimum over every local alignment;
  * the end is the first end cell, in column-major order (smallest subject
    position, then smallest query position), of any optimal alignment;
  * the operations consume exactly the reported query and subject ranges,
    begin and end with a residue pair, and score the optimum;
  * read backwards from the end, each operation is the greatest (M > D > I)
    that some optimal alignment with the same backward prefix uses there, and
    the alignment stops at the first point where an optimal alignment stops.
Hand examples (tests/golden/align_examples.txt) fix whole answers; planted
mistakes in the traceback must fail these pins.
"""
import os
import tempfile

import numpy as np
import pytest

import oracle
import synth
from pinlib import expand, optimal_alignments, ops_score

ORDER = {"M": 2, "D": 1, "I": 0}
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "align_examples.txt")


def _cases(n, seed):
    rng = np.random.default_rng(seed)
    for t in range(n):
        m, k = int(rng.integers(1, 6)), int(rng.integers(1, 6))
        alpha = int(rng.integers(2, 4))
        q = rng.integers(0, alpha, m).astype(np.uint8)
        d = rng.integers(0, alpha, k).astype(np.uint8)
        if t % 2:
            sm = synth.random_matrix(rng, -2, 2)
        else:
            sm = synth.dna_matrix(int(rng.integers(1, 3)), -int(rng.integers(0, 3)))
        yield q, d, sm, int(rng.integers(0, 3)), int(rng.integers(0, 3))


def _violations(lib, n=300, seed=3):
    """Pins broken by the oracle at ``lib`` on random tiny cases (list of names)."""
    bad = []
    for q, d, sm, go, ge in _cases(n, seed):
        best, opt = optimal_alignments(q, d, sm, go, ge)
        r = oracle.align(q, d, sm, go, ge, lib=lib)
        if r["score"] != best:
            bad.append("score")
            continue
        if best == 0:
            if r["ops"] or r["q_end"] or r["s_end"]:
                bad.append("empty")
            continue
        first_end = min((o[3], o[2]) for o in opt)           # (subject, query) end
        if (r["s_end"], r["q_end"]) != first_end:
            bad.append("end")
            continue
        s, i, j = ops_score(q, d, sm, go, ge, r["q_begin"], r["s_begin"], r["ops"])
        if (s, i, j) != (best, r["q_end"], r["s_end"]) or not (r["ops"][0] == r["ops"][-1] == "M"):
            bad.append("ops")
            continue
        here = [o for o in opt if (o[2], o[3]) == (r["q_end"], r["s_end"])]
        back = r["ops"][::-1]
        for k in range(len(back)):
            feas = [o[4][::-1][k] for o in here if o[4][::-1][:k] == back[:k] and len(o[4]) > k]
            if not feas or max(feas, key=ORDER.get) != back[k]:
                bad.append("order")
                break
        if any(o[4][::-1] == back[:len(o[4])] and len(o[4]) < len(back) for o in here):
            bad.append("stop")
    return bad


def test_alignment_pins_random():
    assert _violations(oracle.load(), n=400, seed=3) == []


def _golden():
    rows = []
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if not line:
            continue
        f = line.split()
        rows.append(dict(name=f[0], q=expand(f[1]), d=expand(f[2]), match=int(f[3]), mismatch=int(f[4]),
                         go=int(f[5]), ge=int(f[6]), score=int(f[7]), q_begin=int(f[8]), s_begin=int(f[9]),
                         q_end=int(f[10]), s_end=int(f[11]), cigar=f[12]))
    return rows


@pytest.mark.parametrize("ex", _golden(), ids=lambda e: e["name"])
def test_alignment_hand_examples(ex):
    sm = synth.dna_matrix(ex["match"], ex["mismatch"])
    r = oracle.align(np.array(ex["q"], np.uint8), np.array(ex["d"], np.uint8), sm, ex["go"], ex["ge"])
    got = (r["score"], r["q_begin"], r["s_begin"], r["q_end"], r["s_end"], oracle.cigar(r["ops"]))
    assert got == (ex["score"], ex["q_begin"], ex["s_begin"], ex["q_end"], ex["s_end"], ex["cigar"])


def _golden_fails(lib):
    for ex in _golden():
        sm = synth.dna_matrix(ex["match"], ex["mismatch"])
        r = oracle.align(np.array(ex["q"], np.uint8), np.array(ex["d"], np.uint8), sm, ex["go"], ex["ge"], lib=lib)
        if (r["score"], r["q_begin"], r["s_begin"], r["q_end"], r["s_end"], oracle.cigar(r["ops"])) != \
                (ex["score"], ex["q_begin"], ex["s_begin"], ex["q_end"], ex["s_end"], ex["cigar"]):
            return True
    return False


@pytest.mark.parametrize("mutant", [8, 9, 10, 11])
def test_traceback_mutants_are_caught(mutant):
    """Row-major end cell, gap before diagonal, extend before open, running on
    through H = 0: each planted slip fails the pins above."""
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, f"liboracle_m{mutant}.so")
        oracle.build(path, mutant=mutant)
        lib = oracle.load(path)
        try:
            caught = _golden_fails(lib) or bool(_violations(lib, n=300, seed=5))
        except RuntimeError:          # the slip walks the traceback off the matrix
            caught = True
        assert caught, f"planted mistake {mutant} went unnoticed"
