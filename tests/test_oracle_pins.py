"""Pins of the CPU oracle against the mathematics (no GPU).

The oracle evaluates the paper's Section 2.2 recurrence (H with zero floor,
affine-gap E along the subject and F along the query, zero borders, S = max H).
These tests tie it to values obtained by other routes, chosen so that a
plausible slip anywhere in the recurrence (dropped term, sign, transposed
operand, wrong neighbour, wrong gap convention, missing floor, wrong maximum)
fails at least one of them; ``test_mutants_are_caught`` plants each such slip
in a rebuilt oracle and checks exactly that.
"""
import os
import tempfile

import numpy as np
import pytest

import oracle
import pinlib
import synth


def _rand_case(rng, alpha, mmax=5, nmax=5, lo=-5, hi=5, go_ge="ge_le_go"):
    m = int(rng.integers(0, mmax + 1))
    n = int(rng.integers(0, nmax + 1))
    q = rng.integers(0, alpha, size=m).tolist()
    d = rng.integers(0, alpha, size=n).tolist()
    sm = rng.integers(lo, hi + 1, size=(32, 32)).astype(np.int32)   # asymmetric
    ge = int(rng.integers(0, 4))
    if go_ge == "ge_le_go":
        go = ge + int(rng.integers(0, 5))
    else:
        go = int(rng.integers(0, ge + 1))
    return q, d, sm, go, ge


# ------------------------------------------------------------------ brute force

@pytest.mark.parametrize("alpha", [2, 3, 4])
def test_bruteforce_random(alpha):
    rng = np.random.default_rng(100 + alpha)
    for _ in range(120):
        q, d, sm, go, ge = _rand_case(rng, alpha)
        assert oracle.score(q, d, sm, go, ge) == pinlib.brute_force(q, d, sm, go, ge), (q, d, go, ge)


def test_bruteforce_open_cheaper_than_extend():
    # Go < Ge: the E/F equations let a gap re-open at cost Go at any residue.
    rng = np.random.default_rng(7)
    for _ in range(150):
        q, d, sm, go, ge = _rand_case(rng, 3, go_ge="go_le_ge")
        assert oracle.score(q, d, sm, go, ge) == pinlib.brute_force(q, d, sm, go, ge)


def test_python_form_agrees():
    rng = np.random.default_rng(3)
    for _ in range(100):
        q, d, sm, go, ge = _rand_case(rng, 4, 9, 9)
        assert oracle.score(q, d, sm, go, ge) == oracle.score_py(q, d, sm, go, ge)


# ------------------------------------------------------------------ hand-worked

@pytest.mark.parametrize("row", pinlib.hand_examples(), ids=lambda r: r["name"])
def test_hand_examples(row):
    sm = synth.dna_matrix(row["match"], row["mismatch"])
    assert oracle.score(row["q"], row["d"], sm, row["go"], row["ge"]) == row["expected"]


def test_single_residue_query():
    rng = np.random.default_rng(5)
    for _ in range(50):
        sm = rng.integers(-6, 7, size=(32, 32)).astype(np.int32)
        q = [int(rng.integers(0, 32))]
        d = rng.integers(0, 32, size=int(rng.integers(1, 30))).tolist()
        expect = max(0, max(int(sm[q[0], x]) for x in d))
        assert oracle.score(q, d, sm, int(rng.integers(0, 9)), int(rng.integers(0, 4))) == expect


def test_empty_inputs():
    sm = synth.blosum_style_matrix()
    assert oracle.score([], [1, 2, 3], sm, 10, 2) == 0
    assert oracle.score([1, 2, 3], [], sm, 10, 2) == 0
    assert oracle.score([], [], sm, 10, 2) == 0


# ------------------------------------------------------------------ special cases

def test_linear_gap_is_textbook_sw():
    rng = np.random.default_rng(11)
    for _ in range(60):
        m, n = int(rng.integers(1, 25)), int(rng.integers(1, 25))
        q = rng.integers(0, 6, size=m).tolist()
        d = rng.integers(0, 6, size=n).tolist()
        sm = rng.integers(-4, 6, size=(32, 32)).astype(np.int32)
        g = int(rng.integers(0, 7))
        assert oracle.score(q, d, sm, g, g) == pinlib.linear_gap_sw(q, d, sm, g)


def test_prohibitive_gaps_is_ungapped_kadane():
    rng = np.random.default_rng(12)
    big = 10 ** 6
    for _ in range(60):
        m, n = int(rng.integers(1, 40)), int(rng.integers(1, 40))
        q = rng.integers(0, 5, size=m).tolist()
        d = rng.integers(0, 5, size=n).tolist()
        sm = rng.integers(-5, 6, size=(32, 32)).astype(np.int32)
        assert oracle.score(q, d, sm, big, big) == pinlib.ungapped_kadane(q, d, sm)


def test_longest_common_substring():
    rng = np.random.default_rng(13)
    big = 10 ** 6
    sm = np.full((32, 32), -big, dtype=np.int32)
    np.fill_diagonal(sm, 1)
    for _ in range(80):
        m, n = int(rng.integers(0, 30)), int(rng.integers(0, 30))
        q = rng.integers(0, 3, size=m).tolist()
        d = rng.integers(0, 3, size=n).tolist()
        assert oracle.score(q, d, sm, big, big) == pinlib.longest_common_substring(q, d)


def test_self_alignment_is_diagonal_sum():
    sm = synth.blosum_style_matrix()
    assert pinlib.diagonal_dominant(sm, range(20))
    rng = np.random.default_rng(14)
    for _ in range(20):
        q = synth.residues(rng, int(rng.integers(1, 400)))
        assert oracle.score(q, q, sm, 10, 2) == pinlib.diagonal_sum(q, sm)


# ------------------------------------------------------------------ invariants

def test_invariants():
    rng = np.random.default_rng(15)
    sm = synth.blosum_style_matrix()
    for _ in range(40):
        q = synth.residues(rng, int(rng.integers(1, 120)))
        d = synth.residues(rng, int(rng.integers(1, 120)))
        go, ge = int(rng.integers(0, 14)), int(rng.integers(0, 4))
        s = oracle.score(q, d, sm, go, ge)
        assert 0 <= s <= min(len(q), len(d)) * int(sm.max())
        # some positive pair exists <=> positive score
        pos = any(sm[a, b] > 0 for a in set(q.tolist()) for b in set(d.tolist()))
        assert (s > 0) == pos
        # swap symmetry under the transposed matrix
        assert oracle.score(d, q, sm.T.copy(), go, ge) == s
        # reversal of both sequences
        assert oracle.score(q[::-1], d[::-1], sm, go, ge) == s
        # non-increasing in each penalty
        assert oracle.score(q, d, sm, go + 3, ge) <= s
        assert oracle.score(q, d, sm, go, ge + 1) <= s
        # extending the subject cannot lower the score
        ext = np.concatenate([d, synth.residues(rng, 7)])
        assert oracle.score(q, ext, sm, go, ge) >= s
        assert oracle.score(q, np.concatenate([synth.residues(rng, 5), d]), sm, go, ge) >= s


def test_asymmetric_matrix_swap():
    rng = np.random.default_rng(16)
    for _ in range(40):
        sm = rng.integers(-5, 6, size=(32, 32)).astype(np.int32)
        q = rng.integers(0, 8, size=int(rng.integers(1, 30)))
        d = rng.integers(0, 8, size=int(rng.integers(1, 30)))
        go, ge = int(rng.integers(0, 8)), int(rng.integers(0, 4))
        assert oracle.score(q, d, sm, go, ge) == oracle.score(d, q, sm.T.copy(), go, ge)


# ------------------------------------------------------------------ search driver

def test_threaded_search_matches_pairs():
    rng = np.random.default_rng(17)
    sm = synth.blosum_style_matrix()
    q = synth.residues(rng, 50)
    seqs = [synth.residues(rng, int(n)) for n in rng.integers(0, 90, size=300)]
    db = synth.Database.from_list(seqs)
    full = oracle.search_db(q, db, sm, 10, 2, threads=4)
    ref = np.array([oracle.score(q, s, sm, 10, 2) for s in seqs])
    assert np.array_equal(full, ref)
    ids = rng.choice(len(seqs), size=40, replace=False)
    assert np.array_equal(oracle.search_db(q, db, sm, 10, 2, ids=ids, threads=3), ref[ids])
    assert len(oracle.search_db(q, db, sm, 10, 2, ids=[])) == 0


# ------------------------------------------------------------------ mutants

def _pin_battery(lib) -> bool:
    """True when every pin passes for the oracle in ``lib``."""
    try:
        for row in pinlib.hand_examples():
            sm = synth.dna_matrix(row["match"], row["mismatch"])
            if oracle.score(row["q"], row["d"], sm, row["go"], row["ge"], lib=lib) != row["expected"]:
                return False
        rng = np.random.default_rng(21)
        for _ in range(60):
            q, d, sm, go, ge = _rand_case(rng, 3)
            if oracle.score(q, d, sm, go, ge, lib=lib) != pinlib.brute_force(q, d, sm, go, ge):
                return False
        sm = synth.blosum_style_matrix()
        for _ in range(5):
            q = synth.residues(rng, 60)
            if oracle.score(q, q, sm, 10, 2, lib=lib) != pinlib.diagonal_sum(q, sm):
                return False
        return True
    except Exception:
        return False


def test_pin_battery_passes_on_oracle():
    assert _pin_battery(oracle.load())


@pytest.mark.parametrize("mutant", [1, 2, 3, 4, 5, 6, 7])
def test_mutants_are_caught(mutant):
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, f"liboracle_m{mutant}.so")
        oracle.build(path, mutant=mutant)
        lib = oracle.load(path)
        assert not _pin_battery(lib), f"planted mistake {mutant} went unnoticed"
