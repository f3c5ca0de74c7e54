"""Seeded synthetic inputs for protein database search.

This module only draws inputs: sequences, lengths, a substitution matrix, gap
penalties and arrival times.  It performs none of the alignment arithmetic, so
both the CPU oracle (test infrastructure) and the GPU path may consume what it
produces without sharing any of the method's code.

The paper's workload (Section 4.1, protein database search) is 20 Swiss-Prot
queries of 144-5,478 residues against the Env. NR database scored with BLOSUM62
and gap penalties 10 (open) / 2 (extend).  Neither data set nor the BLOSUM62
table is available here, so every input is synthetic:

* residues are i.i.d. over the 20 amino acids (codes 0-19) at an approximate
  background composition (``BACKGROUND``; rounded illustrative values, not a
  published table);
* the scoring matrix is ``blosum_style_matrix()``: a seeded symmetric integer
  matrix with BLOSUM62's value range and sign structure (see its docstring);
  ``load_ncbi_matrix`` accepts a real NCBI-format matrix file when one exists;
* database lengths follow a clamped log-normal law (median 300).

All draws use numpy ``Generator(PCG64)`` streams spawned from one
``SeedSequence`` per workload, so every array is a pure function of
(workload, seed, scale).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

ALPHA = 32                      # residue codes 0..31; matrices are 32x32
AMINO = "ARNDCQEGHILKMFPSTWYV"  # codes 0..19
PAD_SCORE = -4                  # matrix entries for codes 20..31

# Approximate amino-acid background composition (order = AMINO).  Rounded,
# illustrative values of typical protein composition; normalised on use.
_BG_RAW = np.array([0.083, 0.055, 0.041, 0.055, 0.014, 0.039, 0.067, 0.071,
                    0.023, 0.059, 0.097, 0.058, 0.024, 0.039, 0.047, 0.066,
                    0.054, 0.011, 0.029, 0.069])
BACKGROUND = _BG_RAW / _BG_RAW.sum()

GAP_OPEN = 10     # protein search penalties of the paper's workload
GAP_EXTEND = 2


def _streams(seed: int, n: int) -> List[np.random.Generator]:
    return [np.random.Generator(np.random.PCG64(s))
            for s in np.random.SeedSequence(seed).spawn(n)]


# --------------------------------------------------------------------------- matrices

def blosum_style_matrix(seed: int = 62) -> np.ndarray:
    """A BLOSUM62-style 32x32 int32 substitution matrix (rows = query residue).

    BLOSUM62 itself is not available in this environment.  This stand-in is a
    seeded symmetric 20x20 integer matrix with BLOSUM62's shape:

    * diagonal entries in [4, 11], off-diagonal entries in [-4, 3];
    * ``2*SM[a,b] <= SM[a,a] + SM[b,b]`` for every pair (self-alignment of a
      gap-free sequence then scores its diagonal sum);
    * negative expected score under ``BACKGROUND`` (local alignments stay local);
    * codes 20..31 score ``PAD_SCORE`` against everything.

    Speed of the search does not depend on the values; only how often 16-bit
    lanes overflow does.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    vals = np.arange(-4, 4)
    probs = np.array([0.06, 0.16, 0.24, 0.22, 0.16, 0.09, 0.05, 0.02])
    while True:
        m = np.zeros((20, 20), dtype=np.int64)
        iu = np.triu_indices(20, 1)
        off = rng.choice(vals, size=len(iu[0]), p=probs / probs.sum())
        m[iu] = off
        m = m + m.T
        m[np.diag_indices(20)] = rng.integers(4, 12, size=20)
        d = np.diag(m)
        ok_pair = np.all(2 * m <= d[:, None] + d[None, :])
        expect = float(BACKGROUND @ m @ BACKGROUND)
        if ok_pair and expect < 0:
            break
    full = np.full((ALPHA, ALPHA), PAD_SCORE, dtype=np.int32)
    full[:20, :20] = m
    return full


def dna_matrix(match: int = 1, mismatch: int = -3) -> np.ndarray:
    """32x32 matrix scoring codes 0..3 (A, C, G, T) as match/mismatch.

    The paper's pairwise-DNA workload scores +1 / -3 with gap penalties 5 / 2
    (Section 4.1); this matrix is used for small hand-checkable examples.
    """
    full = np.full((ALPHA, ALPHA), mismatch, dtype=np.int32)
    for a in range(ALPHA):
        full[a, a] = match
    return full


def load_ncbi_matrix(text: str, alphabet: str = AMINO) -> np.ndarray:
    """Parse an NCBI-format substitution matrix into the 32x32 ABI layout.

    Letters of ``alphabet`` map to codes 0..len-1; letters of the file that are
    not in ``alphabet`` are ignored; unlisted codes score ``PAD_SCORE``.
    """
    rows = [ln.split() for ln in text.splitlines()
            if ln.strip() and not ln.lstrip().startswith("#")]
    cols = rows[0]
    out = np.full((ALPHA, ALPHA), PAD_SCORE, dtype=np.int32)
    code = {c: i for i, c in enumerate(alphabet)}
    for r in rows[1:]:
        a = r[0]
        if a not in code:
            continue
        for c, v in zip(cols, r[1:]):
            if c in code:
                out[code[a], code[c]] = int(v)
    return out


# --------------------------------------------------------------------------- sequences

def residues(rng: np.random.Generator, n: int, freqs: np.ndarray = BACKGROUND) -> np.ndarray:
    """``n`` i.i.d. residue codes drawn from ``freqs`` (uint8)."""
    return rng.choice(len(freqs), size=int(n), p=freqs).astype(np.uint8)


def lognormal_lengths(rng: np.random.Generator, n: int, median: float, sigma: float,
                      lo: int, hi: int) -> np.ndarray:
    x = np.exp(math.log(median) + sigma * rng.standard_normal(int(n)))
    return np.clip(np.rint(x), lo, hi).astype(np.int32)


def mutate(rng: np.random.Generator, src: np.ndarray, identity: float,
           indel_rate: float = 0.02, indel_mean: float = 3.0, freqs: np.ndarray = BACKGROUND) -> np.ndarray:
    """A near-homolog of ``src``: each position kept with probability
    ``identity`` (else redrawn from ``freqs``), plus indel events at
    ``indel_rate`` per position, half deletions and half insertions, with
    geometric lengths of mean ``indel_mean``."""
    src = np.asarray(src, dtype=np.uint8)
    n = len(src)
    out = src.copy()
    sub = rng.random(n) >= identity
    out[sub] = residues(rng, int(sub.sum()), freqs)
    ev = np.nonzero(rng.random(n) < indel_rate)[0]
    if len(ev) == 0:
        return out
    pieces = []
    pos = 0
    for e in ev:
        if e < pos:
            continue
        pieces.append(out[pos:e])
        L = int(rng.geometric(1.0 / indel_mean))
        if rng.random() < 0.5:          # deletion of L source positions
            pos = min(n, e + L)
        else:                           # insertion of L random residues before e
            pieces.append(residues(rng, L, freqs))
            pos = e
    pieces.append(out[pos:])
    return np.concatenate(pieces).astype(np.uint8)


@dataclass
class Database:
    """Concatenated subjects: ``residues[offsets[i]:offsets[i]+lengths[i]]``."""
    residues: np.ndarray   # uint8 [sum n]
    offsets: np.ndarray    # int64 [nseq]
    lengths: np.ndarray    # int32 [nseq]

    @property
    def nseq(self) -> int:
        return int(len(self.lengths))

    @property
    def total(self) -> int:
        return int(self.lengths.sum())

    def subject(self, i: int) -> np.ndarray:
        o = int(self.offsets[i])
        return self.residues[o:o + int(self.lengths[i])]

    @staticmethod
    def from_list(seqs: Sequence[np.ndarray]) -> "Database":
        lens = np.array([len(s) for s in seqs], dtype=np.int32)
        offs = np.zeros(len(seqs), dtype=np.int64)
        if len(seqs) > 1:
            offs[1:] = np.cumsum(lens[:-1], dtype=np.int64)
        res = (np.concatenate([np.asarray(s, np.uint8) for s in seqs])
               if len(seqs) and lens.sum() else np.zeros(0, np.uint8))
        return Database(res.astype(np.uint8), offs, lens)


def make_db(rng: np.random.Generator, lengths: np.ndarray) -> Database:
    lengths = np.asarray(lengths, dtype=np.int32)
    offs = np.zeros(len(lengths), dtype=np.int64)
    if len(lengths) > 1:
        offs[1:] = np.cumsum(lengths[:-1], dtype=np.int64)
    return Database(residues(rng, int(lengths.sum())), offs, lengths)


# --------------------------------------------------------------------------- configs

@dataclass
class Workload:
    name: str
    queries: List[np.ndarray]
    db: Database
    matrix: np.ndarray
    gap_open: int = GAP_OPEN
    gap_extend: int = GAP_EXTEND
    note: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        return int(sum(len(q) for q in self.queries)) * self.db.total


def c3_query_lengths(nq: int = 20, lo: int = 144, hi: int = 5478) -> List[int]:
    """Query lengths spread log-uniformly (geometrically) over [lo, hi]."""
    if nq == 1:
        return [lo]
    return [int(round(lo * (hi / lo) ** (k / (nq - 1)))) for k in range(nq)]


# Workload names -> internal stream index (the index only seeds the streams).
_WORKLOADS = {"q64_vs_2k": 0, "q567_vs_200k": 1, "20q_vs_200k": 2, "q8000_planted_vs_200k": 3,
              "serve_500k": 4}


def workload(name: str, seed: int = 0, scale: float = 1.0) -> Workload:
    """The five synthetic workloads.

    q64_vs_2k:     query 64 vs 2,000 subjects, lengths uniform 32..512 (parity).
    q567_vs_200k:  query 567 vs 200,000 subjects, log-normal lengths (median
                   300, sigma 0.668, clamped 10..35,000; about 75M residues).
    20q_vs_200k:   20 queries, lengths geometric over 144..5,478, against the
                   200,000-subject database.
    q8000_planted_vs_200k: that database with 0.5% subjects resampled
                   log-uniform 10,000..35,000 and 1% replaced by near-homologs
                   (30-90% identity, with indels) of a long query (8,000
                   residues), so that 16-bit lanes overflow.
    serve_500k:    500,000 subjects with the same length law (about 190M
                   residues); queries log-normal (median 350, sigma 0.75,
                   clamped 50..5,000).

    ``scale`` shrinks subject counts (for quick tests); lengths keep their law.
    """
    if name not in _WORKLOADS:
        raise ValueError(f"no workload {name!r}; known: {sorted(_WORKLOADS)}")
    return _build(_WORKLOADS[name], seed, scale)


def _build(k: int, seed: int, scale: float) -> Workload:
    sm = blosum_style_matrix()
    if k == 0:
        r_len, r_res, r_q = _streams(seed, 3)
        n = max(1, int(round(2000 * scale)))
        lens = r_len.integers(32, 513, size=n).astype(np.int32)
        db = make_db(r_res, lens)
        return Workload("q64_vs_2k_uniform32-512", [residues(r_q, 64)], db, sm)
    if k in (1, 2, 3):
        r_len, r_res, r_q, r_q2, r_plant = _streams(seed + 1, 5)
        n = max(1, int(round(200_000 * scale)))
        lens = lognormal_lengths(r_len, n, 300, 0.668, 10, 35_000)
        db = make_db(r_res, lens)
        if k == 1:
            return Workload("q567_vs_200k_lognormal", [residues(r_q, 567)], db, sm)
        if k == 2:
            qs = [residues(r_q2, m) for m in c3_query_lengths()]
            return Workload("20q_144-5478_vs_200k", qs, db, sm)
        w = _plant(db, sm, r_plant, seed)
        w.extra["control_query"] = residues(r_q, 567)
        return w
    if k == 4:
        r_len, r_res, r_q = _streams(seed + 4, 3)
        n = max(1, int(round(500_000 * scale)))
        lens = lognormal_lengths(r_len, n, 300, 0.668, 10, 35_000)
        db = make_db(r_res, lens)
        qlens = lognormal_lengths(r_q, 64, 350, 0.75, 50, 5000)
        return Workload("serve_500k", [residues(r_q, int(m)) for m in qlens], db, sm)
    raise ValueError(f"no workload index {k}")


def _plant(db: Database, sm: np.ndarray, rng: np.random.Generator, seed: int,
           qlen: int = 8000) -> Workload:
    n = db.nseq
    query = residues(rng, qlen)
    seqs = [db.subject(i) for i in range(n)]
    idx = rng.permutation(n)
    n_long = max(1, n // 200)
    n_hom = max(1, n // 100)
    long_ids = idx[:n_long]
    hom_ids = idx[n_long:n_long + n_hom]
    for i in long_ids:
        L = int(round(math.exp(rng.uniform(math.log(10_000), math.log(35_000)))))
        seqs[i] = residues(rng, L)
    embedded = []
    for t, i in enumerate(hom_ids):
        ident = rng.uniform(0.30, 0.90)
        h = mutate(rng, query, ident)
        if t % 10 == 0 and n_long:
            # some homologs sit inside long random subjects
            host = int(long_ids[t // 10 % n_long])
            s = seqs[host]
            at = int(rng.integers(0, max(1, len(s) - len(h))))
            seqs[host] = np.concatenate([s[:at], h, s[at + len(h):]])[:35_000]
            embedded.append(host)
        seqs[i] = h[:35_000]
    out = Database.from_list(seqs)
    return Workload("planted_int16_overflow", [query], out, sm,
                    note="query 8,000 residues; 0.5% long subjects; 1% homologs",
                    extra={"long_ids": np.sort(long_ids), "hom_ids": np.sort(hom_ids),
                           "embedded_hosts": np.array(sorted(set(embedded)), dtype=np.int64)})


def planted(seed: int = 0, scale: float = 1.0, qlen: int = 8000) -> Workload:
    """The planted overflow workload with an explicit query length (the
    567-residue query is the zero-overflow control)."""
    r_len, r_res, r_q, r_q2, r_plant = _streams(seed + 1, 5)
    n = max(1, int(round(200_000 * scale)))
    lens = lognormal_lengths(r_len, n, 300, 0.668, 10, 35_000)
    db = make_db(r_res, lens)
    return _plant(db, blosum_style_matrix(), r_plant, seed, qlen)


# --------------------------------------------------------------------------- DNA pairs

DNA_FREQS = np.full(4, 0.25)              # codes 0..3 = A, C, G, T
DNA_MATCH, DNA_MISMATCH = 1, -3           # pairwise DNA scoring of the paper (Section 4.1)
DNA_GAP_OPEN, DNA_GAP_EXTEND = 5, 2
# (query, subject) lengths of the paper's five DNA alignments (its DNA table)
DNA_PAIR_SIZES = [(162_000, 172_000), (543_000, 536_000), (1_000_000, 1_000_000),
                  (3_000_000, 3_000_000), (7_000_000, 5_000_000)]


def dna_pair(m: int, n: int, seed: int = 0, identity: float = 0.8,
             indel_rate: float = 0.005) -> Tuple[np.ndarray, np.ndarray]:
    """Synthetic stand-in for one of the paper's DNA pairs: a random query of
    ``m`` bases and a subject of ``n`` bases made from a mutated copy of the
    query (``identity``, indels at ``indel_rate``), cut or extended with random
    bases to length ``n``, so that the best local alignment spans most of both."""
    rq, rs = _streams(seed + 7, 2)
    a = residues(rq, m, DNA_FREQS)
    b = mutate(rs, a[:min(m, n)], identity, indel_rate=indel_rate, freqs=DNA_FREQS)
    if len(b) >= n:
        b = b[:n]
    else:
        b = np.concatenate([b, residues(rs, n - len(b), DNA_FREQS)])
    return a, b.astype(np.uint8)


def poisson_arrivals(rng: np.random.Generator, rate: float, n: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson stream with the given rate."""
    return np.cumsum(rng.exponential(1.0 / rate, size=int(n)))


def serve_requests(n: int, seed: int = 77) -> List[np.ndarray]:
    """The serving workload's request stream: ``n`` queries with log-normal
    lengths (median 350, sigma 0.75, clamped 50..5,000), in arrival order.
    Lengths and residues come from separate streams, drawn in order, so the
    first k requests are the same for every n >= k (the first requests of the
    default stream carry stored oracle digests)."""
    r_len, r_res = _streams(seed, 2)
    out = []
    for _ in range(int(n)):
        m = int(lognormal_lengths(r_len, 1, 350, 0.75, 50, 5000)[0])
        out.append(residues(r_res, m))
    return out


def random_case(rng: np.random.Generator, m: int, n_list: Sequence[int], alpha: int = 20,
                matrix: Optional[np.ndarray] = None):
    """A query and a database with given subject lengths over ``alpha`` codes."""
    q = rng.integers(0, alpha, size=int(m)).astype(np.uint8)
    seqs = [rng.integers(0, alpha, size=int(n)).astype(np.uint8) for n in n_list]
    return q, Database.from_list(seqs)


def random_matrix(rng: np.random.Generator, lo: int = -5, hi: int = 5,
                  symmetric: bool = False) -> np.ndarray:
    """A random 32x32 int32 matrix with entries in [lo, hi] (asymmetric by default)."""
    m = rng.integers(lo, hi + 1, size=(ALPHA, ALPHA)).astype(np.int32)
    if symmetric:
        m = np.triu(m) + np.triu(m, 1).T
    return m
