"""Independent checks that pin the CPU oracle to the mathematics.

None of these functions evaluates the Gotoh H/E/F recurrence.  Each is a
different route to a value the recurrence must reproduce:

* ``brute_force``: enumerate every local alignment explicitly (tiny inputs);
* ``linear_gap_sw``: the single-matrix Smith-Waterman of the 1981 paper
  (Go = Ge reduces Gotoh's recurrence to it);
* ``ungapped_kadane``: maximum-subarray (Kadane) over every diagonal, which is
  the local score when gaps can never pay;
* ``longest_common_substring``: by substring sets (match +1, mismatch and gaps
  prohibitive);
* ``diagonal_sum``: self-alignment score for matrices whose diagonal dominates.
"""
from __future__ import annotations

import os
from typing import Dict, List, Tuple

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def brute_force(q, d, sm, go: int, ge: int) -> int:
    """Best local alignment score by explicit enumeration.

    An alignment is a start cell and a sequence of operations: M (pair Q[i]
    with D[j], add SM), X (subject residue against a gap) or Y (query residue
    against a gap).  A gap operation costs ``ge`` when it continues a run of the
    same kind and ``go`` when it opens one; a run may also be re-opened at cost
    ``go`` (this only matters when go < ge).  Every prefix of every operation
    sequence from every start is a candidate; the empty alignment scores 0.
    """
    m, n = len(q), len(d)
    best = 0
    sm = np.asarray(sm)

    def dfs(i, j, prev, s):
        nonlocal best
        if s > best:
            best = s
        if i < m and j < n:
            dfs(i + 1, j + 1, "M", s + int(sm[q[i]][d[j]]))
        if j < n:
            if prev == "X":
                dfs(i, j + 1, "X", s - ge)
                if go < ge:
                    dfs(i, j + 1, "X", s - go)
            else:
                dfs(i, j + 1, "X", s - go)
        if i < m:
            if prev == "Y":
                dfs(i + 1, j, "Y", s - ge)
                if go < ge:
                    dfs(i + 1, j, "Y", s - go)
            else:
                dfs(i + 1, j, "Y", s - go)

    for a in range(m):
        for c in range(n):
            dfs(a, c, "", 0)
    return best


def linear_gap_sw(q, d, sm, g: int) -> int:
    """Smith-Waterman with a linear gap cost g per residue (single H matrix)."""
    m, n = len(q), len(d)
    H = np.zeros((m + 1, n + 1), dtype=np.int64)
    best = 0
    for i in range(1, m + 1):
        for j in range(1, n + 1):
            H[i, j] = max(0, H[i - 1, j - 1] + int(sm[q[i - 1]][d[j - 1]]),
                          H[i - 1, j] - g, H[i, j - 1] - g)
            best = max(best, int(H[i, j]))
    return best


def ungapped_kadane(q, d, sm) -> int:
    """max(0, best contiguous diagonal segment sum) via Kadane per diagonal."""
    m, n = len(q), len(d)
    best = 0
    for off in range(-(m - 1), n):
        run = 0
        for i in range(m):
            j = i + off
            if 0 <= j < n:
                run = max(0, run + int(sm[q[i]][d[j]]))
                best = max(best, run)
    return best


def longest_common_substring(q, d) -> int:
    qs, ds = bytes(bytearray(q)), bytes(bytearray(d))
    for L in range(min(len(qs), len(ds)), 0, -1):
        subs = {qs[i:i + L] for i in range(len(qs) - L + 1)}
        if any(ds[j:j + L] in subs for j in range(len(ds) - L + 1)):
            return L
    return 0


def diagonal_sum(q, sm) -> int:
    return int(sum(int(sm[a][a]) for a in q))


def diagonal_dominant(sm, codes) -> bool:
    """SM[a,a] > 0 and 2*SM[a,b] <= SM[a,a] + SM[b,b] over ``codes``."""
    sm = np.asarray(sm, dtype=np.int64)
    c = np.asarray(list(codes))
    sub = sm[np.ix_(c, c)]
    dg = np.diag(sub)
    return bool(np.all(dg > 0) and np.all(2 * sub <= dg[:, None] + dg[None, :]))


DNA = {"A": 0, "C": 1, "G": 2, "T": 3}


def expand(spec: str) -> List[int]:
    """'A10TTA10' -> codes of A*10 + T + T + A*10 (letter optionally followed
    by a repeat count)."""
    out: List[int] = []
    i = 0
    while i < len(spec):
        ch = spec[i]
        i += 1
        k = i
        while k < len(spec) and spec[k].isdigit():
            k += 1
        rep = int(spec[i:k]) if k > i else 1
        out.extend([DNA[ch]] * rep)
        i = k
    return out


def hand_examples() -> List[Dict]:
    """Rows of golden/hand_examples.txt."""
    rows = []
    with open(os.path.join(GOLDEN, "hand_examples.txt")) as fh:
        for ln in fh:
            ln = ln.strip()
            if not ln or ln.startswith("#"):
                continue
            name, qs, ds, ma, mi, go, ge, exp = ln.split()
            rows.append(dict(name=name, q=expand(qs), d=expand(ds), match=int(ma),
                             mismatch=int(mi), go=int(go), ge=int(ge), expected=int(exp)))
    return rows


def optimal_alignments(q, d, sm, go: int, ge: int):
    """Every local alignment reaching the best score, by explicit enumeration
    (tiny inputs only).  Returns (best, [(q_begin, s_begin, q_end, s_end,
    ops)]) with 1-based inclusive positions and ops over 'M' (a residue pair),
    'D' (a subject residue against a gap) and 'I' (a query residue against a
    gap); gap runs cost ``go`` for the first residue and ``ge`` for each
    further one (a run may be re-opened at ``go`` when go < ge).  Only
    alignments that begin and end with 'M' are listed: trimming a trailing or
    leading gap never lowers a score."""
    m, n = len(q), len(d)
    sm = np.asarray(sm)
    found = []

    def dfs(a, c, i, j, prev, s, ops):
        if ops and ops[-1] == "M":
            found.append((s, a + 1, c + 1, i, j, "".join(ops)))
        if i < m and j < n:
            ops.append("M")
            dfs(a, c, i + 1, j + 1, "M", s + int(sm[q[i]][d[j]]), ops)
            ops.pop()
        if not ops:
            return
        for op, di, dj in (("D", 0, 1), ("I", 1, 0)):
            if i + di > m or j + dj > n:
                continue
            costs = [ge] if prev == op else []
            if prev != op or go < ge:
                costs.append(go)
            for cst in set(costs):
                ops.append(op)
                dfs(a, c, i + di, j + dj, op, s - cst, ops)
                ops.pop()

    for a in range(m):
        for c in range(n):
            dfs(a, c, a, c, "", 0, [])
    best = max([f[0] for f in found] + [0])
    return best, sorted({f[1:] for f in found if f[0] == best and best > 0})


def ops_score(q, d, sm, go: int, ge: int, q_begin: int, s_begin: int, ops: str):
    """Score of an alignment given by its begin positions (1-based) and ops,
    and the (query, subject) positions it ends at; gap runs cost go + (L-1) ge."""
    sm = np.asarray(sm)
    i, j = q_begin - 1, s_begin - 1
    s, prev = 0, ""
    for op in ops:
        if op == "M":
            s += int(sm[q[i]][d[j]])
            i += 1
            j += 1
        else:
            s -= min(ge, go) if op == prev else go
            if op == "D":
                j += 1
            else:
                i += 1
        prev = op
    return s, i, j
