"""CPU oracle for score-only Smith-Waterman/Gotoh database search.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The GPU library never imports or links
this package, and this package imports nothing from the GPU library.

``score`` / ``search`` call the plain C implementation in ``sw_oracle.c``
(literal recurrence of the paper's Section 2.2 equations for H, E and F, int64
arithmetic, borders initialised to 0, result = largest H).  ``align`` adds the
traceback (full matrices, stated tie-breaks), pinned in
``tests/test_oracle_align.py``.  ``score_py`` is the same recurrence in pure
Python for tiny cases.

Parity is pinned against the mathematics in ``tests/test_oracle_pins.py``:
brute-force enumeration of local alignments, hand-worked examples in
``tests/golden/``, textbook special cases (linear gaps, ungapped Kadane,
longest common substring), invariants, and self-alignment sums.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

from .build import LIB, build

_lib = None
_libs = {}


def load(path: Optional[str] = None):
    """Load (building first if needed) the oracle library at ``path``."""
    global _lib
    path = path or LIB
    if path in _libs:
        return _libs[path]
    if not os.path.exists(path):
        build(path)
    lib = ctypes.CDLL(path)
    lib.swo_score.restype = ctypes.c_int64
    lib.swo_score.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                              ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64]
    lib.swo_search.restype = ctypes.c_int
    lib.swo_search.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                               ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                               ctypes.c_void_p, ctypes.c_int]
    lib.swo_align.restype = ctypes.c_int64
    lib.swo_align.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                              ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                              ctypes.c_char_p, ctypes.c_int64]
    _libs[path] = lib
    if path == LIB:
        _lib = lib
    return lib


def _u8(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint8))


def _sm(sm) -> np.ndarray:
    sm = np.ascontiguousarray(np.asarray(sm, dtype=np.int32))
    if sm.shape != (32, 32):
        raise ValueError("substitution matrix must be 32x32")
    return sm


def score(q, d, sm, go: int, ge: int, lib=None) -> int:
    """Optimal local alignment score of query ``q`` against subject ``d``."""
    lib = lib or load()
    q, d, sm = _u8(q), _u8(d), _sm(sm)
    v = lib.swo_score(q.ctypes.data, len(q), d.ctypes.data, len(d), sm.ctypes.data,
                      int(go), int(ge))
    if v < 0:
        raise MemoryError("oracle allocation failed")
    return int(v)


def search(q, residues, offsets, lengths, sm, go: int, ge: int,
           ids: Optional[Sequence[int]] = None, threads: Optional[int] = None,
           lib=None) -> np.ndarray:
    """Scores (int64) of ``q`` against database subjects ``ids`` (default: all)."""
    lib = lib or load()
    q, res, sm = _u8(q), _u8(residues), _sm(sm)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    ln = np.ascontiguousarray(np.asarray(lengths, dtype=np.int32))
    if ids is None:
        idp, nids = None, len(ln)
    else:
        ida = np.ascontiguousarray(np.asarray(ids, dtype=np.int64))
        if len(ida) and (ida.min() < 0 or ida.max() >= len(ln)):
            raise IndexError("subject id out of range")
        idp, nids = ida.ctypes.data, len(ida)
    out = np.zeros(nids, dtype=np.int64)
    if nids == 0:
        return out
    nth = threads or os.cpu_count() or 1
    rc = lib.swo_search(q.ctypes.data, len(q), res.ctypes.data if len(res) else None,
                        off.ctypes.data, ln.ctypes.data, idp, nids, sm.ctypes.data,
                        int(go), int(ge), out.ctypes.data, int(nth))
    if rc != 0:
        raise RuntimeError("oracle search failed")
    return out


def search_db(q, db, sm, go: int, ge: int, ids=None, threads=None, lib=None) -> np.ndarray:
    """``search`` over a ``synth.Database``-like object."""
    return search(q, db.residues, db.offsets, db.lengths, sm, go, ge, ids, threads, lib)


def align(q, d, sm, go: int, ge: int, lib=None) -> dict:
    """Optimal local alignment with its traceback (``swo_align``): score,
    1-based inclusive begin/end positions in the query and the subject, and
    the operations ('M', 'I' = query residue against a gap, 'D' = subject
    residue against a gap) from begin to end.  Tie-breaks: end = first cell
    with H = S in column-major order; diagonal before E before F; a gap opens
    rather than extends when both give its value."""
    lib = lib or load()
    q, d, sm = _u8(q), _u8(d), _sm(sm)
    out = np.zeros(5, dtype=np.int64)
    cap = len(q) + len(d) + 1
    buf = ctypes.create_string_buffer(cap)
    n = lib.swo_align(q.ctypes.data, len(q), d.ctypes.data, len(d), sm.ctypes.data, int(go), int(ge),
                      out.ctypes.data, buf, cap)
    if n == -1:
        raise MemoryError("oracle alignment: out of memory")
    if n < 0:
        raise RuntimeError("oracle alignment: traceback left the matrix")
    return {"score": int(out[0]), "q_begin": int(out[1]), "s_begin": int(out[2]), "q_end": int(out[3]),
            "s_end": int(out[4]), "ops": buf.raw[:n].decode()}


def cigar(ops: str) -> str:
    """Run-length form of an operation string ("MMMID" -> "3M1I1D")."""
    out, k = [], 0
    while k < len(ops):
        r = k
        while r < len(ops) and ops[r] == ops[k]:
            r += 1
        out.append(f"{r - k}{ops[k]}")
        k = r
    return "".join(out)


def score_py(q, d, sm, go: int, ge: int) -> int:
    """Pure-Python form of the same recurrence (tiny inputs only)."""
    m, n = len(q), len(d)
    if m == 0 or n == 0:
        return 0
    Hp = [0] * (n + 1)
    Fp = [0] * (n + 1)
    S = 0
    for i in range(1, m + 1):
        Hc = [0] * (n + 1)
        Fc = [0] * (n + 1)
        El = 0
        for j in range(1, n + 1):
            E = max(Hc[j - 1] - go, El - ge)
            F = max(Hp[j] - go, Fp[j] - ge)
            H = max(0, Hp[j - 1] + int(sm[q[i - 1]][d[j - 1]]), E, F)
            Hc[j], Fc[j], El = H, F, E
            S = max(S, H)
        Hp, Fp = Hc, Fc
    return S
