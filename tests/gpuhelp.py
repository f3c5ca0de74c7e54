"""Helpers for GPU tests: run the HIP path through the binding and the oracle
on the same seeded inputs."""
from __future__ import annotations

import sys

import numpy as np

import oracle
import synth


def have_gpu() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def announce(msg: str):
    """Name the case on stdout before a GPU step (flushed)."""
    sys.stdout.write(f"[gpu-case] {msg}\n")
    sys.stdout.flush()


def gpu_db(db):
    import paper_2412_08308_amd as swdb
    return swdb.Database.from_host(db)


def _opt(mode, kw):
    """Options for a mode name; a trailing "w" asks for 16-bit profile entries
    (the wide-profile kernel variants) where 8 bits would hold them."""
    import paper_2412_08308_amd as swdb
    if mode.endswith("w"):
        mode, kw = mode[:-1], dict(kw, wide_profile=1)
    return swdb.options(mode=mode, **kw)


def gpu_scores(gdb, q, sm, go, ge, mode="auto", **kw):
    import torch
    opt = _opt(mode, kw)
    qt = torch.from_numpy(np.ascontiguousarray(q, dtype=np.uint8)).cuda()
    out = gdb.search(qt, sm, go, ge, opt=opt)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.int64)


def gpu_batch(gdb, qs, sm, go, ge, mode="auto", **kw):
    import torch
    opt = _opt(mode, kw)
    qts = [torch.from_numpy(np.ascontiguousarray(q, dtype=np.uint8)).cuda() for q in qs]
    out = gdb.search_batch(qts, sm, go, ge, opt=opt)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.int64)


def oracle_scores(db, q, sm, go, ge, ids=None):
    return oracle.search_db(q, db, sm, go, ge, ids=ids)


def oracle_pair(a, b, sm, go, ge):
    return int(oracle.score(a, b, sm, go, ge))


def mismatch_report(got, exp, ids=None, limit=8):
    bad = np.nonzero(got != exp)[0]
    if len(bad) == 0:
        return ""
    rows = []
    for k in bad[:limit]:
        sid = int(ids[k]) if ids is not None else int(k)
        rows.append(f"subject {sid}: gpu {int(got[k])} oracle {int(exp[k])}")
    return f"{len(bad)} mismatches; " + "; ".join(rows)


def overflow_matrix(top: int = 127, low: int = -128):
    """Matrix for constructed 16-bit overflow cases: code 0 scores `top` with
    itself, every other code 1 with itself, everything else `low`; a sequence
    over codes {0, 1} placed in the query as a substring then scores its
    diagonal sum exactly (no residue can contribute more than its match)."""
    sm = np.full((32, 32), low, dtype=np.int32)
    sm[0, 0] = top
    for c in range(1, 32):
        sm[c, c] = 1
    return sm


def overflow_sequence(target: int, top: int = 127) -> np.ndarray:
    """Codes over {0, 1} whose diagonal sum under overflow_matrix(top) is target."""
    n0 = target // top
    n1 = target - top * n0
    return np.array([0] * n0 + [1] * n1, dtype=np.uint8)
