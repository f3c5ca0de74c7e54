"""Autotuned schedules with a persistent cache.

``tuned(db, qlens, matrix, go, ge, cache_path)`` returns the per-length
schedules for a resident database: taken from the JSON cache when an entry
matches this device, library build, database (sorted-length signature) and
scoring, otherwise measured by ``sw_autotune`` on the device and stored.  The
schedules are installed on the handle, so searches with mode ``"tuned"`` use
them.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Optional, Sequence

import numpy as np

from . import Database, version

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "swdb", "autotune.json")


def cache_key(db: Database, matrix, gap_open: int, gap_extend: int, device_name: str) -> str:
    h = hashlib.sha1()
    h.update(np.ascontiguousarray(db.sorted_lengths()).tobytes())
    h.update(np.ascontiguousarray(np.asarray(matrix, dtype=np.int32)).tobytes())
    h.update(f"{gap_open}/{gap_extend}/{device_name}/{version()}".encode())
    return h.hexdigest()


def _device_name() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{p.gcnArchName}/{p.multi_processor_count}cu"


def tuned(db: Database, qlens: Sequence[int], matrix, gap_open: int, gap_extend: int,
          cache_path: Optional[str] = DEFAULT_CACHE, stream=None):
    qlens = sorted(int(m) for m in qlens)
    key = cache_key(db, matrix, gap_open, gap_extend, _device_name())
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as fh:
                cache = json.load(fh)
        except (OSError, ValueError):
            cache = {}
    hit = cache.get(key)
    if hit and [e["qlen"] for e in hit] == qlens:
        db.set_tuning(hit)
        return hit
    entries = db.autotune(qlens, matrix, gap_open, gap_extend, stream=stream)
    if cache_path:
        cache[key] = entries
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1)
        os.replace(tmp, cache_path)
    return entries
