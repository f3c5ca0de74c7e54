"""Python binding of ``libswdb.so``: score-only Smith-Waterman / Gotoh protein
database search on MI355X (gfx950).

Every step of the search runs in the library's HIP kernels; this module only
marshals arguments through ctypes.  PyTorch supplies device memory (tensors)
and streams.  If the library is missing, every entry point raises
``SwdbError`` -- there is no CPU fallback.

Names mirror the C-ABI in ``include/swdb.h``:

* ``search`` -> ``sw_db_search`` (one-shot, blocking);
* ``Database`` -> ``sw_db_prepare_bytes`` / ``sw_db_prepare`` /
  ``sw_db_release`` (resident database in a torch-allocated layout tensor),
  with ``search`` -> ``sw_db_search_ex`` and ``search_batch`` ->
  ``sw_db_search_batch`` (asynchronous on the current stream), ``status`` ->
  ``sw_search_status``, and ``workspace_bytes`` / ``plan_info``.

Searches check their status (``sw_search_status``: a query residue code >= 32,
an incomplete exact rescore) before returning unless ``check=False`` is
passed; the check synchronises the stream.  ``check=False`` callers read
``Database.status`` themselves.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# SWDB_LIBRARY names another build of the library (e.g. a host-sanitized one)
LIB_PATH = os.environ.get("SWDB_LIBRARY") or os.path.join(HERE, "libswdb.so")

SW_OK = 0
MODE_AUTO, MODE_I32, MODE_I16, MODE_TUNED = 0, 1, 2, 3
MODES = {"auto": MODE_AUTO, "i32": MODE_I32, "i16": MODE_I16, "tuned": MODE_TUNED}
MAX_GAP = 32000


class SwdbError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str = ""):
        super().__init__(f"{where}: {detail or 'error'} (code {code})")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("lane_cells", ctypes.c_int32), ("max_lanes", ctypes.c_int32),
                ("lds_limit", ctypes.c_int32), ("grid_limit", ctypes.c_int32),
                ("wide_profile", ctypes.c_int32), ("pair_cols", ctypes.c_int32),
                ("pair_rows", ctypes.c_int32), ("align_block", ctypes.c_int32),
                ("slice_mcells", ctypes.c_int32), ("pair_mode", ctypes.c_int32),
                ("pair_sm_max", ctypes.c_int32), ("slice_begin", ctypes.c_int32),
                ("slice_count", ctypes.c_int32), ("pair_entry_bytes", ctypes.c_int32),
                ("strict_groups", ctypes.c_int32), ("pair_group_waves", ctypes.c_int32),
                ("ev_search_begin", ctypes.c_void_p), ("ev_search_end", ctypes.c_void_p),
                ("ev_rescore_end", ctypes.c_void_p)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("qlen", ctypes.c_int32), ("pad", ctypes.c_int32), ("gcups", ctypes.c_double),
                ("opt", Options)]

    def as_dict(self):
        return {"qlen": self.qlen, "gcups": self.gcups, "mode": self.opt.mode, "waves": self.opt.waves,
                "lane_cells": self.opt.lane_cells, "max_lanes": self.opt.max_lanes,
                "lds_limit": self.opt.lds_limit, "grid_limit": self.opt.grid_limit,
                "strict_groups": self.opt.strict_groups}

    @classmethod
    def from_dict(cls, d):
        e = cls()
        e.qlen, e.gcups = int(d["qlen"]), float(d.get("gcups", 0.0))
        e.opt = options(mode=int(d["mode"]), waves=d.get("waves", 0), lane_cells=d.get("lane_cells", 0),
                        max_lanes=d.get("max_lanes", 0), lds_limit=d.get("lds_limit", 0),
                        grid_limit=d.get("grid_limit", 0), strict_groups=d.get("strict_groups", 0))
        return e


class PlanStats(ctypes.Structure):
    _fields_ = [("cells", ctypes.c_int64), ("lane_cells", ctypes.c_int64),
                ("items", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("grid", ctypes.c_int64), ("slot_bytes", ctypes.c_int64),
                ("workspace", ctypes.c_int64), ("variant", ctypes.c_int32),
                ("rows", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PairStats(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32), ("lanes", ctypes.c_int32), ("cols", ctypes.c_int32),
                ("flow", ctypes.c_int32), ("bands", ctypes.c_int64),
                ("chunks", ctypes.c_int64), ("launches", ctypes.c_int64), ("est_ms", ctypes.c_double),
                ("workspace", ctypes.c_int64), ("groups", ctypes.c_int32), ("group_waves", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Status(ctypes.Structure):
    """``sw_status``: the status words of a search workspace."""
    _fields_ = [("bad_query", ctypes.c_int32), ("rescore_failed", ctypes.c_int32),
                ("flagged", ctypes.c_int32), ("bad_items", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Alignment(ctypes.Structure):
    _fields_ = [("score", ctypes.c_int32), ("q_begin", ctypes.c_int32), ("s_begin", ctypes.c_int32),
                ("q_end", ctypes.c_int32), ("s_end", ctypes.c_int32), ("n_ops", ctypes.c_int32)]


_lib = None


def lib():
    """The loaded ``libswdb.so`` (raises ``SwdbError`` when it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise SwdbError(-100, "load", f"{LIB_PATH} is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    L.sw_db_search.restype = ctypes.c_int
    L.sw_db_search.argtypes = [vp, i32, vp, vp, vp, i32, vp, i32, i32, vp, vp]
    L.sw_db_prepare.restype = ctypes.c_int
    L.sw_db_prepare.argtypes = [vp, vp, vp, i32, vp, sz, vp, ctypes.POINTER(vp)]
    L.sw_db_prepare_bytes.restype = sz
    L.sw_db_prepare_bytes.argtypes = [i64, i32, i32]
    L.sw_search_status.restype = ctypes.c_int
    L.sw_search_status.argtypes = [vp, vp, ctypes.POINTER(Status)]
    L.sw_search_status_async.restype = ctypes.c_int
    L.sw_search_status_async.argtypes = [vp, vp, vp]
    L.sw_status_code.restype = ctypes.c_int
    L.sw_status_code.argtypes = [ctypes.POINTER(Status)]
    L.sw_db_release.restype = ctypes.c_int
    L.sw_db_release.argtypes = [vp]
    L.sw_db_info.restype = ctypes.c_int
    L.sw_db_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.sw_workspace_bytes.restype = sz
    L.sw_workspace_bytes.argtypes = [vp, i32, vp, ctypes.POINTER(Options)]
    L.sw_plan_info.restype = ctypes.c_int
    L.sw_plan_info.argtypes = [vp, i32, vp, ctypes.POINTER(Options), ctypes.POINTER(PlanStats)]
    L.sw_pair_workspace_bytes.restype = sz
    L.sw_pair_workspace_bytes.argtypes = [i64, i64, ctypes.POINTER(Options)]
    L.sw_pair_plan.restype = ctypes.c_int
    L.sw_pair_plan.argtypes = [i64, i64, ctypes.POINTER(Options), i32, ctypes.POINTER(PairStats)]
    L.sw_pair_score.restype = ctypes.c_int
    L.sw_pair_score.argtypes = [vp, i64, vp, i64, vp, i32, i32, ctypes.POINTER(Options), vp, sz, vp, vp]
    L.sw_pair_score_static.restype = ctypes.c_int
    L.sw_pair_score_static.argtypes = [vp, i64, vp, i64, vp, i32, i32, ctypes.POINTER(Options), vp, vp]
    L.sw_align_workspace_bytes.restype = sz
    L.sw_align_workspace_bytes.argtypes = [i64, i64, ctypes.POINTER(Options)]
    L.sw_align_pair.restype = ctypes.c_int
    L.sw_align_pair.argtypes = [vp, i64, vp, i64, vp, i32, i32, ctypes.POINTER(Options), vp, sz, vp, vp, vp]
    L.sw_select_variant.restype = i32
    L.sw_select_variant.argtypes = [vp, i32, ctypes.POINTER(Options)]
    L.sw_db_search_ex.restype = ctypes.c_int
    L.sw_db_search_ex.argtypes = [vp, vp, i32, vp, i32, i32, ctypes.POINTER(Options), vp, sz, vp, vp]
    L.sw_db_search_batch.restype = ctypes.c_int
    L.sw_db_search_batch.argtypes = [vp, vp, vp, vp, i32, vp, i32, i32, ctypes.POINTER(Options),
                                     vp, sz, vp, vp]
    L.sw_db_describe.restype = ctypes.c_int
    L.sw_db_describe.argtypes = [vp, i32, i32, i32, ctypes.POINTER(vp)]
    L.sw_plan_items.restype = ctypes.c_int64
    L.sw_plan_items.argtypes = [vp, i32, vp, ctypes.POINTER(Options), vp, i64]
    L.sw_db_sorted_lengths.restype = ctypes.c_int
    L.sw_db_sorted_lengths.argtypes = [vp, vp]
    L.sw_autotune.restype = ctypes.c_int
    L.sw_autotune.argtypes = [vp, vp, i32, vp, i32, i32, vp, ctypes.POINTER(TuneEntry)]
    L.sw_autotune_batch.restype = ctypes.c_int
    L.sw_autotune_batch.argtypes = [vp, vp, vp, vp, i32, vp, i32, i32, vp, ctypes.POINTER(TuneEntry)]
    L.sw_tune_set.restype = ctypes.c_int
    L.sw_tune_set.argtypes = [vp, ctypes.POINTER(TuneEntry), i32]
    L.sw_tune_get.restype = ctypes.c_int32
    L.sw_tune_get.argtypes = [vp, ctypes.POINTER(TuneEntry), i32]
    L.sw_graph_create.restype = ctypes.c_int
    L.sw_graph_create.argtypes = [vp, vp, vp, vp, i32, vp, i32, i32, ctypes.POINTER(Options), vp, sz, vp,
                                  ctypes.POINTER(vp)]
    L.sw_graph_launch.restype = ctypes.c_int
    L.sw_graph_launch.argtypes = [vp, vp]
    L.sw_graph_destroy.restype = ctypes.c_int
    L.sw_graph_destroy.argtypes = [vp]
    L.sw_flagged_count.restype = ctypes.c_int64
    L.sw_flagged_count.argtypes = [vp, vp]
    L.sw_strerror.restype = ctypes.c_char_p
    L.sw_strerror.argtypes = [ctypes.c_int]
    L.sw_last_error.restype = ctypes.c_char_p
    L.sw_last_error.argtypes = []
    L.sw_version.restype = ctypes.c_char_p
    L.sw_version.argtypes = []
    _lib = L
    return L


def _check(rc: int, where: str):
    if rc != SW_OK:
        L = lib()
        raise SwdbError(rc, where, f"{L.sw_strerror(rc).decode()}: {L.sw_last_error().decode()}")


def version() -> str:
    return lib().sw_version().decode()


PAIR_MODES = {"auto": 0, "tiles": 1, "flow": 2}


def options(mode="auto", waves=0, lane_cells=0, max_lanes=0, lds_limit=0, grid_limit=0,
            wide_profile=0, pair_cols=0, pair_rows=0, align_block=0, slice_mcells=0, pair_mode=0,
            pair_sm_max=0, slice_begin=0, slice_count=0, pair_entry_bytes=0, strict_groups=0,
            pair_group_waves=0) -> Options:
    o = Options()
    o.pair_group_waves = int(pair_group_waves)
    o.strict_groups = int(strict_groups)
    o.pair_entry_bytes = int(pair_entry_bytes)
    o.slice_mcells = int(slice_mcells)
    o.slice_begin, o.slice_count = int(slice_begin), int(slice_count)
    o.pair_mode = PAIR_MODES[pair_mode] if isinstance(pair_mode, str) else int(pair_mode)
    o.pair_sm_max = int(pair_sm_max)
    o.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    o.waves, o.lane_cells, o.max_lanes = int(waves), int(lane_cells), int(max_lanes)
    o.lds_limit, o.grid_limit = int(lds_limit), int(grid_limit)
    o.wide_profile, o.pair_cols, o.pair_rows = int(wide_profile), int(pair_cols), int(pair_rows)
    o.align_block = int(align_block)
    return o


def select_variant(sm, gap_open: int, opt: Optional[Options] = None) -> int:
    """``sw_select_variant``: the kernel variant a search with this matrix,
    gap-open penalty and options runs (numbering of ``plan_info()["variant"]``)."""
    m = _matrix(sm)
    v = lib().sw_select_variant(m.ctypes.data, int(gap_open), ctypes.byref(opt) if opt is not None else None)
    _check(min(v, 0), "sw_select_variant")
    return int(v)


def _matrix(sm) -> np.ndarray:
    """Host int32 32x32 copy (the ABI takes the matrix from host memory)."""
    if hasattr(sm, "detach"):
        sm = sm.detach().cpu().numpy()
    m = np.ascontiguousarray(np.asarray(sm, dtype=np.int32))
    if m.shape != (32, 32):
        raise ValueError("substitution matrix must be 32x32")
    return m


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _on_stream(stream, *tensors):
    """Tensors allocated on torch's current stream but used by work on another
    ``stream``: tell the caching allocator, so that it does not hand their
    memory out again before that work is done."""
    import torch
    if stream is None or stream == torch.cuda.current_stream():
        return
    for t in tensors:
        if t is not None and t.numel():
            t.record_stream(stream)


def status_error(host) -> Optional["SwdbError"]:
    """``sw_status_code`` of status words copied to the host (a 4-element int32
    tensor or array): None, or the ``SwdbError`` the status reports."""
    a = np.ascontiguousarray(np.asarray(host.numpy() if hasattr(host, "numpy") else host, dtype=np.int32))
    st = Status.from_buffer_copy(a[:4].tobytes())
    rc = lib().sw_status_code(ctypes.byref(st))
    if rc == SW_OK:
        return None
    L = lib()
    return SwdbError(rc, "search status", f"{L.sw_strerror(rc).decode()}: {L.sw_last_error().decode()}")


def prepare_bytes(total_residues: int, nseq: int, max_len: int) -> int:
    """``sw_db_prepare_bytes``: device bytes of a prepared database's layout."""
    v = lib().sw_db_prepare_bytes(int(total_residues), int(nseq), int(max_len))
    if v == 0:
        raise SwdbError(-1, "sw_db_prepare_bytes", lib().sw_last_error().decode())
    return int(v)


def _dev(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr() if t.numel() else 0)


class SearchGraph:
    """A captured batched search (``sw_graph_*``).  ``queries`` is the device
    buffer the graph reads: write new residues of the same lengths into it
    (``queries.copy_(...)``) between launches."""

    def __init__(self, handle, db, queries, workspace, out):
        self._g = handle
        self.db = db
        self.queries, self.workspace, self.out = queries, workspace, out

    def launch(self, stream=None):
        """Replay the search on ``stream`` (asynchronous; ``status`` checks it)."""
        _check(lib().sw_graph_launch(self._g, _stream(stream)), "sw_graph_launch")
        return self.out

    def status(self, stream=None, raise_on_error: bool = True) -> dict:
        """Status words of the last replay (synchronises ``stream``)."""
        return self.db.status(self.workspace, stream, raise_on_error=raise_on_error)

    def destroy(self):
        if getattr(self, "_g", None) is not None:
            lib().sw_graph_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def search(query, residues, offsets, lengths, matrix, gap_open: int, gap_extend: int,
           out=None, stream=None):
    """One-shot ``sw_db_search`` (blocking).  Returns int32 scores on the device."""
    import torch
    n = int(lengths.numel())
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=lengths.device)
    sm = _matrix(matrix)
    rc = lib().sw_db_search(_dev(query, torch.uint8, "query"), int(query.numel()),
                            _dev(residues, torch.uint8, "residues"), _dev(offsets, torch.int64, "offsets"),
                            _dev(lengths, torch.int32, "lengths"), n, sm.ctypes.data,
                            int(gap_open), int(gap_extend), _dev(out, torch.int32, "out"), _stream(stream))
    _check(rc, "sw_db_search")
    return out


def pair_plan(m: int, n: int, opt: Optional[Options] = None, cu_count: int = 0) -> dict:
    """``sw_pair_plan``: the tile schedule of one long pair (host only)."""
    st = PairStats()
    _check(lib().sw_pair_plan(int(m), int(n), ctypes.byref(opt) if opt is not None else None, int(cu_count),
                              ctypes.byref(st)), "sw_pair_plan")
    return st.as_dict()


def pair_workspace_bytes(m: int, n: int, opt: Optional[Options] = None) -> int:
    v = lib().sw_pair_workspace_bytes(int(m), int(n), ctypes.byref(opt) if opt is not None else None)
    if v == 0:
        raise SwdbError(-1, "sw_pair_workspace_bytes", lib().sw_last_error().decode())
    return int(v)


def pair_score(query, subject, matrix, gap_open: int, gap_extend: int, opt: Optional[Options] = None,
               workspace=None, out=None, stream=None):
    """``sw_pair_score``: score of one long pair on the device (asynchronous on
    ``stream``).  Returns a device int32 tensor of one element."""
    import torch
    m, n = int(query.numel()), int(subject.numel())
    dev = query.device if m else subject.device
    if workspace is None:
        workspace = torch.empty(pair_workspace_bytes(m, n, opt), dtype=torch.uint8, device=dev)
    if out is None:
        out = torch.empty(1, dtype=torch.int32, device=dev)
    sm = _matrix(matrix)
    o = ctypes.byref(opt) if opt is not None else None
    rc = lib().sw_pair_score(_dev(query, torch.uint8, "query") if m else None, m,
                             _dev(subject, torch.uint8, "subject") if n else None, n, sm.ctypes.data,
                             int(gap_open), int(gap_extend), o, _dev(workspace, torch.uint8, "workspace"),
                             int(workspace.numel()), _dev(out, torch.int32, "out"), _stream(stream))
    _check(rc, "sw_pair_score")
    return out


STATIC_SCRATCH_BYTES = 64 << 20


def pair_score_static(query, subject, matrix, gap_open: int, gap_extend: int, opt: Optional[Options] = None,
                      out=None, stream=None):
    """``sw_pair_score_static``: ``pair_score`` on the library's static device
    scratch (no allocation by the library; ``out`` is allocated here unless
    given).  Calls overlapping on one GPU race on that scratch."""
    import torch
    m, n = int(query.numel()), int(subject.numel())
    dev = query.device if m else subject.device
    if out is None:
        out = torch.empty(1, dtype=torch.int32, device=dev)
    sm = _matrix(matrix)
    o = ctypes.byref(opt) if opt is not None else None
    rc = lib().sw_pair_score_static(_dev(query, torch.uint8, "query") if m else None, m,
                                    _dev(subject, torch.uint8, "subject") if n else None, n, sm.ctypes.data,
                                    int(gap_open), int(gap_extend), o, _dev(out, torch.int32, "out"),
                                    _stream(stream))
    _check(rc, "sw_pair_score_static")
    return out


def align_workspace_bytes(m: int, n: int, opt: Optional[Options] = None) -> int:
    v = lib().sw_align_workspace_bytes(int(m), int(n), ctypes.byref(opt) if opt is not None else None)
    if v == 0:
        raise SwdbError(-1, "sw_align_workspace_bytes", lib().sw_last_error().decode())
    return int(v)


def align_pair(query, subject, matrix, gap_open: int, gap_extend: int, opt: Optional[Options] = None,
               workspace=None, stream=None) -> dict:
    """``sw_align_pair``: optimal local alignment of one pair on the device.
    Blocking (copies the result back): score, 1-based inclusive begin/end
    positions and the operation string ('M', 'I', 'D') from begin to end."""
    import torch
    m, n = int(query.numel()), int(subject.numel())
    dev = query.device if m else subject.device
    if workspace is None:
        workspace = torch.empty(align_workspace_bytes(m, n, opt), dtype=torch.uint8, device=dev)
    out = torch.zeros(ctypes.sizeof(Alignment), dtype=torch.uint8, device=dev)
    ops = torch.zeros(max(m + n, 1), dtype=torch.uint8, device=dev)
    sm = _matrix(matrix)
    o = ctypes.byref(opt) if opt is not None else None
    rc = lib().sw_align_pair(_dev(query, torch.uint8, "query") if m else None, m,
                             _dev(subject, torch.uint8, "subject") if n else None, n, sm.ctypes.data,
                             int(gap_open), int(gap_extend), o, _dev(workspace, torch.uint8, "workspace"),
                             int(workspace.numel()), _dev(out, torch.uint8, "out"), _dev(ops, torch.uint8, "ops"),
                             _stream(stream))
    _check(rc, "sw_align_pair")
    (torch.cuda.current_stream(dev) if stream is None else stream).synchronize()
    a = Alignment.from_buffer_copy(out.cpu().numpy().tobytes())
    if a.n_ops < 0:
        raise SwdbError(-3, "sw_align_pair", "inconsistent direction codes")
    if a.score < 0:
        raise SwdbError(-3, "sw_align_pair", "a wait of the pipelined score pass gave up")
    return {"score": a.score, "q_begin": a.q_begin, "s_begin": a.s_begin, "q_end": a.q_end, "s_end": a.s_end,
            "ops": ops[:a.n_ops].cpu().numpy().tobytes().decode() if a.n_ops > 0 else ""}


class Database:
    """A resident, length-sorted, lane-interleaved database (``sw_db_prepare``)."""

    @classmethod
    def describe(cls, lengths, cu_count: int = 0, lds_bytes: int = 0) -> "Database":
        """Planning-only handle from host lengths (``sw_db_describe``): no GPU needed."""
        self = cls.__new__(cls)
        ln = np.ascontiguousarray(np.asarray(lengths, dtype=np.int32))
        h = ctypes.c_void_p()
        _check(lib().sw_db_describe(ln.ctypes.data if len(ln) else None, len(ln), int(cu_count),
                                    int(lds_bytes), ctypes.byref(h)), "sw_db_describe")
        self._h = h
        self.nseq = len(ln)
        self.device = None
        self.total = int(ln.sum())
        self.device_bytes = 0
        return self

    def plan_items(self, qlens: Sequence[int], opt: Optional[Options] = None) -> np.ndarray:
        """``sw_plan_items``: the work queue as an int32 array [n, 4]."""
        ql = np.ascontiguousarray(np.asarray(qlens, dtype=np.int32))
        o = ctypes.byref(opt) if opt is not None else None
        n = lib().sw_plan_items(self._handle(), len(ql), ql.ctypes.data if len(ql) else None, o, None, 0)
        if n < 0:
            _check(int(n), "sw_plan_items")
        out = np.zeros((max(n, 1), 4), dtype=np.int32)
        n2 = lib().sw_plan_items(self._handle(), len(ql), ql.ctypes.data if len(ql) else None, o,
                                 out.ctypes.data, n)
        if n2 < 0:
            _check(int(n2), "sw_plan_items")
        return out[:n]

    def sorted_lengths(self) -> np.ndarray:
        out = np.zeros(max(self.nseq, 1), dtype=np.int32)
        _check(lib().sw_db_sorted_lengths(self._handle(), out.ctypes.data), "sw_db_sorted_lengths")
        return out[:self.nseq]

    def __init__(self, residues, offsets, lengths, stream=None, total=None, max_len=None, layout=None):
        """``sw_db_prepare`` into a caller-owned layout tensor: ``layout`` (a
        device uint8 tensor of at least ``prepare_bytes`` bytes) or one
        allocated here from torch's allocator.  ``total`` / ``max_len``
        (residues, longest subject) size it; computed from ``lengths`` when
        not given."""
        import torch
        self._h = None
        self.nseq = int(lengths.numel())
        self.device = lengths.device
        if total is None or max_len is None:
            total = int(lengths.sum().item()) if self.nseq else 0
            max_len = int(lengths.max().item()) if self.nseq else 0
        if layout is None:
            layout = torch.empty(prepare_bytes(total, self.nseq, max_len), dtype=torch.uint8, device=self.device)
        self.layout = layout
        h = ctypes.c_void_p()
        rc = lib().sw_db_prepare(_dev(residues, torch.uint8, "residues"),
                                 _dev(offsets, torch.int64, "offsets"),
                                 _dev(lengths, torch.int32, "lengths"), self.nseq,
                                 _dev(layout, torch.uint8, "layout"), int(layout.numel()),
                                 _stream(stream), ctypes.byref(h))
        _check(rc, "sw_db_prepare")
        self._h = h
        n, r, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().sw_db_info(h, ctypes.byref(n), ctypes.byref(r), ctypes.byref(b)), "sw_db_info")
        self.total = int(r.value)
        self.device_bytes = int(b.value)

    @classmethod
    def from_host(cls, db, device="cuda", stream=None, layout=None):
        """From a ``synth.Database``-like object with numpy arrays."""
        import torch
        lens = np.ascontiguousarray(db.lengths, dtype=np.int32)
        res = torch.from_numpy(np.ascontiguousarray(db.residues)).to(device)
        off = torch.from_numpy(np.ascontiguousarray(db.offsets, dtype=np.int64)).to(device)
        ln = torch.from_numpy(lens).to(device)
        total = int(lens.sum(dtype=np.int64)) if len(lens) else 0
        mx = int(lens.max()) if len(lens) else 0
        return cls(res, off, ln, stream, total=total, max_len=mx, layout=layout)

    def _handle(self):
        if self._h is None:
            raise SwdbError(-1, "Database", "released")
        return self._h

    def release(self):
        if getattr(self, "_h", None) is not None:
            lib().sw_db_release(self._h)
            self._h = None
        self.layout = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass

    def workspace_bytes(self, qlens: Sequence[int], opt: Optional[Options] = None) -> int:
        ql = np.ascontiguousarray(np.asarray(qlens, dtype=np.int32))
        n = lib().sw_workspace_bytes(self._handle(), len(ql), ql.ctypes.data if len(ql) else None,
                                     ctypes.byref(opt) if opt is not None else None)
        if n == 0 and len(ql):
            raise SwdbError(-1, "sw_workspace_bytes", lib().sw_last_error().decode())
        return int(n)

    def plan_info(self, qlens: Sequence[int], opt: Optional[Options] = None) -> dict:
        ql = np.ascontiguousarray(np.asarray(qlens, dtype=np.int32))
        st = PlanStats()
        _check(lib().sw_plan_info(self._handle(), len(ql), ql.ctypes.data if len(ql) else None,
                                  ctypes.byref(opt) if opt is not None else None, ctypes.byref(st)),
               "sw_plan_info")
        return st.as_dict()

    def alloc_workspace(self, qlens: Sequence[int], opt: Optional[Options] = None):
        import torch
        n = self.workspace_bytes(qlens, opt)
        return torch.empty(max(n, 256), dtype=torch.uint8, device=self.device)

    def search(self, query, matrix, gap_open: int, gap_extend: int, opt: Optional[Options] = None,
               out=None, workspace=None, stream=None, check: bool = True):
        """``sw_db_search_ex``: one device query on ``stream``.  With ``check``
        the call waits for the search and raises ``SwdbError`` if its status
        reports an error; without it the call is asynchronous."""
        import torch
        m = int(query.numel())
        if workspace is None:
            workspace = self.alloc_workspace([m], opt)
        if out is None:
            out = torch.empty(self.nseq, dtype=torch.int32, device=self.device)
        _on_stream(stream, query, workspace, out)
        sm = _matrix(matrix)
        rc = lib().sw_db_search_ex(self._handle(), _dev(query, torch.uint8, "query"), m, sm.ctypes.data,
                                   int(gap_open), int(gap_extend),
                                   ctypes.byref(opt) if opt is not None else None,
                                   _dev(workspace, torch.uint8, "workspace"), int(workspace.numel()),
                                   _dev(out, torch.int32, "out"), _stream(stream))
        _check(rc, "sw_db_search_ex")
        if check and self.nseq:
            self.status(workspace, stream, raise_on_error=True)
        return out

    def search_batch(self, queries, matrix, gap_open: int, gap_extend: int,
                     opt: Optional[Options] = None, out=None, workspace=None, stream=None,
                     check: bool = True):
        """``sw_db_search_batch``.  ``queries``: a list of device uint8 tensors,
        or a tuple (concatenated device tensor, host offsets, host lengths).
        ``check`` as for ``search``."""
        import torch
        cat, offs, lens = self._batch_args(queries)
        nq = len(lens)
        if workspace is None:
            workspace = self.alloc_workspace(lens, opt)
        if out is None:
            out = torch.empty((nq, self.nseq), dtype=torch.int32, device=self.device)
        _on_stream(stream, cat, workspace, out)
        sm = _matrix(matrix)
        rc = lib().sw_db_search_batch(self._handle(), _dev(cat, torch.uint8, "queries"),
                                      offs.ctypes.data if nq else None, lens.ctypes.data if nq else None,
                                      nq, sm.ctypes.data, int(gap_open), int(gap_extend),
                                      ctypes.byref(opt) if opt is not None else None,
                                      _dev(workspace, torch.uint8, "workspace"), int(workspace.numel()),
                                      _dev(out, torch.int32, "out"), _stream(stream))
        _check(rc, "sw_db_search_batch")
        if check and nq and self.nseq:
            self.status(workspace, stream, raise_on_error=True)
        return out

    def capture(self, queries, matrix, gap_open: int, gap_extend: int, opt: Optional[Options] = None,
                out=None, workspace=None) -> "SearchGraph":
        """``sw_graph_create``: a replayable graph of one batched search."""
        import torch
        cat, offs, lens = self._batch_args(queries)
        nq = len(lens)
        if workspace is None:
            workspace = self.alloc_workspace(lens, opt)
        if out is None:
            out = torch.empty((nq, self.nseq), dtype=torch.int32, device=self.device)
        sm = _matrix(matrix)
        g = ctypes.c_void_p()
        rc = lib().sw_graph_create(self._handle(), _dev(cat, torch.uint8, "queries"),
                                   offs.ctypes.data if nq else None, lens.ctypes.data if nq else None, nq,
                                   sm.ctypes.data, int(gap_open), int(gap_extend),
                                   ctypes.byref(opt) if opt is not None else None,
                                   _dev(workspace, torch.uint8, "workspace"), int(workspace.numel()),
                                   _dev(out, torch.int32, "out"), ctypes.byref(g))
        _check(rc, "sw_graph_create")
        return SearchGraph(g, self, cat, workspace, out)

    def _batch_args(self, queries):
        import torch
        if isinstance(queries, tuple):
            cat, offs, lens = queries
            return (cat, np.ascontiguousarray(np.asarray(offs, dtype=np.int64)),
                    np.ascontiguousarray(np.asarray(lens, dtype=np.int32)))
        lens = np.array([int(q.numel()) for q in queries], dtype=np.int32)
        offs = np.zeros(len(lens), dtype=np.int64)
        if len(lens) > 1:
            offs[1:] = np.cumsum(lens[:-1])
        cat = (torch.cat([q.reshape(-1) for q in queries]) if len(queries)
               else torch.empty(0, dtype=torch.uint8, device=self.device))
        return cat, offs, lens

    def autotune(self, qlens: Sequence[int], matrix, gap_open: int, gap_extend: int, stream=None):
        """``sw_autotune``: time candidate schedules per query length; installs
        the winners for mode ``"tuned"`` and returns them as dicts."""
        ql = np.ascontiguousarray(np.sort(np.asarray(qlens, dtype=np.int32)))
        out = (TuneEntry * len(ql))()
        sm = _matrix(matrix)
        _check(lib().sw_autotune(self._handle(), ql.ctypes.data, len(ql), sm.ctypes.data, int(gap_open),
                                 int(gap_extend), _stream(stream), out), "sw_autotune")
        return [e.as_dict() for e in out]

    def autotune_batch(self, queries, matrix, gap_open: int, gap_extend: int, stream=None):
        """``sw_autotune_batch``: tune one batch as a unit.  ``queries`` as for
        ``search_batch``.  Returns (Options for ``search_batch`` / ``capture``
        of this batch, dict of the schedule and its measured GCUPS); installs
        nothing."""
        import torch
        cat, offs, lens = self._batch_args(queries)
        nq = len(lens)
        if nq == 0:
            raise ValueError("empty batch")
        _on_stream(stream, cat)
        sm = _matrix(matrix)
        out = TuneEntry()
        _check(lib().sw_autotune_batch(self._handle(), _dev(cat, torch.uint8, "queries"), offs.ctypes.data,
                                       lens.ctypes.data, nq, sm.ctypes.data, int(gap_open), int(gap_extend),
                                       _stream(stream), ctypes.byref(out)), "sw_autotune_batch")
        d = out.as_dict()
        return TuneEntry.from_dict(d).opt, d

    def set_tuning(self, entries):
        arr = (TuneEntry * len(entries))(*[TuneEntry.from_dict(d) for d in entries])
        _check(lib().sw_tune_set(self._handle(), arr, len(entries)), "sw_tune_set")

    def get_tuning(self):
        n = lib().sw_tune_get(self._handle(), None, 0)
        if n < 0:
            _check(int(n), "sw_tune_get")
        arr = (TuneEntry * max(n, 1))()
        lib().sw_tune_get(self._handle(), arr, n)
        return [arr[k].as_dict() for k in range(n)]

    def status(self, workspace, stream=None, raise_on_error: bool = False) -> dict:
        """``sw_search_status``: the status words of the last search that used
        ``workspace`` (synchronises ``stream``).  With ``raise_on_error`` a
        status error raises ``SwdbError``."""
        import torch
        st = Status()
        rc = lib().sw_search_status(_dev(workspace, torch.uint8, "workspace"), _stream(stream),
                                    ctypes.byref(st))
        if raise_on_error or rc == -3:
            _check(rc, "search status")
        d = st.as_dict()
        d["code"] = int(rc)
        return d

    def status_async(self, workspace, host, stream=None):
        """``sw_search_status_async``: enqueue on ``stream`` a copy of the status
        words into ``host`` (a pinned int32 CPU tensor of 4 elements);
        ``status_error(host)`` decodes it once the stream has passed the copy."""
        import torch
        if host.dtype != torch.int32 or host.numel() < 4 or host.is_cuda or not host.is_contiguous():
            raise TypeError("host status buffer must be a contiguous CPU int32 tensor of 4 elements")
        _check(lib().sw_search_status_async(_dev(workspace, torch.uint8, "workspace"),
                                            ctypes.c_void_p(host.data_ptr()), _stream(stream)),
               "sw_search_status_async")

    def flagged_count(self, workspace, stream=None) -> int:
        import torch
        v = lib().sw_flagged_count(_dev(workspace, torch.uint8, "workspace"), _stream(stream))
        if v < 0:
            _check(int(v), "sw_flagged_count")
        return int(v)
