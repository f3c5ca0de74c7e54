"""Scheduler logic of the serving loop, on the CPU with a fake backend.

The fake backend scores with the CPU oracle (test infrastructure) after a
simulated device delay; it lets these tests check admission by memory, slot
limits, continuous batching, cancellation, failure isolation and the latency
statistics without a GPU.  The GPU backend is exercised in test_gpu_serve.py.
"""
import threading
import time

import numpy as np
import pytest

import oracle
import synth
from paper_2412_08308_amd.serve import Server, percentiles


class FakeBackend:
    slots = 3

    def __init__(self, db, sm, delay=0.02, bytes_per_residue=100, fail_len=None):
        self.db, self.sm, self.delay = db, sm, delay
        self.bpr = bytes_per_residue
        self.fail_len = fail_len
        self.launches = []
        self.active = 0
        self.max_active = 0
        self.lock = threading.Lock()

    def need_bytes(self, qlens):
        return 1000 + self.bpr * int(sum(qlens))

    def cells(self, qlens):
        return int(sum(qlens)) * self.db.total

    def launch(self, slot, queries):
        if self.fail_len is not None and any(len(q) == self.fail_len for q in queries):
            raise RuntimeError("injected launch failure")
        with self.lock:
            self.active += 1
            self.max_active = max(self.max_active, self.active)
        h = {"t": time.perf_counter() + self.delay, "q": queries, "slot": slot, "closed": False}
        self.launches.append((slot, [len(q) for q in queries]))
        return h

    def poll(self, h):
        done = time.perf_counter() >= h["t"]
        if done and not h["closed"]:
            with self.lock:
                self.active -= 1
            h["closed"] = True
        return done

    def results(self, h):
        return [oracle.search_db(q, self.db, self.sm, 10, 2).astype(np.int32) for q in h["q"]]


def _db(n=60):
    rng = np.random.default_rng(4)
    return synth.Database.from_list([synth.residues(rng, int(x)) for x in rng.integers(1, 80, size=n)])


def test_results_equal_alone_and_in_mix():
    db, sm = _db(), synth.blosum_style_matrix()
    rng = np.random.default_rng(5)
    qs = [synth.residues(rng, int(m)) for m in rng.integers(1, 60, size=25)]
    be = FakeBackend(db, sm)
    with Server(be, max_batch=6, mem_budget=10**9) as srv:
        futs = []
        for q in qs:
            futs.append(srv.submit(q))
            time.sleep(0.002)
        got = [f.result(timeout=30) for f in futs]
    for q, g in zip(qs, got):
        assert np.array_equal(g, oracle.search_db(q, db, sm, 10, 2))
    st = srv.stats()
    assert st["completed"] == len(qs)
    assert st["max_batch"] > 1, "arrivals during a running batch must be batched together"
    assert be.max_active <= be.slots
    assert all(f.latency > 0 for f in futs)


def test_admission_respects_memory_budget():
    db, sm = _db(), synth.blosum_style_matrix()
    rng = np.random.default_rng(6)
    be = FakeBackend(db, sm, delay=0.01)
    budget = 1000 + 100 * 120          # about two 50-residue requests at a time
    with Server(be, max_batch=8, mem_budget=budget) as srv:
        futs = [srv.submit(synth.residues(rng, 50)) for _ in range(12)]
        for f in futs:
            f.result(timeout=30)
    assert srv.stats()["max_bytes_in_use"] <= budget
    assert srv.stats()["completed"] == 12


def test_oversize_and_bad_requests():
    db, sm = _db(), synth.blosum_style_matrix()
    be = FakeBackend(db, sm)
    with Server(be, mem_budget=5000) as srv:
        f = srv.submit(np.zeros(100, np.uint8))          # needs 11,000 bytes > budget
        with pytest.raises(MemoryError):
            f.result(timeout=5)
        with pytest.raises(ValueError):
            srv.submit(np.array([1, 2, 40], np.uint8))
        with pytest.raises(ValueError):
            srv.submit(np.array([1.0, 2.0]))
        ok = srv.submit(np.array([1, 2, 3], np.uint8))
        assert len(ok.result(timeout=10)) == db.nseq


def test_failed_launch_is_isolated():
    db, sm = _db(), synth.blosum_style_matrix()
    be = FakeBackend(db, sm, fail_len=13)
    with Server(be, max_batch=1, mem_budget=10**9) as srv:
        bad = srv.submit(np.ones(13, np.uint8))
        good = [srv.submit(np.ones(n, np.uint8)) for n in (5, 7, 9)]
        with pytest.raises(RuntimeError):
            bad.result(timeout=10)
        for f in good:
            assert f.result(timeout=10) is not None
    assert srv.stats()["errors"] == 1


def test_cancel_pending():
    db, sm = _db(), synth.blosum_style_matrix()
    be = FakeBackend(db, sm, delay=0.2)
    srv = Server(be, max_batch=1, max_inflight=1, mem_budget=10**9).start()
    first = srv.submit(np.ones(5, np.uint8))
    time.sleep(0.05)
    second = srv.submit(np.ones(6, np.uint8))
    assert second.cancel()
    assert first.result(timeout=10) is not None
    srv.stop()
    assert second.cancelled()
    assert srv.stats()["completed"] == 1


@pytest.mark.parametrize("policy", ["edf", "fifo"])
def test_admission_order(policy):
    """While one request runs, a long and then a short one arrive: deadline
    order (arrival + estimated service time) runs the short one first, arrival
    order the long one."""
    db, sm = _db(), synth.blosum_style_matrix()
    be = FakeBackend(db, sm, delay=0.05)
    rate = be.cells([1]) / 1e-3        # 1 ms of service per query residue
    srv = Server(be, max_batch=1, max_inflight=1, mem_budget=10**9, policy=policy, rate_guess=rate).start()
    first = srv.submit(np.ones(20, np.uint8))
    time.sleep(0.01)
    long_ = srv.submit(np.ones(60, np.uint8))      # deadline about +60 ms
    time.sleep(0.002)
    short = srv.submit(np.ones(5, np.uint8))       # deadline about +7 ms
    for f in (first, long_, short):
        f.result(timeout=10)
    srv.stop()
    order = [lens[0] for _, lens in be.launches]
    assert order[0] == 20
    assert order[1:] == ([5, 60] if policy == "edf" else [60, 5])


def test_policy_checked():
    db, sm = _db(), synth.blosum_style_matrix()
    with pytest.raises(ValueError):
        Server(FakeBackend(db, sm), mem_budget=10**9, policy="lifo")


def test_percentiles_known_values():
    p50, p99 = percentiles(list(range(1, 101)))
    assert p50 == pytest.approx(50.5) and p99 == pytest.approx(99.01)
    assert percentiles([]) == (None, None)


class PollRaises(FakeBackend):
    """poll() raises on its n-th call, like an asynchronous device error
    surfacing through Event.query()."""

    def __init__(self, *a, raise_after=3, **kw):
        super().__init__(*a, **kw)
        self.calls = 0
        self.raise_after = raise_after

    def poll(self, h):
        self.calls += 1
        if self.calls >= self.raise_after:
            raise RuntimeError("injected device error")
        return super().poll(h)


def test_scheduler_error_fails_every_request():
    db, sm = _db(20), synth.blosum_style_matrix()
    be = PollRaises(db, sm, delay=0.05)
    srv = Server(be, max_batch=2, mem_budget=10**9).start()
    rng = np.random.default_rng(9)
    futs = [srv.submit(rng.integers(0, 20, size=30).astype(np.uint8)) for _ in range(8)]
    for f in futs:
        with pytest.raises(RuntimeError):
            f.result(timeout=10)
    srv.stop()
    assert srv.errors and "injected device error" in str(srv.errors[-1])
    late = srv.submit(np.zeros(5, np.uint8))
    with pytest.raises(RuntimeError):
        late.result(timeout=1)


class StatusFails(FakeBackend):
    """results() raises for batches holding a query of a given length, as the
    GPU backend does when a batch's search status reports an error."""

    def __init__(self, *a, bad_len=None, **kw):
        super().__init__(*a, **kw)
        self.bad_len = bad_len

    def results(self, h):
        if any(len(q) == self.bad_len for q in h["q"]):
            raise RuntimeError("search status: exact int32 rescore incomplete")
        return super().results(h)


def test_status_error_fails_its_batch_only():
    db, sm = _db(20), synth.blosum_style_matrix()
    be = StatusFails(db, sm, delay=0.01, bad_len=13)
    rng = np.random.default_rng(10)
    with Server(be, max_batch=1, mem_budget=10**9) as srv:
        good = [srv.submit(rng.integers(0, 20, size=40).astype(np.uint8)) for _ in range(3)]
        bad = srv.submit(rng.integers(0, 20, size=13).astype(np.uint8))
        good.append(srv.submit(rng.integers(0, 20, size=41).astype(np.uint8)))
        with pytest.raises(RuntimeError):
            bad.result(timeout=10)
        for f in good:
            assert f.result(timeout=10).shape == (db.nseq,)


def test_short_requests_not_batched_with_long():
    """A batch holds requests within size_ratio of its first request's cells:
    short and long requests pending together go to different batches."""
    db, sm = _db(), synth.blosum_style_matrix()
    be = FakeBackend(db, sm, delay=0.05)
    rate = be.cells([1]) / 1e-3
    srv = Server(be, max_batch=8, max_inflight=1, mem_budget=10**9, rate_guess=rate, long_s=10.0).start()
    blocker = srv.submit(np.ones(30, np.uint8))
    time.sleep(0.01)
    futs = [srv.submit(np.ones(m, np.uint8)) for m in (40, 5, 45, 6, 4)]
    for f in [blocker] + futs:
        f.result(timeout=10)
    srv.stop()
    batches = [sorted(lens) for _, lens in be.launches]
    assert batches[0] == [30]
    assert sorted(map(tuple, batches[1:])) == [(4, 5, 6), (40, 45)]


def test_one_slot_kept_for_short_requests():
    """Long requests hold at most all but one in-flight slot: with two slots
    and two long requests pending, a short one arriving later runs before the
    second long one starts."""
    db, sm = _db(), synth.blosum_style_matrix()
    be = FakeBackend(db, sm, delay=0.08)
    be.slots = 2
    rate = be.cells([1]) / 1e-3        # 1 ms per residue: 40 residues = 40 ms > long_s
    srv = Server(be, max_batch=1, mem_budget=10**9, rate_guess=rate, long_s=0.02).start()
    l1 = srv.submit(np.ones(40, np.uint8))
    l2 = srv.submit(np.ones(41, np.uint8))
    time.sleep(0.02)
    sh = srv.submit(np.ones(5, np.uint8))
    for f in (l1, l2, sh):
        f.result(timeout=10)
    srv.stop()
    order = [lens[0] for _, lens in be.launches]
    assert order == [40, 5, 41]
    assert be.max_active <= 2


def test_latency_by_length_class():
    db, sm = _db(), synth.blosum_style_matrix()
    be = FakeBackend(db, sm, delay=0.005)
    with Server(be, max_batch=4, mem_budget=10**9) as srv:
        fs = [srv.submit(np.ones(m, np.uint8)) for m in (3, 8, 15, 30, 31, 60)]
        for f in fs:
            f.result(timeout=10)
    cls = srv.stats_by_length([10, 30])
    assert [c["requests"] for c in cls] == [2, 1, 3]
    assert cls[0]["qlen_lo"] == 0 and cls[2]["qlen_hi"] is None
    assert all(c["p50_s"] > 0 and c["p99_s"] >= c["p50_s"] for c in cls)


class StepBackend(FakeBackend):
    """A device that runs enqueued work in order, one piece at a time.  A
    batch launched ``stepped`` has ``qlen // 10`` launches of ``slice_s``
    each, which the scheduler enqueues with ``advance``; other batches run
    whole (``delay``)."""

    def __init__(self, *a, slice_s=0.01, **kw):
        super().__init__(*a, **kw)
        self.slice_s = slice_s
        self.free_at = 0.0
        self.log = []                  # (kind, query lengths, enqueued, start, end)

    def _run(self, dur, kind, h):
        now = time.perf_counter()
        start = max(now, self.free_at)
        self.free_at = start + dur
        self.log.append((kind, [len(q) for q in h["q"]], now, start, self.free_at))
        return self.free_at

    def launch(self, slot, queries, stepped=False):
        h = {"q": queries, "next": 0, "total": 1, "t": None, "ends": []}
        self.launches.append((slot, [len(q) for q in queries]))
        if stepped:
            h["total"] = max(1, sum(len(q) for q in queries) // 10)
        else:
            h["t"] = self._run(self.delay, "whole", h)
        return h

    def advance(self, h):
        h["ends"].append(self._run(self.slice_s, "slice", h))
        h["next"] += 1
        if h["next"] == h["total"]:
            h["t"] = h["ends"][-1]

    def remaining(self, h):
        return h["total"] - h["next"]

    def queued(self, h):
        now = time.perf_counter()
        return sum(1 for t in h["ends"] if now < t)

    def poll(self, h):
        return h["t"] is not None and time.perf_counter() >= h["t"]


@pytest.mark.parametrize("depth", [1, 2])
def test_long_batches_step_around_short_ones(depth):
    """A long request runs launch by launch; a short one arriving meanwhile is
    enqueued at once, waits only for the long launches already queued (at most
    long_depth), and no long launch is enqueued while it is in flight."""
    db, sm = _db(), synth.blosum_style_matrix()
    be = StepBackend(db, sm, delay=0.02, slice_s=0.01)
    rate = be.cells([1]) / 1e-3        # 1 ms per residue: 80 residues = 80 ms > long_s
    srv = Server(be, max_batch=1, mem_budget=10**9, rate_guess=rate, long_s=0.03, long_depth=depth).start()
    rng = np.random.default_rng(12)
    long_q = rng.integers(0, 20, size=80).astype(np.uint8)
    short_q = rng.integers(0, 20, size=6).astype(np.uint8)
    fl = srv.submit(long_q)
    time.sleep(0.035)
    fs = srv.submit(short_q)
    got_l, got_s = fl.result(timeout=10), fs.result(timeout=10)
    srv.stop()
    assert np.array_equal(got_l, oracle.search_db(long_q, db, sm, 10, 2))
    assert np.array_equal(got_s, oracle.search_db(short_q, db, sm, 10, 2))
    whole = [x for x in be.log if x[0] == "whole"]
    slices = [x for x in be.log if x[0] == "slice"]
    assert len(whole) == 1 and len(slices) == 8
    _, _, enq, start, end = whole[0]
    # at most `depth` long launches were queued ahead of the short request ...
    assert sum(1 for x in slices if x[2] < enq and x[4] > enq) <= depth
    # ... and none was enqueued while it was in flight
    assert not [x for x in slices if enq <= x[2] < end]
    assert fs.latency < 0.02 + depth * 0.01 + 0.03
    # the long batch's time includes launches held back for the short one: it
    # does not count as a measure of the device rate
    assert srv.rate == rate


class StepFails(StepBackend):
    """advance() raises for batches holding a query of a given length."""

    def __init__(self, *a, bad_len=None, **kw):
        super().__init__(*a, **kw)
        self.bad_len = bad_len

    def advance(self, h):
        if any(len(q) == self.bad_len for q in h["q"]) and h["next"] >= 2:
            raise RuntimeError("injected launch failure in a stepped batch")
        super().advance(h)


def test_failed_stepped_launch_fails_its_batch_only():
    db, sm = _db(), synth.blosum_style_matrix()
    be = StepFails(db, sm, delay=0.01, slice_s=0.005, bad_len=70)
    rate = be.cells([1]) / 1e-3
    rng = np.random.default_rng(13)
    with Server(be, max_batch=1, mem_budget=10**9, rate_guess=rate, long_s=0.03) as srv:
        bad = srv.submit(rng.integers(0, 20, size=70).astype(np.uint8))
        good = [srv.submit(rng.integers(0, 20, size=m).astype(np.uint8)) for m in (80, 6, 9)]
        with pytest.raises(RuntimeError):
            bad.result(timeout=10)
        for f in good:
            assert f.result(timeout=10).shape == (db.nseq,)
    assert srv.stats()["errors"] == 1 and srv.stats()["completed"] == 3
