"""Scheduling logic of the serving loop on the CPU, with a simulated
executor and clock (no GPU)."""

import numpy as np
import pytest

from paper_2009_09500_amd import serving


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class SimExecutor:
    """Runs batches one after another like a single GPU queue: a batch takes
    `fixed + per_seg * segments` seconds from when the previous one ends."""

    def __init__(self, clock, sched, fixed=1e-4, per_seg=1e-8, failing_batches=()):
        self.clock, self.sched = clock, sched
        self.fixed, self.per_seg = fixed, per_seg
        self.failing = set(failing_batches)   # indices of batches whose status reports an error
        self.busy_until = 0.0
        self.uploaded = []
        self.batches = []
        self.slot_owner = {}
        self.chunks = {}

    def upload(self, r):
        assert self.sched.used_bytes <= self.sched.budget
        assert r.slot not in self.slot_owner, "slot handed out twice"
        self.slot_owner[r.slot] = r.rid
        self.uploaded.append(r.rid)

    def launch(self, chunks):
        segs = sum(c.hi - c.lo for c in chunks)
        assert segs <= self.sched.max_batch_segments
        assert len(chunks) <= self.sched.max_batch_scenes
        assert len({c.req.rid for c in chunks}) == len(chunks)
        for c in chunks:
            self.chunks.setdefault(c.req.rid, []).append((c.lo, c.hi, c.first, c.last))
        start = max(self.busy_until, self.clock())
        self.busy_until = start + self.fixed + self.per_seg * segs
        self.batches.append(chunks)
        return (self.busy_until, len(self.batches) - 1)

    def poll(self, handle):
        return self.clock() >= handle[0]

    def batch_status(self, handle):
        return 1 if handle[1] in self.failing else 0

    def release(self, r):
        del self.slot_owner[r.slot]


def make_requests(sizes, arrivals):
    reqs = []
    for i, (n, t) in enumerate(zip(sizes, arrivals)):
        segs = np.zeros((n, 6), np.int32)
        segs[:, 3] = i % 7            # N = i % 7
        reqs.append(serving.Request(i, segs, (64, 64, 64), float(t)))
    return reqs


def serve(reqs, slots=4, budget=10**9, max_segs=50_000, max_scenes=8, **kw):
    clock = SimClock()
    sched = serving.Scheduler(slots, budget, max_segs, max_scenes)
    ex = SimExecutor(clock, sched, **kw)
    stats = serving.run(reqs, ex, sched, clock=clock, sleep=clock.sleep)
    return stats, ex, sched


def test_every_request_completes_with_exact_chunks():
    rng = np.random.default_rng(0)
    sizes = rng.integers(0, 200_000, 60).tolist() + [0, 1, 50_000, 50_001]
    arrivals = np.sort(rng.uniform(0, 0.05, len(sizes)))
    reqs = make_requests(sizes, arrivals)
    stats, ex, sched = serve(reqs)
    assert stats["requests"] == len(reqs) and sched.idle() and not ex.slot_owner
    for r in reqs:
        ch = ex.chunks[r.rid]
        assert ch[0][0] == 0 and ch[-1][1] == r.n           # covers [0, n) ...
        for (lo, hi, _, _), (lo2, _, _, _) in zip(ch, ch[1:]):
            assert hi == lo2                                # ... in order, once
        assert [c[2] for c in ch] == [True] + [False] * (len(ch) - 1)
        assert [c[3] for c in ch] == [False] * (len(ch) - 1) + [True]
        assert r.done >= r.admitted >= r.arrival
        assert r.voxels == r.n * (r.rid % 7 + 1)
    assert stats["latency_p99_ms"] >= stats["latency_p50_ms"] > 0


def test_admission_is_fifo_and_within_budget():
    sizes = [40_000, 10_000, 30_000, 5_000, 45_000, 1_000] * 5
    reqs = make_requests(sizes, np.zeros(len(sizes)))
    budget = 24 * 60_000                                   # at most ~2 requests' segments
    stats, ex, sched = serve(reqs, slots=3, budget=budget)
    assert ex.uploaded == list(range(len(reqs)))           # admitted in arrival order
    assert sched.peak_bytes <= budget
    assert stats["requests"] == len(reqs)


def test_slots_limit_admission():
    reqs = make_requests([1000] * 20, np.zeros(20))
    clock = SimClock()
    sched = serving.Scheduler(2, 10**12, 10**6, 16)
    admitted = sched.admit(0.0)
    for r in reqs:
        sched.arrive(r)
    admitted = sched.admit(0.0)
    assert [r.rid for r in admitted] == [0, 1] and not sched.free_slots
    chunks = sched.form_batch()
    assert [c.req.rid for c in chunks] == [0, 1]
    done = sched.complete(chunks, 1.0)
    assert [r.rid for r in done] == [0, 1]
    assert [r.rid for r in sched.admit(1.0)] == [2, 3]


def test_large_request_is_chunked_and_small_ones_overtake():
    """Continuous batching: a request arriving while a large one is being
    processed chunk by chunk finishes long before the large one."""
    sizes = [1_000_000, 2_000]
    reqs = make_requests(sizes, [0.0, 0.002])
    stats, ex, _ = serve(reqs, max_segs=100_000, per_seg=1e-7)
    big, small = reqs
    assert len(ex.chunks[big.rid]) == 11          # one chunk shrank to make room
    assert small.done < big.done
    # At most the batches already queued (two) and its own one ahead of it.
    batch_time = 1e-4 + 1e-7 * 100_000
    assert small.done - small.arrival <= 3 * batch_time + 1e-4
    assert small.done - small.arrival < 0.35 * (big.done - big.arrival)


def test_batch_limits():
    reqs = make_requests([10] * 40, np.zeros(40))
    stats, ex, _ = serve(reqs, slots=40, max_scenes=6)
    assert max(len(b) for b in ex.batches) == 6
    assert stats["batches"] == 7


def test_request_beyond_budget_rejected():
    sched = serving.Scheduler(2, 1000, 10, 2)
    with pytest.raises(ValueError):
        sched.arrive(make_requests([100], [0.0])[0])


def test_percentile_nearest_rank():
    v = [5.0, 1.0, 3.0, 2.0, 4.0]
    assert serving.percentile(v, 50) == 3.0
    assert serving.percentile(v, 100) == 5.0
    assert serving.percentile(v, 20) == 1.0
    assert serving.percentile(list(range(1, 101)), 99) == 99
    assert np.isnan(serving.percentile([], 50))


def test_poisson_arrivals():
    t = serving.poisson_arrivals(20_000, rate=250.0, seed=3)
    assert np.all(np.diff(t) > 0)
    assert abs(np.mean(np.diff(t)) - 1 / 250.0) < 0.05 / 250.0


def test_failed_batch_fails_only_its_requests():
    """A batch whose device status reports an error (copied per batch) fails
    every request with a chunk in it, including a chunked request whose last
    chunk comes later; the requests of the other batches complete normally."""
    clock = SimClock()
    sizes = [300, 40, 40, 40, 40, 40, 40, 40]
    reqs = make_requests(sizes, [0.0] * len(sizes))
    sched = serving.Scheduler(n_slots=8, budget_bytes=1 << 30, max_batch_segments=100, max_batch_scenes=3)
    ex = SimExecutor(clock, sched, failing_batches={1})
    stats = serving.run(reqs, ex, sched, clock=clock, sleep=clock.sleep)
    bad = {c.req.rid for c in ex.batches[1]}
    assert bad and len(ex.batches) > 2
    assert {r.rid for r in reqs if r.failed} == bad
    assert all(r.done is not None for r in reqs)
    assert 0 in bad and len(ex.chunks[0]) > 2   # the long request: failed mid-stream, finished later
    assert stats["failed_requests"] == len(bad) and stats["requests"] == len(reqs)
