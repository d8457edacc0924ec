"""Serving loop for voxelization requests on one GPU.

Requests (a segment set and a volume each) arrive over time.  The engine

* admits a waiting request, first come first served, when a resident grid
  slot is free and its segment buffer fits the device-memory budget (the
  GPU executor measures it: free HBM once the grid slots, the batch
  workspace and the scene tables are allocated, less a reserve);
* uploads the admitted request's segments on a copy stream;
* forms batches at chunk granularity (continuous batching): every
  iteration takes up to `max_batch_segments` segments from the admitted
  requests, at most `max_batch_scenes` of them, so a large request is cut
  into chunks (its first chunk clears its grid, later chunks OR into it)
  and small requests that arrive meanwhile join the next iteration instead
  of waiting for the large one to finish (policy in Scheduler.form_batch);
* runs each batch as one vox_batch_scenes launch sequence on the compute
  stream, keeping up to `max_inflight` batches queued on the GPU while the
  host forms the next;
* copies each batch's device status word right after the batch, so a
  batch that reports an error (an end point outside the volume) fails the
  requests it served; they are reported as failed, the others as done;
* completes a request when the batch holding its last chunk has finished;
  its grid stays resident in its slot until the completion callback returns.

This applies the paper's observation that many segments per kernel call and
few calls are what load the GPU (Section 5, conclusions) to requests arriving
one by one.  The scheduling logic is independent of the GPU (an executor
object does the device work), so it is tested on the CPU with a simulated
executor.
"""

from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    segs: np.ndarray                  # host int32 [n, 6]
    dims: tuple
    arrival: float                    # seconds after the stream's start
    voxels: int = 0                   # sum of N + 1 (computed by run() if 0)
    admitted: float | None = None
    done: float | None = None
    slot: int | None = None
    next_seg: int = 0                 # segments already put into batches
    started: bool = False
    failed: bool = False              # a batch with one of its chunks reported an error
    dev: dict = field(default_factory=dict)   # executor's per-request state

    @property
    def n(self) -> int:
        return int(self.segs.shape[0])

    @property
    def seg_bytes(self) -> int:
        return 24 * self.n


@dataclass
class Chunk:
    req: Request
    lo: int
    hi: int
    first: bool                       # clears the grid
    last: bool                        # completes the request


class Scheduler:
    """Admission and chunk-level batch formation (host logic only)."""

    def __init__(self, n_slots: int, budget_bytes: int, max_batch_segments: int,
                 max_batch_scenes: int):
        if n_slots < 1 or max_batch_segments < 1 or max_batch_scenes < 1:
            raise ValueError("slots, batch segments and batch scenes must be >= 1")
        self.n_slots = n_slots
        self.budget = int(budget_bytes)
        self.max_batch_segments = int(max_batch_segments)
        self.max_batch_scenes = int(max_batch_scenes)
        self.waiting: collections.deque[Request] = collections.deque()
        self.active: list[Request] = []          # admitted, not complete
        self.free_slots = list(range(n_slots - 1, -1, -1))
        self.used_bytes = 0
        self.peak_bytes = 0

    def arrive(self, r: Request):
        if r.seg_bytes > self.budget:
            raise ValueError("request %d needs %d bytes, more than the whole budget"
                             % (r.rid, r.seg_bytes))
        self.waiting.append(r)

    def admit(self, now: float) -> list:
        """Admits waiting requests in arrival order while a slot and budget
        remain (no request overtakes an earlier one)."""
        out = []
        while self.waiting and self.free_slots:
            r = self.waiting[0]
            if self.used_bytes + r.seg_bytes > self.budget:
                break
            self.waiting.popleft()
            r.slot = self.free_slots.pop()
            r.admitted = now
            self.used_bytes += r.seg_bytes
            self.peak_bytes = max(self.peak_bytes, self.used_bytes)
            self.active.append(r)
            out.append(r)
        return out

    def form_batch(self) -> list:
        """Next batch of chunks within the batch's segment and scene limits.

        The oldest admitted request with segments left is always in the batch
        with at least a quarter of the segment room (so it progresses however
        many requests arrive); the rest of the room goes to the other
        requests, fewest remaining segments first (which keeps short requests
        from queueing behind long ones), and what they leave returns to the
        oldest."""
        cand = [r for r in self.active if not (r.started and r.next_seg == r.n)]
        if not cand:
            return []
        oldest = cand[0]
        reserve = min(oldest.n - oldest.next_seg, self.max_batch_segments // 4)
        room = self.max_batch_segments - reserve
        picks = []
        for r in sorted(cand[1:], key=lambda r: r.n - r.next_seg):
            if len(picks) == self.max_batch_scenes - 1:
                break
            left = r.n - r.next_seg
            if left > 0 and room == 0:
                break
            take = min(left, room)
            picks.append((r, take))
            room -= take
        picks.insert(0, (oldest, min(oldest.n - oldest.next_seg, reserve + room)))
        chunks = []
        for r, take in picks:
            chunks.append(Chunk(r, r.next_seg, r.next_seg + take, not r.started,
                                r.next_seg + take == r.n))
            r.started = True
            r.next_seg += take
        return chunks

    def complete(self, chunks: list, now: float, failed: bool = False) -> list:
        """Marks the requests whose last chunk was in `chunks` as done and
        frees their slot and budget; returns them.  failed: the batch of
        these chunks reported an error, so every request it served is marked
        failed (one with chunks still to come completes, failed, with its
        last chunk)."""
        done = []
        for c in chunks:
            if failed:
                c.req.failed = True
            if c.last:
                r = c.req
                r.done = now
                self.active.remove(r)
                self.free_slots.append(r.slot)
                self.used_bytes -= r.seg_bytes
                done.append(r)
        return done

    def idle(self) -> bool:
        return not self.waiting and not self.active


def percentile(values, q: float) -> float:
    """q-th percentile (nearest rank, q in (0, 100])."""
    v = sorted(values)
    if not v:
        return float("nan")
    k = max(1, int(math.ceil(q / 100.0 * len(v))))
    return float(v[k - 1])


def run(requests, executor, scheduler: Scheduler, max_inflight: int = 2,
        on_done=None, clock=time.perf_counter, sleep=time.sleep,
        poll_sleep: float = 20e-6) -> dict:
    """Serves `requests` (sorted by arrival time, seconds from the start) in
    real time on `executor`; returns throughput and latency statistics.
    `on_done(request, executor)` runs when a request completes, before its
    slot is reused."""
    reqs = sorted(requests, key=lambda r: r.arrival)
    for r in reqs:
        if r.voxels == 0 and r.n:
            d = np.abs(r.segs[:, 3:].astype(np.int64) - r.segs[:, :3])
            r.voxels = int((d.max(axis=1) + 1).sum())
    inflight: collections.deque = collections.deque()
    t0 = clock()
    i = 0
    batches = 0
    batch_segments = []
    finished = []
    while i < len(reqs) or not scheduler.idle() or inflight:
        now = clock() - t0
        while i < len(reqs) and reqs[i].arrival <= now:
            scheduler.arrive(reqs[i])
            i += 1
        for r in scheduler.admit(now):
            executor.upload(r)
        progressed = False
        while inflight and executor.poll(inflight[0][1]):
            chunks, handle = inflight.popleft()
            failed = executor.batch_status(handle) != 0
            for r in scheduler.complete(chunks, clock() - t0, failed=failed):
                if on_done is not None:
                    on_done(r, executor)
                executor.release(r)
                finished.append(r)
            progressed = True
        if len(inflight) < max_inflight:
            chunks = scheduler.form_batch()
            if chunks:
                inflight.append((chunks, executor.launch(chunks)))
                batches += 1
                batch_segments.append(sum(c.hi - c.lo for c in chunks))
                progressed = True
        if not progressed:
            sleep(poll_sleep)
    makespan = clock() - t0
    good = [r for r in finished if not r.failed]
    lat = [r.done - r.arrival for r in good]
    voxels = sum(r.voxels for r in good)
    return {
        "requests": len(finished),
        "failed_requests": len(finished) - len(good),
        "makespan_s": makespan,
        "requests_per_s": len(good) / makespan if makespan > 0 else float("nan"),
        "voxels_per_s": voxels / makespan if makespan > 0 else float("nan"),
        "latency_p50_ms": 1e3 * percentile(lat, 50),
        "latency_p99_ms": 1e3 * percentile(lat, 99),
        "latency_mean_ms": 1e3 * float(np.mean(lat)) if lat else float("nan"),
        "batches": batches,
        "mean_batch_segments": float(np.mean(batch_segments)) if batch_segments else 0.0,
        "peak_segment_bytes": scheduler.peak_bytes,
    }


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process of `rate` per second."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


class GpuExecutor:
    """Device side of the serving loop: resident grid slots, a copy stream
    for segment uploads and a compute stream for batches (libvox through the
    binding; nothing here computes voxels).

    Everything the batches need is allocated once, up front: the grid slots,
    one batch workspace for `max_batch_segments` segments over
    `max_batch_scenes` scenes (vox_workspace_bytes), and a ring of device
    scene tables with pinned staging and a pinned status word per in-flight
    batch.  `admission_budget()` is then what free HBM remains for the
    requests' segment buffers, measured, less `reserve_bytes`."""

    def __init__(self, dims, n_slots: int, max_batch_segments: int = 2_000_000,
                 max_batch_scenes: int = 32, max_inflight: int = 2, device=None, tuning=None,
                 reserve_bytes: int = 1 << 30):
        import torch
        from . import binding
        self.torch = torch
        self.binding = binding
        binding.load()
        self.device = device or torch.device("cuda:0")
        self.dims = tuple(int(d) for d in dims)
        self.max_batch_segments = int(max_batch_segments)
        self.max_batch_scenes = int(max_batch_scenes)
        self.tuning = tuning
        self.copy_stream = torch.cuda.Stream(device=self.device)
        self.compute = torch.cuda.Stream(device=self.device)
        with torch.cuda.stream(self.compute):
            self.grids = [torch.empty(binding.grid_words(self.dims), dtype=torch.int32,
                                      device=self.device) for _ in range(n_slots)]
            self.work = binding.workspace(
                binding.batch_workspace_bytes(self.max_batch_segments, self.max_batch_scenes), self.device)
        ring = max_inflight + 1
        table_bytes = 48 * self.max_batch_scenes
        self.d_tables = [torch.empty(table_bytes, dtype=torch.uint8, device=self.device) for _ in range(ring)]
        self.h_tables = [torch.empty(table_bytes, dtype=torch.uint8).pin_memory() for _ in range(ring)]
        self.h_status = torch.zeros(ring, dtype=torch.int32).pin_memory()
        self.status_word = self.work[:4].view(torch.int32)
        assert self.status_word.data_ptr() == binding.vox_device_status(self.work)
        self.slot = 0
        self.reserve = int(reserve_bytes)
        torch.cuda.synchronize(self.device)

    def admission_budget(self) -> int:
        """Bytes of request segment buffers that fit in the free HBM left
        (measured now), less the reserve."""
        free, _ = self.torch.cuda.mem_get_info(self.device)
        return max(int(free) - self.reserve, 0)

    @staticmethod
    def pin(segs: np.ndarray):
        """Pinned host copy of a request's segments for upload: int16 when
        every coordinate fits (half the bytes over PCIe; volumes up to 32768
        a side), else int32."""
        import torch
        a = np.ascontiguousarray(segs)
        if a.size and a.min() >= -32768 and a.max() <= 32767:
            a = a.astype(np.int16)
        return torch.from_numpy(a).pin_memory()

    def upload(self, r: Request):
        """Copies the request's segments to the device on the copy stream.
        int16 uploads are widened to the library's int32 segments on the
        device (a dtype conversion on the copy stream)."""
        torch = self.torch
        host = r.dev.get("pinned")
        if host is None:
            host = self.pin(r.segs)
        with torch.cuda.stream(self.copy_stream):
            d = torch.empty((max(r.n, 1), 6), dtype=torch.int32, device=self.device)
            if host.dtype == torch.int16:
                staged = torch.empty((max(r.n, 1), 6), dtype=torch.int16, device=self.device)
                staged[:r.n].copy_(host, non_blocking=True)
                d[:r.n].copy_(staged[:r.n])
                r.dev["staged"] = staged
            else:
                d[:r.n].copy_(host, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.copy_stream)
        r.dev.update(d_segs=d, uploaded=ev, host=host, upload_bytes=host.numel() * host.element_size())

    def launch(self, chunks):
        torch, binding = self.torch, self.binding
        if len(chunks) > self.max_batch_scenes:
            raise ValueError("batch of %d chunks, the executor holds %d" % (len(chunks), self.max_batch_scenes))
        scenes = []
        for c in chunks:
            r = c.req
            if c.first:
                self.compute.wait_event(r.dev["uploaded"])
            segs = r.dev["d_segs"][c.lo:c.hi]
            flags = binding.VOX_GRID_CLEAR if c.first else 0
            scenes.append((segs, self.dims, self.grids[r.slot], None, flags))
        total = sum(c.hi - c.lo for c in chunks)
        if total > self.max_batch_segments:
            raise ValueError("batch of %d segments, the executor holds %d" % (total, self.max_batch_segments))
        k = self.slot
        self.slot = (self.slot + 1) % len(self.d_tables)
        table = binding.scene_table(scenes)
        self.h_tables[k][:table.size].copy_(torch.from_numpy(table))
        with torch.cuda.stream(self.compute):
            self.d_tables[k][:table.size].copy_(self.h_tables[k][:table.size], non_blocking=True)
            binding.vox_batch_scenes(self.d_tables[k], len(scenes), total, self.work, tuning=self.tuning,
                                     stream=self.compute)
            # This batch's status word, before the next batch rewrites it.
            self.h_status[k:k + 1].copy_(self.status_word, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.compute)
        for c in chunks:
            c.req.dev["d_segs"].record_stream(self.compute)
        return (ev, k)

    def poll(self, handle) -> bool:
        return handle[0].query()

    def batch_status(self, handle) -> int:
        """Device status bits of a finished batch (0: no error)."""
        return int(self.h_status[handle[1]])

    def release(self, r: Request):
        r.dev.pop("d_segs", None)
        r.dev.pop("staged", None)
        r.dev.pop("uploaded", None)

    def grid(self, r: Request):
        return self.grids[r.slot]

    def status(self) -> int:
        return self.binding.vox_read_status(self.work, stream=self.compute)
