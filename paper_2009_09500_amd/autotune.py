"""Launch-shape autotuning for the grid and batch paths.

A candidate is a brick shape (LDS brick of 2^lx x 2^ly x 2^lz voxels) with a
number of fill workgroups per compute unit; it changes speed and workspace
size, never the output.  `tune_grid` times every candidate on the caller's
own segments and volume, each as a one-scene batch with its own per-call
tuning (no process-wide state changes while timing), keeps the fastest in a
JSON cache keyed by device, volume and segment-count bucket, and installs it
in the library's autotune cache for that volume and count
(vox_tuning_cache_set), which plain grid calls consult.  `apply` installs a
cached choice without timing anything.
"""

from __future__ import annotations

import json
import math
import os
import tempfile
import threading

# (lx, ly, lz, fill workgroups per CU; 0 = the shape's default).
CANDIDATES = [(8, 6, 5, 2), (8, 6, 5, 1), (8, 6, 6, 0), (7, 6, 6, 2), (7, 6, 6, 1), (7, 7, 6, 0)]
SHAPES = sorted({c[:3] for c in CANDIDATES})

_lock = threading.Lock()


def cache_path() -> str:
    p = os.environ.get("VOX_TUNE_CACHE")
    if p:
        return p
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "paper_2009_09500_amd", "brick_tuning.json")


def key(device: str, dims, n: int) -> str:
    """Cache key: device name, exact volume, segment count to the nearest
    power of two (timings move little within a factor of two)."""
    b = int(round(math.log2(n))) if n > 0 else -1
    return "%s|%dx%dx%d|n~2^%d" % (device, int(dims[0]), int(dims[1]), int(dims[2]), b)


def _name(c) -> str:
    return "%d,%d,%d,%d" % tuple(c)


class TuneCache:
    """JSON file {key: {"candidate": [lx, ly, lz, wgs], "ms": {name: ms}}}."""

    def __init__(self, path: str | None = None):
        self.path = path or cache_path()
        self.entries = {}
        if os.path.exists(self.path):
            try:
                with open(self.path) as f:
                    self.entries = json.load(f)
            except (OSError, ValueError):
                self.entries = {}

    def get(self, k: str):
        e = self.entries.get(k)
        if not isinstance(e, dict) or "candidate" not in e:
            return None
        c = tuple(int(v) for v in e["candidate"])
        return c if c in CANDIDATES else None

    def put(self, k: str, cand, times: dict):
        self.entries[k] = {"candidate": list(cand),
                           "ms": {_name(c): round(t, 5) for c, t in times.items()}}

    def save(self):
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        fd, tmp = tempfile.mkstemp(dir=d or ".", prefix=".tune")
        with os.fdopen(fd, "w") as f:
            json.dump(self.entries, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def best_candidate(times: dict):
    """Fastest candidate; ties go to the earlier entry of CANDIDATES."""
    return min(times, key=lambda c: (times[c], CANDIDATES.index(c)))


def tuning_of(cand):
    from . import binding
    return binding.make_tuning(cand[:3], cand[3])


def device_name(device=None) -> str:
    import torch
    return torch.cuda.get_device_name(device)


def _time_candidate(segs, dims, grid, cand, reps: int, stream) -> float:
    """Mean ms of one cleared one-scene batch with this candidate's tuning
    (a workspace big enough that the brick kernels serve the scene)."""
    import torch
    from . import binding
    n = int(segs.shape[0])
    tuning = tuning_of(cand)
    d_scenes = torch.from_numpy(binding.scene_table([(segs, dims, grid, None, binding.VOX_GRID_CLEAR)])).to(
        segs.device)
    nbytes = binding.batch_workspace_bytes(n, 1)
    work = binding.workspace(nbytes, segs.device)
    binding.vox_batch_scenes(d_scenes, 1, n, work, tuning=tuning, stream=stream)
    pieces, direct_all = binding.vox_read_batch_info(work, stream=stream)
    if direct_all:  # records did not fit: give them room
        work = binding.workspace(nbytes + 16 * pieces, segs.device)
        binding.vox_batch_scenes(d_scenes, 1, n, work, tuning=tuning, stream=stream)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        binding.vox_batch_scenes(d_scenes, 1, n, work, tuning=tuning, stream=stream)
    end.record(stream)
    end.synchronize()
    return start.elapsed_time(end) / reps


def tune_grid(segs, dims, reps: int = 3, candidates=None, cache: TuneCache | None = None,
              timer=None, device: str | None = None, install: bool = True):
    """Times each candidate on (segs, dims) with a scratch volume, stores the
    fastest in the cache and (install) in the library's cache for (dims,
    n), and returns (candidate, {candidate: ms}).  `timer(candidate) -> ms`
    replaces the GPU timing (tests).  Plain calls of at most 16384 segments
    take the direct path, where the tuning changes nothing."""
    from . import binding
    cands = list(candidates or CANDIDATES)
    cache = cache if cache is not None else TuneCache()
    times = {}
    with _lock:
        if timer is None:
            import torch
            grid = torch.empty(binding.grid_words(dims), dtype=torch.int32, device=segs.device)
            stream = torch.cuda.current_stream(segs.device)
            for c in cands:
                times[c] = _time_candidate(segs, dims, grid, c, reps, stream)
            del grid
        else:
            for c in cands:
                times[c] = float(timer(c))
        best = best_candidate(times)
        dev = device if device is not None else device_name(segs.device)
        cache.put(key(dev, dims, segs.shape[0]), best, times)
        cache.save()
        if install:
            binding.vox_tuning_cache_set(dims, int(segs.shape[0]), tuning_of(best))
    return best, times


def apply(dims, n: int, device: str, cache: TuneCache | None = None):
    """Installs the cached candidate for (device, dims, n) in the library's
    cache if there is one; returns it (None: the library default stays)."""
    from . import binding
    cache = cache if cache is not None else TuneCache()
    cand = cache.get(key(device, dims, n))
    if cand is not None:
        binding.vox_tuning_cache_set(dims, n, tuning_of(cand))
    return cand
