"""Brick-shape autotuning for the grid and batch paths.

The brick shape (LDS brick of 2^lx x 2^ly x 2^lz voxels) changes speed and
workspace size, never the output.  `tune_grid` times every compiled shape on
the caller's own segments and volume, keeps the fastest in a JSON cache keyed
by device, volume and segment-count bucket, and makes it the process-wide
tuning (vox_set_tuning); `apply` looks a configuration up in the cache
without timing anything.
"""

from __future__ import annotations

import json
import math
import os
import tempfile
import threading

SHAPES = [(8, 6, 5), (8, 6, 6), (7, 6, 6), (7, 7, 6)]

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


class TuneCache:
    """JSON file {key: {"shape": [lx, ly, lz], "ms": {shape: ms}}}."""

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
        if not e:
            return None
        shape = tuple(int(v) for v in e["shape"])
        return shape if shape in SHAPES else None

    def put(self, k: str, shape, times: dict):
        self.entries[k] = {"shape": list(shape),
                           "ms": {"%d,%d,%d" % s: round(t, 5) for s, t in times.items()}}

    def save(self):
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        fd, tmp = tempfile.mkstemp(dir=d or ".", prefix=".tune")
        with os.fdopen(fd, "w") as f:
            json.dump(self.entries, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def best_shape(times: dict):
    """Fastest shape; ties go to the earlier entry of SHAPES."""
    return min(times, key=lambda s: (times[s], SHAPES.index(s)))


def device_name(device=None) -> str:
    import torch
    return torch.cuda.get_device_name(device)


def _time_shape(segs, dims, grid, shape, reps: int, stream) -> float:
    import torch
    from . import binding
    binding.vox_set_tuning(shape)
    n = segs.shape[0]
    work = binding.workspace(binding.vox_grid_workspace_bytes(n, dims), segs.device)
    binding.vox_segments_to_grid(segs, dims, grid, None, binding.VOX_GRID_CLEAR, work,
                                 stream=stream)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        binding.vox_segments_to_grid(segs, dims, grid, None, binding.VOX_GRID_CLEAR, work,
                                     stream=stream)
    end.record(stream)
    end.synchronize()
    return start.elapsed_time(end) / reps


def tune_grid(segs, dims, reps: int = 3, shapes=None, cache: TuneCache | None = None,
              timer=None, device: str | None = None):
    """Times each shape on (segs, dims) with a scratch volume, stores the
    fastest in the cache, sets it as the process-wide tuning and returns
    (shape, {shape: ms}).  `timer(shape) -> ms` replaces the GPU timing
    (tests).  Plain calls of at most 16384 segments take the direct path,
    where the shape changes nothing: tune with more segments than that."""
    from . import binding
    shapes = list(shapes or SHAPES)
    cache = cache if cache is not None else TuneCache()
    times = {}
    with _lock:
        prev = binding.vox_get_tuning()
        try:
            if timer is None:
                import torch
                grid = torch.empty(binding.grid_words(dims), dtype=torch.int32, device=segs.device)
                stream = torch.cuda.current_stream(segs.device)
                for s in shapes:
                    times[s] = _time_shape(segs, dims, grid, s, reps, stream)
                del grid
            else:
                for s in shapes:
                    times[s] = float(timer(s))
        finally:
            binding.vox_set_tuning(prev if any(prev) else None)
        best = best_shape(times)
        dev = device if device is not None else device_name(segs.device)
        cache.put(key(dev, dims, segs.shape[0]), best, times)
        cache.save()
        binding.vox_set_tuning(best)
    return best, times


def apply(dims, n: int, device: str, cache: TuneCache | None = None):
    """Sets the cached shape for (device, dims, n) if there is one; returns
    it (None: the library default stays)."""
    from . import binding
    cache = cache if cache is not None else TuneCache()
    shape = cache.get(key(device, dims, n))
    if shape is not None:
        binding.vox_set_tuning(shape)
    return shape
