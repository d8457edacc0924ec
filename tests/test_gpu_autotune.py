"""Autotuning on the GPU: every candidate is timed, the choice is cached and
installed for its volume and count, and the volume made with it is the
oracle's (GPU)."""

import numpy as np
import pytest

from oracle import oracle
from paper_2009_09500_amd import autotune, binding, workloads
from tests.gpu_helpers import grid_host, to_dev

pytestmark = pytest.mark.gpu


def test_tune_then_grid(tmp_path):
    c = workloads.arbitrary_length(n=40_000, volume=512)
    segs = to_dev(c["segs"])
    cache = autotune.TuneCache(str(tmp_path / "tune.json"))
    try:
        best, times = autotune.tune_grid(segs, c["dims"], reps=1, cache=cache)
        assert set(times) == set(autotune.CANDIDATES) and all(t > 0 for t in times.values())
        t = binding.vox_tuning_cache_get(c["dims"], 40_000)
        assert (tuple(t.brick_lg), t.fill_wgs_per_cu) == (best[:3], best[3])
        dev = autotune.device_name(segs.device)
        assert autotune.TuneCache(cache.path).get(autotune.key(dev, c["dims"], 40_000)) == best
        g = binding.segments_to_grid(segs, c["dims"])
        assert np.array_equal(grid_host(g), oracle.grid(c["segs"], c["dims"]))
    finally:
        binding.vox_tuning_cache_clear()
