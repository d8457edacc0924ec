"""The serving loop on the GPU: every request's resident grid, produced in
mixed chunked batches, equals the oracle's volume of that request alone."""

import numpy as np
import pytest

from oracle import oracle
from paper_2009_09500_amd import serving, workloads
from tests.gpu_helpers import grid_host

pytestmark = pytest.mark.gpu


def test_mixed_requests_match_alone():
    reqs = []
    arrivals = serving.poisson_arrivals(24, rate=400.0, seed=7)
    for r in range(24):
        w = workloads.wireframe_request(r, volume=256, e_lo=1e3, e_hi=3e4)
        reqs.append(serving.Request(r, w["segs"], w["dims"], float(arrivals[r])))
    sched = serving.Scheduler(n_slots=6, budget_bytes=24 * 40_000, max_batch_segments=25_000,
                              max_batch_scenes=5)
    ex = serving.GpuExecutor((256, 256, 256), n_slots=6)
    bad = []

    def check(r, executor):
        if not np.array_equal(grid_host(executor.grid(r)), oracle.grid(r.segs, r.dims)):
            bad.append(r.rid)

    stats = serving.run(reqs, ex, sched, on_done=check)
    assert ex.status() == 0
    assert stats["requests"] == 24 and not bad, bad
    assert stats["batches"] > 1 and stats["latency_p99_ms"] >= stats["latency_p50_ms"] > 0
    assert sched.peak_bytes <= 24 * 40_000
