"""Full-size parity: the benchmark workloads in the launch configuration the
benchmark times, compared with the oracle's results (GPU).

The expected volumes come from tests/oracle_jobs.py (the CPU oracle run on
shards in the background) as SHA-256 digests of 16 MiB blocks; the GPU
volume is copied to the host and digested the same way, so every word is
compared.
"""

import numpy as np
import pytest

from oracle import oracle
from paper_2009_09500_amd import binding, workloads
from tests import oracle_jobs
from tests.gpu_helpers import dev, grid_host, to_dev, to_host

pytestmark = pytest.mark.gpu


def test_full_arbitrary_length_grid(oracle_jobs_dir):
    """4 194 304 segments -> cleared 2048^3 volume + counts, every word."""
    torch = pytest.importorskip("torch")
    c = workloads.arbitrary_length()
    segs = to_dev(c["segs"])
    n = segs.shape[0]
    grid = torch.empty(binding.grid_words(c["dims"]), dtype=torch.int32, device=dev())
    counts = torch.empty(n, dtype=torch.int32, device=dev())
    work = binding.workspace(binding.vox_grid_workspace_bytes(n, c["dims"]), dev())
    binding.vox_segments_to_grid(segs, c["dims"], grid, counts, binding.VOX_GRID_CLEAR, work)
    assert binding.vox_read_status(work) == binding.VOX_OK
    assert np.array_equal(to_host(counts), oracle.counts(c["segs"]))
    got = grid_host(grid)
    del grid, work
    exp = oracle_jobs.wait_result(oracle_jobs_dir, "arbitrary4m", timeout=100)
    dg = oracle_jobs.block_digests(got)
    bad = [i for i, (a, b) in enumerate(zip(dg, exp["digests"])) if a != b]
    assert len(dg) == len(exp["digests"]) and not bad, "blocks differ: %s" % bad[:10]
    assert oracle_jobs.popcount(got) == exp["popcount"]


def test_full_scenes_plain_calls(oracle_jobs_dir):
    """All 256 scenes of the batch workload, one plain call each."""
    torch = pytest.importorskip("torch")
    sc = workloads.scenes()
    exp = oracle_jobs.wait_result(oracle_jobs_dir, "scenes", timeout=100)
    bad = []
    for s, x in enumerate(sc):
        segs = to_dev(x["segs"])
        g = torch.empty(binding.grid_words(x["dims"]), dtype=torch.int32, device=dev())
        work = binding.workspace(binding.vox_grid_workspace_bytes(segs.shape[0], x["dims"]), dev())
        binding.vox_segments_to_grid(segs, x["dims"], g, None, binding.VOX_GRID_CLEAR, work)
        if oracle_jobs.block_digests(grid_host(g)) != exp["digests"][s]:
            bad.append(s)
    assert not bad, "scenes differ: %s" % bad[:10]


def test_full_scenes_one_batch(oracle_jobs_dir):
    """All 256 scenes of the batch workload in one batched launch sequence."""
    torch = pytest.importorskip("torch")
    sc = workloads.scenes()
    grids = [torch.empty(binding.grid_words(x["dims"]), dtype=torch.int32, device=dev())
             for x in sc]
    segs = [to_dev(x["segs"]) for x in sc]
    table = binding.scene_table([(s, x["dims"], g, None, binding.VOX_GRID_CLEAR)
                                 for s, x, g in zip(segs, sc, grids)])
    total = sum(int(s.shape[0]) for s in segs)
    work = binding.workspace(binding.batch_workspace_bytes(total, len(sc)), dev())
    binding.vox_batch_scenes(torch.from_numpy(table).to(dev()), len(sc), total, work)
    assert binding.vox_read_status(work) == binding.VOX_OK
    assert not binding.vox_read_batch_info(work)[1]          # the brick kernels served every scene
    exp = oracle_jobs.wait_result(oracle_jobs_dir, "scenes", timeout=100)
    bad = [s for s, g in enumerate(grids)
           if oracle_jobs.block_digests(grid_host(g)) != exp["digests"][s]]
    assert not bad, "scenes differ: %s" % bad[:10]
