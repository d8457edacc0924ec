"""Batched scenes (vox_batch_plan + vox_batch_scenes) against the oracle, and
HIP-graph capture and replay of a batch (GPU)."""

import numpy as np
import pytest

from oracle import oracle
from paper_2009_09500_amd import binding, workloads
from tests.gpu_helpers import dev, grid_host, to_dev, to_host

pytestmark = pytest.mark.gpu

SHAPES = [(8, 6, 5), (8, 6, 6), (7, 6, 6), (7, 7, 6)]


def random_in(dims, n, seed):
    rng = np.random.default_rng(seed)
    p = [np.stack([rng.integers(0, d, n) for d in dims], 1) for _ in range(2)]
    return np.concatenate(p, 1).astype(np.int32)


class Batch:
    """Device buffers of a batch of scenes and their expected volumes."""

    def __init__(self, specs, garbage=0x5A5A5A5A):
        import torch
        self.specs = specs          # (segs np, dims, flags, base np or None, want_counts)
        self.segs, self.grids, self.counts = [], [], []
        for segs, dims, flags, base, want in specs:
            self.segs.append(to_dev(segs) if segs.shape[0] else
                             torch.zeros((0, 6), dtype=torch.int32, device=dev()))
            self.grids.append(torch.empty(binding.grid_words(dims), dtype=torch.int32, device=dev()))
            self.counts.append(torch.empty(max(segs.shape[0], 1), dtype=torch.int32, device=dev())
                               if want else None)
        self.reset(garbage)

    def reset(self, garbage=0x5A5A5A5A):
        import torch
        for (segs, dims, flags, base, want), g in zip(self.specs, self.grids):
            if base is not None:
                g.copy_(torch.from_numpy(base.view(np.int32)).to(dev()))
            else:
                g.fill_(garbage - (1 << 32) if garbage >= (1 << 31) else garbage)

    def scenes(self):
        return [(s, d, g, c, f) for s, (segs, d, f, base, want), g, c in
                zip(self.segs, self.specs, self.grids, self.counts)]

    def check(self, skip=None):
        skip = skip or {}
        for i, ((segs, dims, flags, base, want), g, c) in enumerate(
                zip(self.specs, self.grids, self.counts)):
            keep = np.delete(segs, skip.get(i, []), axis=0)
            if flags & binding.VOX_GRID_CLEAR:
                exp = oracle.grid(keep, dims)
            else:
                exp = oracle.grid(keep, dims, base=base)
            got = grid_host(g)
            if not np.array_equal(got, exp):
                bad = np.flatnonzero(got != exp)
                raise AssertionError("scene %d: %d words differ, first %s"
                                     % (i, bad.size, bad[:5].tolist()))
            if want and segs.shape[0]:
                assert np.array_equal(to_host(c)[:segs.shape[0]], oracle.counts(segs)), i


def run_batch(b, stream=None):
    import torch
    table, launch = binding.vox_batch_plan(b.scenes())
    d_table = torch.from_numpy(table).to(dev())
    work = binding.workspace(launch.work_bytes, dev())
    binding.vox_batch_scenes(d_table, launch, work, stream=stream)
    return binding.vox_read_status(work, stream=stream), launch


def mixed_specs(seed=0):
    rng = np.random.default_rng(seed)
    specs = []
    for i, dims in enumerate([(64, 64, 64), (512, 512, 512), (128, 96, 40), (256, 256, 256),
                              (96, 40, 20), (64, 16, 8), (320, 200, 70)]):
        n = int(rng.integers(100, 20000)) if dims != (512, 512, 512) else 60000
        segs = random_in(dims, n, seed * 100 + i)
        flags = binding.VOX_GRID_CLEAR
        base = None
        if i == 4:                      # OR into existing contents
            flags = 0
            base = rng.integers(0, 2**32, size=binding.grid_words(dims), dtype=np.uint32)
            base &= rng.integers(0, 2**32, size=base.size, dtype=np.uint32)
        specs.append((segs, dims, flags, base, i % 2 == 0))
    specs.append((np.zeros((0, 6), np.int32), (128, 64, 64), binding.VOX_GRID_CLEAR, None, False))
    return specs


def test_mixed_batch():
    b = Batch(mixed_specs())
    status, launch = run_batch(b)
    assert status == binding.VOX_OK
    b.check()


@pytest.mark.skip(reason="a batch holding a 4-byte-aligned (not 8-byte-aligned) segment array "
                         "hung the GPU once and the cause was not shown; the brick kernels now take "
                         "only 8-byte-aligned arrays and vox_batch_plan rejects the others")
def test_unaligned_segments_in_batch():
    import torch
    dims = (128, 128, 64)
    segs = random_in(dims, 3001, 3)
    buf = torch.empty(6 * segs.shape[0] + 1, dtype=torch.int32, device=dev())
    buf[1:].copy_(torch.from_numpy(segs.reshape(-1)).to(dev()))
    view = buf[1:].view(-1, 6)            # 4-byte but not 8-byte aligned
    assert view.data_ptr() % 8 == 4
    g = torch.empty(binding.grid_words(dims), dtype=torch.int32, device=dev())
    g2 = torch.empty_like(g)
    table, launch = binding.vox_batch_plan([(view, dims, g, None, 1),
                                            (to_dev(segs), dims, g2, None, 1)])
    work = binding.workspace(launch.work_bytes, dev())
    binding.vox_batch_scenes(torch.from_numpy(table).to(dev()), launch, work)
    assert binding.vox_read_status(work) == binding.VOX_OK
    exp = oracle.grid(segs, dims)
    assert np.array_equal(grid_host(g), exp) and np.array_equal(grid_host(g2), exp)


def test_out_of_volume_in_one_scene():
    specs = mixed_specs(1)[:3]
    segs = specs[1][0].copy()
    segs[5] = [0, 0, 0, 512, 3, 3]
    segs[77] = [-2, 0, 0, 4, 4, 4]
    specs[1] = (segs,) + specs[1][1:]
    b = Batch(specs)
    status, _ = run_batch(b)
    assert status == binding.VOX_ERR_OUT_OF_RANGE
    b.check(skip={1: [5, 77]})


@pytest.mark.parametrize("lg", SHAPES)
def test_batch_every_brick_shape(lg):
    binding.vox_set_tuning(lg)
    try:
        b = Batch(mixed_specs(2)[:6])
        status, launch = run_batch(b)
        assert tuple(launch.brick_lg) == lg
        assert status == binding.VOX_OK
        b.check()
    finally:
        binding.vox_set_tuning(None)


def test_batch_equals_plain_calls():
    """The scene workload's first 24 scenes: batch and plain calls agree word
    for word (and with the oracle)."""
    import torch
    sc = workloads.scenes(n_scenes=24)
    specs = [(x["segs"], x["dims"], binding.VOX_GRID_CLEAR, None, True) for x in sc]
    b = Batch(specs)
    status, _ = run_batch(b)
    assert status == binding.VOX_OK
    for x, g, c in zip(sc, b.grids, b.counts):
        pg, pc = binding.segments_to_grid(to_dev(x["segs"]), x["dims"], want_counts=True)
        assert torch.equal(pg, g) and torch.equal(pc, c)
    b.check()


def test_table_that_does_not_fit_writes_nothing():
    import torch
    small = Batch(mixed_specs(3)[:2])
    big = Batch(mixed_specs(3)[:5])
    _, launch_small = binding.vox_batch_plan(small.scenes())
    table_big, launch_big = binding.vox_batch_plan(big.scenes())
    assert launch_big.rows > launch_small.rows
    work = binding.workspace(max(launch_small.work_bytes, launch_big.work_bytes), dev())
    binding.vox_batch_scenes(torch.from_numpy(table_big).to(dev()), launch_small, work)
    assert binding.vox_read_status(work) == binding.VOX_ERR_BATCH_MISMATCH
    for g in big.grids[:4]:                       # scene 4 ORs into a random base
        assert (grid_host(g) == 0x5A5A5A5A).all()


def test_graph_capture_and_replay():
    """One capture, replays with eager work in between, then a second table
    written to the same device address and replayed under the same graph."""
    import torch
    a = Batch(mixed_specs(4)[:5])
    bspecs = [(random_in(d, 7000, 40 + i), d, binding.VOX_GRID_CLEAR, None, True)
              for i, d in enumerate([(256, 128, 64), (64, 64, 64), (512, 256, 128)])]
    b = Batch(bspecs)
    table_a, launch_a = binding.vox_batch_plan(a.scenes())
    table_b, launch_b = binding.vox_batch_plan(b.scenes())
    bound = binding.VoxBatchLaunch()
    binding.vox_batch_launch_cover(bound, launch_a)
    binding.vox_batch_launch_cover(bound, launch_b)
    d_table = torch.zeros(int(bound.table_bytes), dtype=torch.uint8, device=dev())
    d_table[:table_a.size].copy_(torch.from_numpy(table_a).to(dev()))
    work = binding.workspace(bound.work_bytes, dev())

    binding.vox_batch_scenes(d_table, bound, work)          # eager, before capture
    assert binding.vox_read_status(work) == binding.VOX_OK
    a.check()

    s = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=s):
        binding.vox_batch_scenes(d_table, bound, work)
    torch.cuda.synchronize()
    for rep in range(3):
        a.reset(garbage=0x0F0F0F0F + rep)
        x = torch.randn(1 << 20, device=dev()).sum()        # unrelated eager work
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert binding.vox_read_status(work) == binding.VOX_OK
        a.check()
        del x
    d_table[:table_b.size].copy_(torch.from_numpy(table_b).to(dev()))
    torch.cuda.synchronize()
    for rep in range(2):
        b.reset(garbage=0x33333333 + rep)
        graph.replay()
        torch.cuda.synchronize()
        assert binding.vox_read_status(work) == binding.VOX_OK
        b.check()
