"""Seeded random batches against the oracle (GPU): volumes of assorted
shapes, every compiled brick shape (per-call tuning), both lengths N,
cleared volumes and volumes ORed into, dense spots whose bricks the fill
cuts into several work items, and segments across the whole volume whose
walks the scatter cuts into parts; every volume and every count compared
word by word, then the same scenes as plain calls in the compact
workspace."""

import numpy as np
import pytest

from oracle import oracle
from paper_2009_09500_amd import binding
from tests.gpu_helpers import dev, grid_host, to_dev, to_host
from tests.test_gpu_batch import Batch, run_batch

pytestmark = pytest.mark.gpu

SHAPES = [(8, 6, 5), (8, 6, 6), (7, 6, 6), (7, 7, 6)]


def random_scene(rng):
    dims = (32 * int(rng.integers(1, 17)), int(rng.integers(1, 300)), int(rng.integers(1, 160)))
    d = np.array(dims)
    kind = int(rng.integers(0, 3))
    n = int(rng.integers(0, 5000))
    if kind == 1:     # a dense spot: short segments in a small box
        box = np.minimum(d, rng.integers(4, 48, 3))
        o = np.array([rng.integers(0, x - b + 1) for x, b in zip(d, box)])
        p0 = o + np.stack([rng.integers(0, b, n) for b in box], 1)
        p1 = np.clip(p0 + rng.integers(-5, 6, (n, 3)), o, o + box - 1)
    elif kind == 2:   # across the volume: from one face to the opposite one
        p0 = np.stack([rng.integers(0, x, n) for x in d], 1)
        p1 = np.stack([rng.integers(0, x, n) for x in d], 1)
        ax = rng.integers(0, 3, n)
        p0[np.arange(n), ax] = 0
        p1[np.arange(n), ax] = d[ax] - 1
    else:
        p0 = np.stack([rng.integers(0, x, n) for x in d], 1)
        p1 = np.stack([rng.integers(0, x, n) for x in d], 1)
    segs = np.concatenate([p0, p1], 1).astype(np.int32).reshape(-1, 6)
    flags = binding.VOX_GRID_EUCLID if rng.random() < 0.3 else 0
    base = None
    if rng.random() < 0.7:
        flags |= binding.VOX_GRID_CLEAR
    else:
        base = rng.integers(0, 2**32, size=binding.grid_words(dims), dtype=np.uint32)
        base &= rng.integers(0, 2**32, size=base.size, dtype=np.uint32)
        nbits = dims[0] * dims[1] * dims[2]
        if nbits % 32:
            base[-1] &= (1 << (nbits % 32)) - 1
    return segs, dims, flags, base, bool(rng.random() < 0.5)


@pytest.mark.parametrize("seed", range(32))
def test_random_batch(seed):
    rng = np.random.default_rng(7000 + seed)
    specs = [random_scene(rng) for _ in range(int(rng.integers(1, 7)))]
    b = Batch(specs)
    lg = SHAPES[seed % len(SHAPES)]
    status, work = run_batch(b, tuning=binding.make_tuning(brick_lg=lg))
    assert status == binding.VOX_OK
    b.check()


@pytest.mark.parametrize("seed", range(12))
def test_random_plain_calls(seed):
    """Single scenes of the same kinds as plain grid calls in the compact
    workspace (at least 16 385 segments, so they take the brick path)."""
    import torch
    rng = np.random.default_rng(8000 + seed)
    segs, dims, flags, base, want = random_scene(rng)
    while segs.shape[0] < 16385:
        more, _, _, _, _ = random_scene(np.random.default_rng(rng.integers(1 << 30)))
        more = more % np.array(list(dims) * 2, dtype=np.int32)
        segs = np.concatenate([segs, more])
    n = len(segs)
    work = binding.workspace(binding.vox_workspace_bytes(binding.VOX_OP_GRID, n, 1), dev())
    g = to_dev((base if base is not None else np.zeros(binding.grid_words(dims), np.uint32)).view(np.int32))
    c = torch.empty(n, dtype=torch.int32, device=dev())
    binding.vox_segments_to_grid(to_dev(segs), dims, g, c, flags, work)
    assert binding.vox_read_status(work) == binding.VOX_OK
    euclid = bool(flags & binding.VOX_GRID_EUCLID)
    grid_fn = oracle.grid_euclid if euclid else oracle.grid
    exp = grid_fn(segs, dims, base=None if flags & binding.VOX_GRID_CLEAR else base)
    got = grid_host(g)
    if not np.array_equal(got, exp):
        bad = np.flatnonzero(got != exp)
        raise AssertionError("%d words differ, first %s" % (bad.size, bad[:5].tolist()))
    exp_c = np.diff(oracle.offsets_euclid(segs)) if euclid else oracle.counts(segs)
    assert np.array_equal(to_host(c), exp_c)
