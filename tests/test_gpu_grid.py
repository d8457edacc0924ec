"""HIP bit-volumes against the CPU oracle, word by word (GPU)."""

import numpy as np
import pytest

from oracle import oracle
from paper_2009_09500_amd import binding, workloads
from tests.gpu_helpers import dev, grid_host, to_dev, to_host

pytestmark = pytest.mark.gpu


def assert_grid(segs, dims, base=None):
    torch = pytest.importorskip("torch")
    s = to_dev(segs)
    if base is None:
        g, c = binding.segments_to_grid(s, dims, want_counts=True)
    else:
        g = to_dev(base.view(np.int32))
        g, c = binding.segments_to_grid(s, dims, grid=g, want_counts=True)
    got = grid_host(g)
    exp = oracle.grid(segs, dims, base=base)
    if not np.array_equal(got, exp):
        bad = np.flatnonzero(got != exp)
        raise AssertionError("%d words differ, first %s" % (bad.size, bad[:5].tolist()))
    assert np.array_equal(to_host(c), oracle.counts(segs))


def random_in(dims, n, seed):
    rng = np.random.default_rng(seed)
    p = [np.stack([rng.integers(0, d, n) for d in dims], 1) for _ in range(2)]
    return np.concatenate(p, 1).astype(np.int32)


def test_small_uniform_256():
    c = workloads.small_uniform()
    assert_grid(c["segs"], c["dims"])


def test_single_diagonal_256():
    c = workloads.single_diagonal()
    assert_grid(c["segs"], c["dims"])


@pytest.mark.parametrize("dims", [(37, 5, 3), (100, 30, 7), (1, 1, 1), (33, 64, 2), (64, 64, 64)])
def test_odd_volumes(dims):
    assert_grid(random_in(dims, 500, sum(dims)), dims)


def test_or_into_existing():
    dims = (96, 40, 20)
    rng = np.random.default_rng(9)
    base = rng.integers(0, 2**32, size=binding.grid_words(dims), dtype=np.uint32)
    base &= rng.integers(0, 2**32, size=base.size, dtype=np.uint32)   # ~25% ones
    nbits = dims[0] * dims[1] * dims[2]
    if nbits % 32:
        base[-1] &= (1 << (nbits % 32)) - 1
    assert_grid(random_in(dims, 800, 10), dims, base=base)


def test_arbitrary_length_scaled():
    c = workloads.arbitrary_length(n=100_000, volume=512)
    assert_grid(c["segs"], c["dims"])


def test_wireframe_request():
    q = workloads.wireframe_request(3)
    assert_grid(q["segs"], q["dims"])


def test_scenes_plain_calls():
    for sc in workloads.scenes(n_scenes=6, seed=77):
        assert_grid(sc["segs"], sc["dims"])


def test_out_of_volume_segment_is_skipped():
    torch = pytest.importorskip("torch")
    dims = (64, 64, 64)
    segs = random_in(dims, 200, 5)
    bad = segs.copy()
    bad[17] = [0, 0, 0, 64, 10, 10]
    bad[99] = [-1, 3, 3, 5, 5, 5]
    g = torch.empty(binding.grid_words(dims), dtype=torch.int32, device=dev())
    work = binding.workspace(binding.vox_grid_workspace_bytes(len(bad), dims), dev())
    binding.vox_segments_to_grid(to_dev(bad), dims, g, None, binding.VOX_GRID_CLEAR, work)
    assert binding.vox_read_status(work) == binding.VOX_ERR_OUT_OF_RANGE
    keep = np.delete(segs, [17, 99], axis=0)
    assert np.array_equal(grid_host(g), oracle.grid(keep, dims))


@pytest.mark.parametrize("euclid", [False, True])
def test_out_of_volume_segments_brick_path(euclid):
    """Segments with an end point outside the volume in a brick-path call
    (20 000 segments): the status reports them, the volume holds the others'
    voxels, and a second call on the same workspace without them reports OK
    (the status word starts from zero in every call)."""
    torch = pytest.importorskip("torch")
    dims = (256, 128, 64)
    segs = random_in(dims, 20_000, 15)
    bad = segs.copy()
    bad[17] = [0, 0, 0, 256, 10, 10]
    bad[9_999] = [-1, 3, 3, 5, 5, 5]
    bad[19_999] = [5, 5, 5, 5, 5, 64]
    flags = binding.VOX_GRID_CLEAR | (binding.VOX_GRID_EUCLID if euclid else 0)
    g = torch.empty(binding.grid_words(dims), dtype=torch.int32, device=dev())
    c = torch.empty(len(bad), dtype=torch.int32, device=dev())
    work = binding.workspace(binding.vox_grid_workspace_bytes(len(bad), dims), dev())
    binding.vox_segments_to_grid(to_dev(bad), dims, g, c, flags, work)
    assert binding.vox_read_status(work) == binding.VOX_ERR_OUT_OF_RANGE
    keep = np.delete(segs, [17, 9_999, 19_999], axis=0)
    grid_fn, counts_fn = (oracle.grid_euclid, oracle.counts_euclid) if euclid else (oracle.grid, oracle.counts)
    assert np.array_equal(grid_host(g), grid_fn(keep, dims))
    exp_c = counts_fn(bad)
    if euclid:
        exp_c[[17, 9_999, 19_999]] = 0   # a grid segment outside the volume counts 0 with the Euclidean N
    assert np.array_equal(to_host(c), exp_c)
    binding.vox_segments_to_grid(to_dev(keep), dims, g, None, flags, work)
    assert binding.vox_read_status(work) == binding.VOX_OK
    assert np.array_equal(grid_host(g), grid_fn(keep, dims))


def long_diagonals(dims, n, seed):
    """Segments from near one corner of the volume to near the opposite one
    (every axis flipped at random): about 24 pieces each in 512^3 with
    256 x 64 x 32 bricks."""
    rng = np.random.default_rng(seed)
    hi = np.array(dims) - 1
    p0 = rng.integers(0, 4, (n, 3))
    p1 = hi - rng.integers(0, 4, (n, 3))
    flip = rng.integers(0, 2, (n, 3)).astype(bool)
    return np.concatenate([np.where(flip, hi - p0, p0), np.where(flip, hi - p1, p1)], 1).astype(np.int32)


@pytest.mark.parametrize("euclid", [False, True])
def test_compact_workspace(euclid):
    """Plain brick-path calls in a compact workspace: with room for 16 piece
    records a segment they take the bricks; with only the table and
    histogram part (long diagonal segments: about 480 000 records, room for
    far fewer) the direct kernels serve the call.  Both give the oracle's
    volume and counts, cleared and ORed into a volume."""
    torch = pytest.importorskip("torch")
    dims = (512, 512, 512)
    flags = binding.VOX_GRID_EUCLID if euclid else 0
    grid_fn, counts_fn = (oracle.grid_euclid, oracle.counts_euclid) if euclid else (oracle.grid, oracle.counts)
    rng = np.random.default_rng(31)
    base = rng.integers(0, 2**32, size=binding.grid_words(dims), dtype=np.uint32)
    cases = [(workloads.arbitrary_length(n=40_000, volume=512)["segs"], 0, False),
             (long_diagonals(dims, 20_000, 32), 16 * 16 * 20_000, True)]
    for segs, cut, overflow in cases:
        n = len(segs)
        work = binding.workspace(binding.vox_workspace_bytes(binding.VOX_OP_GRID, n, 1) - cut, dev())
        for clear in (True, False):
            g = to_dev(base.view(np.int32))
            c_ = torch.empty(n, dtype=torch.int32, device=dev())
            binding.vox_segments_to_grid(to_dev(segs), dims, g, c_,
                                         flags | (binding.VOX_GRID_CLEAR if clear else 0), work)
            assert binding.vox_read_status(work) == binding.VOX_OK
            pieces, direct_all = binding.vox_read_batch_info(work)
            assert direct_all == overflow and pieces >= n
            assert np.array_equal(grid_host(g), grid_fn(segs, dims, base=None if clear else base))
            assert np.array_equal(to_host(c_), counts_fn(segs))


def test_unaligned_segment_array():
    """A 4-byte (not 8-byte) aligned segment array takes the direct path."""
    torch = pytest.importorskip("torch")
    dims = (128, 128, 64)
    segs = random_in(dims, 3001, 3)
    buf = torch.empty(6 * segs.shape[0] + 1, dtype=torch.int32, device=dev())
    buf[1:].copy_(torch.from_numpy(segs.reshape(-1)).to(dev()))
    view = buf[1:].view(-1, 6)
    assert view.data_ptr() % 8 == 4
    g, c = binding.segments_to_grid(view, dims, want_counts=True)
    assert np.array_equal(grid_host(g), oracle.grid(segs, dims))
    assert np.array_equal(to_host(c), oracle.counts(segs))


def test_empty_clears():
    torch = pytest.importorskip("torch")
    dims = (128, 16, 16)
    g = torch.full((binding.grid_words(dims),), -1, dtype=torch.int32, device=dev())
    segs = torch.zeros((0, 6), dtype=torch.int32, device=dev())
    binding.segments_to_grid(segs, dims, grid=None)
    work = binding.workspace(binding.vox_grid_workspace_bytes(0, dims), dev())
    binding.vox_segments_to_grid(segs, dims, g, None, binding.VOX_GRID_CLEAR, work)
    assert not grid_host(g).any()


SHAPES = [(8, 6, 5), (8, 6, 6), (7, 6, 6), (7, 7, 6)]


class tuned:
    """Autotune cache entries of a brick shape for the given (dims, n) keys
    of plain calls, removed on exit."""

    def __init__(self, lg, keys, wgs=0):
        self.lg, self.keys, self.wgs = lg, keys, wgs

    def __enter__(self):
        for dims, n in self.keys:
            binding.vox_tuning_cache_set(dims, n, binding.make_tuning(self.lg, self.wgs))
            t = binding.vox_tuning_cache_get(dims, n)
            assert tuple(t.brick_lg) == tuple(self.lg)

    def __exit__(self, *exc):
        binding.vox_tuning_cache_clear()


@pytest.mark.parametrize("lg", SHAPES)
def test_every_brick_shape(lg):
    """Each compiled brick shape, taken from the autotune cache for its
    volume and segment count, gives the oracle's volume."""
    c = workloads.arbitrary_length(n=40_000, volume=512)
    dims = (96, 64, 32)
    rng = np.random.default_rng(11)
    base = rng.integers(0, 2**32, size=binding.grid_words(dims), dtype=np.uint32)
    segs = random_in(dims, 30_000, 12)
    with tuned(lg, [(c["dims"], 40_000), (dims, 30_000)]):
        assert_grid(c["segs"], c["dims"])
        assert_grid(segs, dims, base=base)


@pytest.mark.parametrize("wgs", [1, 2])
def test_fill_workgroups_per_cu(wgs):
    c = workloads.arbitrary_length(n=40_000, volume=512)
    with tuned((8, 6, 5), [(c["dims"], 40_000)], wgs=wgs):
        assert_grid(c["segs"], c["dims"])


@pytest.mark.parametrize("lg", [(8, 6, 5), (8, 6, 6)])
def test_full_length_pieces(lg):
    """Pieces as long as the brick is wide: a fill group's chunks overflow its
    table, so its two record sets run one after the other."""
    dims = (512, 64, 64)
    rng = np.random.default_rng(21)
    n = 20000  # above the direct path's segment limit
    y0 = rng.integers(3, 61, n)
    z0 = rng.integers(3, 61, n)
    segs = np.stack([np.zeros(n, np.int64), y0, z0, np.full(n, 511), y0 + rng.integers(-3, 4, n),
                     z0 + rng.integers(-3, 4, n)], 1).astype(np.int32)
    segs[::2] = segs[::2][:, [3, 4, 5, 0, 1, 2]]  # both directions
    with tuned(lg, [(dims, n)]):
        assert_grid(segs, dims)


def test_more_bricks_than_big_stages():
    """A volume of more than 8192 bricks: its histogram stages 4096 segments
    per round (the big stages leave too little LDS for its counters)."""
    dims = (2048, 2048, 1088)             # 16 x 32 x 17 = 8704 bricks
    with tuned((7, 6, 6), [(dims, 20_000)]):
        assert_grid(random_in(dims, 20_000, 23), dims)


def test_unsupported_shape_rejected():
    with pytest.raises(binding.VoxError):
        binding.vox_tuning_cache_set((512, 512, 512), 10, binding.make_tuning((9, 9, 9)))
    assert binding.vox_tuning_cache_get((512, 512, 512), 10) is None


@pytest.mark.parametrize("n", [16384, 16385])
def test_direct_brick_boundary(n):
    """Plain calls of at most 16384 segments take the direct path, larger
    ones the brick path: both sides, cleared and ORed into a volume."""
    dims = (256, 128, 64)
    segs = random_in(dims, n, 500 + n)
    assert_grid(segs, dims)
    rng = np.random.default_rng(n)
    base = rng.integers(0, 2**32, size=binding.grid_words(dims), dtype=np.uint32)
    assert_grid(segs, dims, base=base)


def dense_spot(dims, spot, n_spot, n_rest, seed):
    """n_spot short segments (up to 6 voxels) inside the box [0, spot) and
    n_rest random ones in the whole volume."""
    rng = np.random.default_rng(seed)
    p0 = np.stack([rng.integers(0, s, n_spot) for s in spot], 1)
    p1 = np.clip(p0 + rng.integers(-6, 7, (n_spot, 3)), 0, np.array(spot) - 1)
    return np.concatenate([np.concatenate([p0, p1], 1).astype(np.int32), random_in(dims, n_rest, seed + 1)])


@pytest.mark.parametrize("euclid", [False, True])
def test_dense_brick_cut_into_items(euclid):
    """A brick holding far more than a workgroup's share of the records
    (100 000 short segments in one 256x64x32 brick of a 512x256x128 volume)
    is cut into several work items of the fill, each ORing its part into the
    volume with device atomics, after the clear kernel zeroed the brick in a
    cleared volume: the oracle's volume, cleared and ORed into a volume,
    through the compact workspace and the worst-case one."""
    torch = pytest.importorskip("torch")
    dims = (512, 256, 128)
    segs = dense_spot(dims, (256, 64, 32), 100_000, 20_000, 77)
    n = len(segs)
    flags = binding.VOX_GRID_EUCLID if euclid else 0
    grid_fn = oracle.grid_euclid if euclid else oracle.grid
    rng = np.random.default_rng(78)
    base = rng.integers(0, 2**32, size=binding.grid_words(dims), dtype=np.uint32)
    base &= rng.integers(0, 2**32, size=base.size, dtype=np.uint32)
    for work_bytes in (binding.vox_workspace_bytes(binding.VOX_OP_GRID, n, 1),
                       binding.vox_grid_workspace_bytes(n, dims)):
        work = binding.workspace(work_bytes, dev())
        for clear in (True, False):
            g = to_dev(base.view(np.int32))
            binding.vox_segments_to_grid(to_dev(segs), dims, g, None,
                                         flags | (binding.VOX_GRID_CLEAR if clear else 0), work)
            assert binding.vox_read_status(work) == binding.VOX_OK
            # Header words 12 and 13 of the workspace (internal layout): the
            # fill's work items and the bricks cut into several.
            hdr = work[:64].cpu().view(torch.int32).numpy()
            assert hdr[13] >= 1 and hdr[12] > hdr[13]
            got = grid_host(g)
            exp = grid_fn(segs, dims, base=None if clear else base)
            if not np.array_equal(got, exp):
                bad = np.flatnonzero(got != exp)
                raise AssertionError("%d words differ, first %s" % (bad.size, bad[:5].tolist()))
