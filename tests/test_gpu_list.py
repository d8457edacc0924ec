"""HIP voxel lists against the CPU oracle, element by element (GPU)."""

import numpy as np
import pytest

from oracle import oracle
from paper_2009_09500_amd import binding, workloads
from tests import pins
from tests.gpu_helpers import canaries_intact, dev, padded, to_dev, to_host

pytestmark = pytest.mark.gpu


def run_list(segs: np.ndarray):
    torch = pytest.importorskip("torch")
    s = to_dev(segs)
    offs, vox = binding.segments_to_list(s)
    torch.cuda.synchronize()
    return to_host(offs), to_host(vox)


def assert_parity(segs: np.ndarray):
    offs, vox = run_list(segs)
    exp_off = oracle.offsets(segs)
    assert np.array_equal(offs, exp_off)
    exp = oracle.voxel_list(segs)
    assert vox.shape == exp.shape
    if not np.array_equal(vox, exp):
        bad = np.argwhere(np.any(vox != exp, axis=1))[:5, 0]
        raise AssertionError("first mismatching voxels %s: got %s expected %s" % (
            bad.tolist(), vox[bad].tolist(), exp[bad].tolist()))


def test_exhaustive_negative_pairs():
    assert_parity(pins.exhaustive(-3, 3))


def test_small_uniform_config():
    assert_parity(workloads.small_uniform()["segs"])


def test_single_diagonal():
    assert_parity(workloads.single_diagonal()["segs"])


def test_fixed_length_scaled():
    # 20 011 segments x 65 voxels: ~1270 tiles, ragged last tile.
    assert_parity(workloads.fixed_length(n=20011)["segs"])


def test_arbitrary_lengths_as_lists():
    assert_parity(workloads.arbitrary_length(n=30001)["segs"])


def test_long_and_negative_segments():
    assert_parity(pins.random_segments(3000, 41, -8000, 8000))


def test_extreme_int16_lengths():
    """N > 32767 takes the 64-bit start-up division."""
    segs = np.array([[-32768, -32768, -32768, 32767, 32767, 32767],
                     [32767, -32768, 0, -32768, 100, -5],
                     [-32768, 0, 0, 32767, 1, -1],
                     [0, 0, 0, 0, 0, 0]], dtype=np.int32)
    assert_parity(segs)


def test_point_segments_only():
    rng = np.random.default_rng(3)
    p = rng.integers(-100, 100, size=(5000, 3))
    assert_parity(np.concatenate([p, p], 1).astype(np.int32))


def test_dense_tiles_mixed_lengths():
    """Tiles holding more segments than one LDS window (256): runs of 1- to
    3-voxel segments, so that window boundaries fall inside a lane's eight
    voxels, between runs of long segments, so that tiles go from dense to
    sparse and back."""
    rng = np.random.default_rng(17)
    parts = []
    for r in range(12):
        if r % 3 == 2:
            parts.append(pins.random_segments(40, 100 + r, -3000, 3000))
        else:
            n = int(rng.integers(2000, 6000))
            p0 = rng.integers(-500, 500, size=(n, 3))
            p1 = p0 + rng.integers(-2, 3, size=(n, 3))
            parts.append(np.concatenate([p0, p1], 1).astype(np.int32))
    segs = np.concatenate(parts)
    assert_parity(segs)
    torch = pytest.importorskip("torch")
    offs, vox = binding.segments_to_list(to_dev(segs), wide=True)
    exp = oracle.voxel_list(segs)
    assert np.array_equal(to_host(vox), exp.astype(np.int32))


def test_empty():
    torch = pytest.importorskip("torch")
    segs = torch.zeros((0, 6), dtype=torch.int32, device=dev())
    offs, vox = binding.segments_to_list(segs)
    assert to_host(offs).tolist() == [0]
    assert vox.shape[0] == 0


def test_full_fixed_length_config():
    """1 048 576 segments x 65 voxels = 68 157 440 voxels, all compared."""
    assert_parity(workloads.fixed_length()["segs"])


def _prepared(segs, capacity, pad=64, fill=0x5A5A):
    torch = pytest.importorskip("torch")
    s = to_dev(segs)
    n = segs.shape[0]
    offs = torch.empty(n + 1, dtype=torch.int64, device=dev())
    whole, payload = padded(max(capacity, 1) * 3 + 5, torch.int16, pad * 8, fill)
    # 16-byte-aligned payload view: pad*8 int16 = 1 KiB of canaries.
    vox = payload[: max(capacity, 1) * 3].view(-1, 3)
    work = binding.workspace(binding.vox_list_workspace_bytes(n, capacity), dev())
    return s, offs, whole, vox, work


def test_capacity_too_small_writes_nothing():
    segs = workloads.small_uniform(n=300)["segs"]
    total = int(oracle.offsets(segs)[-1])
    s, offs, whole, vox, work = _prepared(segs, total - 1)
    with pytest.raises(binding.VoxError) as e:
        binding.vox_segments_to_list(s, offs, vox, total - 1, work, want_total=True)
    assert e.value.status == binding.VOX_ERR_CAPACITY
    assert np.all(to_host(whole) == 0x5A5A)
    # Asynchronous form: the status word carries the error.
    binding.vox_segments_to_list(s, offs, vox, total - 1, work)
    assert binding.vox_read_status(work) == binding.VOX_ERR_CAPACITY
    assert np.all(to_host(whole) == 0x5A5A)
    assert np.array_equal(to_host(offs), oracle.offsets(segs))


def test_out_of_int16_range_writes_nothing():
    segs = workloads.small_uniform(n=100)["segs"].copy()
    segs[37, 4] = 40000
    cap = 10**6
    s, offs, whole, vox, work = _prepared(segs, cap)
    binding.vox_segments_to_list(s, offs, vox, cap, work)
    assert binding.vox_read_status(work) == binding.VOX_ERR_OUT_OF_RANGE
    assert np.all(to_host(whole) == 0x5A5A)


def test_exact_capacity_and_guard_band():
    segs = workloads.arbitrary_length(n=5000, volume=300)["segs"]
    total = int(oracle.offsets(segs)[-1])
    s, offs, whole, vox, work = _prepared(segs, total)
    got = binding.vox_segments_to_list(s, offs, vox, total, work, want_total=True)
    assert got == total
    assert canaries_intact(whole, 64 * 8, 0x5A5A)
    h = to_host(whole)[64 * 8: 64 * 8 + total * 3].reshape(-1, 3)
    assert np.array_equal(h, oracle.voxel_list(segs))


def test_unaligned_segment_array():
    """A 4-byte-aligned (not 8-byte) segment view takes the scalar loads."""
    torch = pytest.importorskip("torch")
    segs = pins.random_segments(2000, 43, -500, 500)
    flat = np.concatenate([[0], segs.ravel()]).astype(np.int32)
    t = to_dev(flat)[1:].view(-1, 6)
    assert t.data_ptr() % 8 == 4
    offs, vox = binding.segments_to_list(t)
    assert np.array_equal(to_host(vox), oracle.voxel_list(segs))


def test_repeatable():
    segs = workloads.arbitrary_length(n=20000, volume=1000)["segs"]
    a = run_list(segs)
    b = run_list(segs)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("n", [1023, 1024, 1025, 2048])
def test_one_block_boundary(n):
    """Lists of at most 1024 segments take the one-block count/scan/offsets
    kernel, larger ones the three-kernel path: both sides of the boundary,
    int16 and int32 lists, the latter with a tile map above 4096 tiles."""
    assert_parity(workloads.arbitrary_length(n=n, seed=300 + n, volume=1024)["segs"])
    long = workloads.paper_segments(np.full(n, 5000), seed=400 + n)["segs"]
    offs, vox = binding.segments_to_list(to_dev(long), wide=True)
    assert np.array_equal(to_host(offs), oracle.offsets(long))
    assert np.array_equal(to_host(vox), oracle.voxel_list32(long))
