"""HIP int32 voxel lists (vox_segments_to_list32) against the CPU oracle,
element by element; the paper's experiment shapes at full size by sampled
rows (GPU)."""

import numpy as np
import pytest

from oracle import oracle
from paper_2009_09500_amd import binding, workloads
from tests import pins
from tests.gpu_helpers import canaries_intact, dev, padded, to_dev, to_host

pytestmark = pytest.mark.gpu


def assert_parity(segs: np.ndarray):
    pytest.importorskip("torch")
    offs, vox = binding.segments_to_list(to_dev(segs), wide=True)
    offs, vox = to_host(offs), to_host(vox)
    assert np.array_equal(offs, oracle.offsets(segs))
    exp = oracle.voxel_list32(segs)
    assert vox.dtype == np.int32 and vox.shape == exp.shape
    if not np.array_equal(vox, exp):
        bad = np.argwhere(np.any(vox != exp, axis=1))[:5, 0]
        raise AssertionError("first mismatching voxels %s: got %s expected %s" % (
            bad.tolist(), vox[bad].tolist(), exp[bad].tolist()))


def test_small_sets_equal_int16_lists():
    segs = np.concatenate([pins.exhaustive(-2, 2), pins.random_segments(3000, 81, -8000, 8000)])
    assert_parity(segs)


def test_single_long_segments():
    # 10^3 .. 10^6 voxels, far outside the int16 range
    assert_parity(workloads.paper_segments([1000, 10 ** 4, 10 ** 5, 10 ** 6])["segs"])


def test_axis_and_extreme_int32():
    segs = np.array([[2 ** 31 - 1, -(2 ** 31), 0, 2 ** 31 - 1 - 70000, -(2 ** 31) + 69999, 5],
                     [-(2 ** 30), 0, 2 ** 30, -(2 ** 30) + 2 ** 20, 0, 2 ** 30],
                     [5, 5, 5, 5, 5, 5],
                     [0, 0, 0, 2 * 40000, 40000, -40000]], np.int32)
    assert_parity(segs)


def test_fixed_length_experiment_scaled():
    # experiment 2's shape: 1024 segments of one length (several tiles each)
    for L in (20, 2000, 20000):
        assert_parity(workloads.paper_segments(np.full(1024, L), seed=90 + L)["segs"])


def test_arbitrary_lengths_scaled():
    L = workloads.paper_arbitrary_lengths(n=1024, total=3 * 10 ** 7)
    assert_parity(workloads.paper_segments(L)["segs"])


def test_span_2p30_rejected_writes_nothing():
    torch = pytest.importorskip("torch")
    segs = np.array([[0, 0, 0, 10, 3, 1], [0, 0, 0, 0, 2 ** 30, 0]], np.int32)
    s = to_dev(segs)
    offs = torch.empty(3, dtype=torch.int64, device=dev())
    whole, vox = padded(100 * 3, torch.int32, 64, 0x5A5A5A5A)
    work = binding.workspace(binding.vox_list_workspace_bytes(2, 100), dev())
    with pytest.raises(binding.VoxError) as e:
        binding.vox_segments_to_list(s, offs, vox.view(-1, 3), 100, work, want_total=True, wide=True)
    assert e.value.status == binding.VOX_ERR_OUT_OF_RANGE
    assert np.all(to_host(whole) == 0x5A5A5A5A)
    # one below the limit is accepted (count only: 2^30 voxels)
    ok = to_dev(np.array([[0, 0, 0, 0, 2 ** 30 - 1, 0]], np.int32))
    offs1 = torch.empty(2, dtype=torch.int64, device=dev())
    w1 = binding.workspace(binding.vox_list_workspace_bytes(1, 0), dev())
    assert binding.vox_segments_to_list(ok, offs1, None, 0, w1, want_total=True, wide=True) == 2 ** 30


def test_capacity_and_empty():
    torch = pytest.importorskip("torch")
    segs = workloads.paper_segments([5000, 7000])["segs"]
    s = to_dev(segs)
    offs = torch.empty(3, dtype=torch.int64, device=dev())
    whole, vox = padded(11999 * 3, torch.int32, 64, 0x5A5A5A5A)
    work = binding.workspace(binding.vox_list_workspace_bytes(2, 11999), dev())
    with pytest.raises(binding.VoxError) as e:
        binding.vox_segments_to_list(s, offs, vox.view(-1, 3), 11999, work, want_total=True, wide=True)
    assert e.value.status == binding.VOX_ERR_CAPACITY
    assert np.all(to_host(whole) == 0x5A5A5A5A)
    whole, vox = padded(12000 * 3, torch.int32, 64, 0x5A5A5A5A)
    work = binding.workspace(binding.vox_list_workspace_bytes(2, 12000), dev())
    assert binding.vox_segments_to_list(s, offs, vox.view(-1, 3), 12000, work, want_total=True,
                                        wide=True) == 12000
    assert canaries_intact(whole, 64, 0x5A5A5A5A)
    assert np.array_equal(to_host(vox).reshape(-1, 3), oracle.voxel_list32(segs))
    o, v = binding.segments_to_list(to_dev(np.zeros((0, 6), np.int32)), wide=True)
    assert to_host(o).tolist() == [0] and v.shape[0] == 0


def test_arbitrary_experiment_full_size_sampled():
    """Experiment 3 at full size: 1024 segments, 10^9 voxels (12 GB of int32
    rows).  Offsets in full; rows at every segment's ends and 64 random k per
    segment against the oracle's voxel function."""
    torch = pytest.importorskip("torch")
    L = workloads.paper_arbitrary_lengths()
    segs = workloads.paper_segments(L)["segs"]
    offs, vox = binding.segments_to_list(to_dev(segs), wide=True)
    h_offs = to_host(offs)
    assert np.array_equal(h_offs, oracle.offsets(segs))
    rng = np.random.default_rng(5)
    rows, exp = [], []
    for i, seg in enumerate(segs):
        n = int(L[i])
        for k in {0, 1, n // 2, n - 2, n - 1} | set(rng.integers(0, n, 64).tolist()):
            if 0 <= k < n:
                rows.append(int(h_offs[i]) + k)
                exp.append(oracle.voxel(seg, k))
    idx = torch.tensor(rows, dtype=torch.int64, device=dev())
    got = to_host(vox.index_select(0, idx))
    assert np.array_equal(got.astype(np.int64), np.array(exp, np.int64))
    del vox
    torch.cuda.empty_cache()
