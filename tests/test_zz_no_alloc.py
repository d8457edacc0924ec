"""vox_segments_to_list_noalloc (the library's own device array as the
workspace) against vox_segments_to_list on the same inputs, element by
element: two calls in a row, the second with a smaller input, so the second
runs on the array the first left behind (GPU)."""

import numpy as np
import pytest

from paper_2009_09500_amd import binding, workloads
from tests.gpu_helpers import dev, to_dev, to_host



def lists_with_workspace(segs):
    offs, vox = binding.segments_to_list(segs)
    return to_host(offs), to_host(vox)


def lists_noalloc(segs):
    import torch
    n = segs.shape[0]
    offs = torch.empty(n + 1, dtype=torch.int64, device=dev())
    total = binding.vox_segments_to_list_noalloc(segs, offs, None, 0, want_total=True)
    vox = torch.empty((max(total, 1), 3), dtype=torch.int16, device=dev())
    vox.fill_(0x5A5A)
    got = binding.vox_segments_to_list_noalloc(segs, offs, vox, total, want_total=True)
    assert got == total
    return to_host(offs), to_host(vox)[:total]


@pytest.mark.gpu
def test_noalloc_equals_workspace_entry_point_twice():
    big = workloads.fixed_length(n=300_000)["segs"]                 # 19.5 M voxels, many tiles
    small = workloads.small_uniform(n=1000)["segs"]                 # one-block path
    mid = workloads.arbitrary_length(n=5000, volume=512)["segs"]    # ragged tail, four kernels
    for segs in (big, small, mid):
        d = to_dev(segs)
        o1, v1 = lists_with_workspace(d)
        o2, v2 = lists_noalloc(d)
        assert np.array_equal(o1, o2) and np.array_equal(v1, v2)


@pytest.mark.gpu
def test_noalloc_errors():
    import torch
    segs = np.array([[0, 0, 0, 40000, 0, 0]], np.int32)            # beyond int16
    d = to_dev(segs)
    offs = torch.empty(2, dtype=torch.int64, device=dev())
    vox = torch.empty((10, 3), dtype=torch.int16, device=dev())
    with pytest.raises(binding.VoxError) as e:
        binding.vox_segments_to_list_noalloc(d, offs, vox, 10, want_total=True)
    assert e.value.status == binding.VOX_ERR_OUT_OF_RANGE
    ok = to_dev(np.array([[0, 0, 0, 9, 3, 1]], np.int32))
    with pytest.raises(binding.VoxError) as e:
        binding.vox_segments_to_list_noalloc(ok, offs, vox, 5, want_total=True)
    assert e.value.status == binding.VOX_ERR_CAPACITY
    o2, v2 = lists_noalloc(ok)                                       # recovers on the next call
    o1, v1 = lists_with_workspace(ok)
    assert np.array_equal(o1, o2) and np.array_equal(v1, v2)


def test_noalloc_rejects_calls_beyond_its_array():
    """Sizes whose workspace exceeds the library's 32 MiB array are refused
    before any device work (CPU: no device is touched)."""
    import ctypes
    lib = binding.load()
    fake = ctypes.c_void_p(1 << 20)
    st = lib.vox_segments_to_list_noalloc(fake, 10_000_000, fake, None, 0, None, None)
    assert st == binding.VOX_ERR_WORKSPACE and b"library" in lib.vox_last_error()
    st = lib.vox_segments_to_list_noalloc(fake, 1000, fake, fake, 1 << 40, None, None)
    assert st == binding.VOX_ERR_WORKSPACE
    assert lib.vox_segments_to_list_noalloc(fake, -1, fake, None, 0, None, None) == binding.VOX_ERR_INVALID_ARGUMENT
    assert binding.vox_list_workspace_bytes(10_000_000, 0) > 32 << 20 > binding.vox_list_workspace_bytes(10_000, 10_000)
