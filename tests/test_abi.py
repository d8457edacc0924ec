"""The C ABI library loads and exports what include/vox.h declares; host-side
argument checks (CPU only: no call here reaches the GPU)."""

import ctypes
import re

import pytest

from paper_2009_09500_amd import binding


@pytest.fixture(scope="module")
def lib():
    return binding.load()


def test_exports_every_declared_function(lib):
    names = binding.header_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name


def test_abi_version_matches_header(lib):
    text = open(binding.HEADER).read()
    v = int(re.search(r"#define VOX_ABI_VERSION (\d+)", text).group(1))
    assert lib.vox_abi_version() == v


def test_status_strings(lib):
    for code in range(7):
        assert lib.vox_status_string(code)
    assert lib.vox_status_string(99) == b"unknown status"


def test_status_codes_match_header():
    text = open(binding.HEADER).read()
    for name in ("VOX_OK", "VOX_ERR_INVALID_ARGUMENT", "VOX_ERR_OUT_OF_RANGE",
                 "VOX_ERR_CAPACITY", "VOX_ERR_DEVICE", "VOX_ERR_WORKSPACE",
                 "VOX_ERR_BATCH_MISMATCH"):
        v = int(re.search(name + r" = (\d+)", text).group(1))
        assert getattr(binding, name) == v


def test_workspace_sizes_grow(lib):
    a = lib.vox_list_workspace_bytes(1000, 0)
    b = lib.vox_list_workspace_bytes(1000, 10**6)
    c = lib.vox_list_workspace_bytes(10**6, 10**6)
    assert 0 < a < b < c
    assert lib.vox_list_workspace_bytes(-1, 0) == 0
    assert lib.vox_grid_workspace_bytes(10, 0, 4, 4) == 0
    assert lib.vox_grid_workspace_bytes(10, 64, 64, 64) > 0


def test_host_argument_errors(lib):
    P = ctypes.c_void_p
    fake = P(1 << 20)          # never dereferenced: the checks fail first
    st = lib.vox_segments_to_list(fake, -1, fake, None, 0, None, fake, 1 << 20, None)
    assert st == binding.VOX_ERR_INVALID_ARGUMENT
    assert b"n must be" in lib.vox_last_error()
    st = lib.vox_segments_to_list(None, 5, fake, None, 0, None, fake, 1 << 20, None)
    assert st == binding.VOX_ERR_INVALID_ARGUMENT
    st = lib.vox_segments_to_list(fake, 5, P((1 << 20) + 4), None, 0, None, fake, 1 << 20, None)
    assert st == binding.VOX_ERR_INVALID_ARGUMENT            # offsets misaligned
    st = lib.vox_segments_to_list(fake, 5, fake, P((1 << 20) + 8), 100, None, fake, 1 << 20, None)
    assert st == binding.VOX_ERR_INVALID_ARGUMENT            # voxels misaligned
    st = lib.vox_segments_to_list(fake, 5, fake, None, 0, None, fake, 16, None)
    assert st == binding.VOX_ERR_WORKSPACE
    st = lib.vox_segments_to_list(fake, 5, fake, None, 0, None, None, 1 << 20, None)
    assert st == binding.VOX_ERR_WORKSPACE
    st = lib.vox_segments_to_grid(fake, 5, 0, 8, 8, fake, None, 1, fake, 1 << 20, None)
    assert st == binding.VOX_ERR_INVALID_ARGUMENT
    st = lib.vox_segments_to_grid(fake, 5, 1 << 21, 8, 8, fake, None, 1, fake, 1 << 20, None)
    assert st == binding.VOX_ERR_INVALID_ARGUMENT
    st = lib.vox_segments_to_grid(fake, 5, 8, 8, 8, fake, None, 6, fake, 1 << 20, None)
    assert st == binding.VOX_ERR_INVALID_ARGUMENT            # unknown flag
    st = lib.vox_segments_to_grid(fake, 5, 8, 8, 8, P((1 << 20) + 4), None, 1, fake, 1 << 20, None)
    assert st == binding.VOX_ERR_INVALID_ARGUMENT            # grid misaligned
    st = lib.vox_segments_to_grid(fake, 5, 8, 8, 8, fake, None, 1, fake, 0, None)
    assert st == binding.VOX_ERR_WORKSPACE


def test_list_variants_share_host_checks(lib):
    """The Euclidean and int32 list entry points reject bad arguments on the
    host, before any device work, as the int16 lists do."""
    P = ctypes.c_void_p
    fake = P(1 << 20)
    for fn in (lib.vox_segments_to_list_euclid, lib.vox_segments_to_list32):
        assert fn(fake, -1, fake, None, 0, None, fake, 1 << 20, None) == binding.VOX_ERR_INVALID_ARGUMENT
        assert fn(None, 5, fake, None, 0, None, fake, 1 << 20, None) == binding.VOX_ERR_INVALID_ARGUMENT
        assert fn(fake, 5, fake, P((1 << 20) + 8), 100, None, fake, 1 << 20, None) == \
            binding.VOX_ERR_INVALID_ARGUMENT                 # voxels misaligned
        assert fn(fake, 5, fake, None, 0, None, fake, 16, None) == binding.VOX_ERR_WORKSPACE


def test_binding_rejects_euclid_with_int32(lib):
    import pytest
    with pytest.raises(ValueError, match="Chebyshev"):
        binding.vox_segments_to_list(None, None, None, 0, None, euclid=True, wide=True)
