"""Host-side batch planning (vox_batch_plan, vox_batch_launch_cover): the
table image, the launch shape and the argument checks.  CPU only: the
planner makes no device call and never dereferences the scene pointers."""

import ctypes
import struct

import numpy as np
import pytest

from paper_2009_09500_amd import binding

HEADER = struct.Struct("<4I3iI4Q")          # BrickTable
SCENE = struct.Struct("<3Q q Q 3i 3i 3i I 4I")  # BrickScene
SCENES_AT = 64
ROWS_PER = 4096
MAX_ROWS = 256


@pytest.fixture(scope="module")
def lib():
    return binding.load()


@pytest.fixture(autouse=True)
def default_tuning():
    binding.vox_set_tuning(None)
    yield
    binding.vox_set_tuning(None)


def scene_array(specs):
    """specs: (n, (dx, dy, dz), flags); fake 256-aligned device pointers."""
    arr = (binding.VoxScene * len(specs))()
    for i, (n, dims, flags) in enumerate(specs):
        arr[i].segs = (1 << 30) + i * (1 << 24) if n else 0
        arr[i].n = n
        arr[i].dim_x, arr[i].dim_y, arr[i].dim_z = dims
        arr[i].flags = flags
        arr[i].grid = (1 << 40) + i * (1 << 28)
        arr[i].counts = 0
    return arr


def plan(lib, specs):
    arr = scene_array(specs)
    launch = binding.VoxBatchLaunch()
    st = lib.vox_batch_plan(arr, len(specs), None, 0, ctypes.byref(launch))
    assert st == binding.VOX_OK, lib.vox_last_error()
    table = np.zeros(launch.table_bytes, dtype=np.uint8)
    st = lib.vox_batch_plan(arr, len(specs), ctypes.c_void_p(table.ctypes.data), table.nbytes,
                            ctypes.byref(launch))
    assert st == binding.VOX_OK, lib.vox_last_error()
    return table, launch


def decode(table):
    h = HEADER.unpack_from(table.tobytes(), 0)
    hdr = dict(magic=h[0], n_scenes=h[1], rows=h[2], bricks=h[3], lg=h[4:7], max_nb=h[7],
               hist_words=h[8], pieces=h[9], work_bytes=h[10], table_bytes=h[11])
    scenes = []
    for i in range(hdr["n_scenes"]):
        v = SCENE.unpack_from(table.tobytes(), SCENES_AT + i * SCENE.size)
        scenes.append(dict(segs=v[0], counts=v[1], grid=v[2], n=v[3], hist_off=v[4],
                           dim=v[5:8], lg=v[8:11], nb=v[11:14], nbricks=v[14],
                           brick_base=v[15], row_base=v[16], rows=v[17], flags=v[18]))
    return hdr, scenes


def expected_rows(n):
    return min(MAX_ROWS, max(1, -(-n // ROWS_PER)))


def test_scene_struct_size():
    assert SCENE.size == 96 and HEADER.size == 64


def test_table_layout(lib):
    specs = [(1000, (64, 64, 64), 1), (0, (128, 96, 64), 0), (200000, (512, 512, 512), 1),
             (5000, (256, 128, 256), 1)]
    table, launch = plan(lib, specs)
    hdr, scenes = decode(table)
    assert hdr["magic"] == 0x564F5842 and hdr["n_scenes"] == 4
    lg = (8, 6, 5)                       # default of the largest volume (512^3)
    assert tuple(launch.brick_lg) == lg and hdr["lg"] == lg
    rows = bricks = hist = pieces = 0
    for (n, dims, flags), sc in zip(specs, scenes):
        nb = tuple(-(-d // (1 << l)) for d, l in zip(dims, lg))
        assert sc["nb"] == nb and sc["nbricks"] == nb[0] * nb[1] * nb[2]
        assert sc["dim"] == dims and sc["n"] == n
        assert sc["rows"] == expected_rows(n)
        assert sc["row_base"] == rows and sc["brick_base"] == bricks and sc["hist_off"] == hist
        assert sc["flags"] & 1 == flags
        rows += sc["rows"]
        bricks += sc["nbricks"]
        hist += sc["rows"] * sc["nbricks"]
        pieces += n * (1 + sum(b - 1 for b in nb))
    assert (hdr["rows"], hdr["bricks"], hdr["hist_words"], hdr["pieces"]) == (rows, bricks, hist, pieces)
    assert launch.rows == rows and launch.bricks == bricks
    assert launch.max_scene_bricks == max(sc["nbricks"] for sc in scenes) == hdr["max_nb"]
    assert launch.work_bytes == hdr["work_bytes"] and launch.table_bytes == hdr["table_bytes"]
    assert hdr["table_bytes"] == SCENES_AT + 4 * SCENE.size + 4 * (rows + bricks)
    tail = np.frombuffer(table.tobytes(), dtype=np.uint32, offset=SCENES_AT + 4 * SCENE.size)
    row_scene, brick_scene = tail[:rows], tail[rows:rows + bricks]
    for i, sc in enumerate(scenes):
        assert (row_scene[sc["row_base"]:sc["row_base"] + sc["rows"]] == i).all()
        assert (brick_scene[sc["brick_base"]:sc["brick_base"] + sc["nbricks"]] == i).all()
    # Workspace: header slots, histogram rows, totals, bin offsets, records.
    up = lambda v: (v + 255) // 256 * 256
    assert hdr["work_bytes"] == 768 + up(4 * hist) + up(4 * bricks) + up(4 * (bricks + 1)) + 16 * pieces


def test_one_scene_table_has_no_lookup_arrays(lib):
    table, launch = plan(lib, [(4096 * 3 + 1, (256, 256, 256), 1)])
    hdr, scenes = decode(table)
    assert hdr["table_bytes"] == SCENES_AT + SCENE.size
    assert scenes[0]["rows"] == 4 and launch.rows == 4


def test_plain_and_batch_workspace_agree(lib):
    """A one-scene batch needs what the plain call on the same volume needs
    when the plain call takes the brick path (more than 16384 segments);
    smaller plain calls take the direct path and need less."""
    for n, dims in ((20000, (256, 256, 256)), (10**6, (512, 512, 512)), (16385, (64, 64, 32))):
        _, launch = plan(lib, [(n, dims, 1)])
        assert launch.work_bytes == lib.vox_grid_workspace_bytes(n, *dims)
    for n, dims in ((1000, (256, 256, 256)), (16384, (512, 512, 512)), (1, (64, 64, 32))):
        _, launch = plan(lib, [(n, dims, 1)])
        assert 0 < lib.vox_grid_workspace_bytes(n, *dims) < launch.work_bytes


def test_tuning_sets_batch_shape(lib):
    binding.vox_set_tuning((7, 6, 6))
    _, launch = plan(lib, [(100, (512, 512, 512), 1)])
    assert tuple(launch.brick_lg) == (7, 6, 6)


def test_plan_errors(lib):
    launch = binding.VoxBatchLaunch()
    arr = scene_array([(10, (64, 64, 64), 1)])
    assert lib.vox_batch_plan(arr, 0, None, 0, ctypes.byref(launch)) == binding.VOX_ERR_INVALID_ARGUMENT
    assert lib.vox_batch_plan(arr, 1, None, 0, None) == binding.VOX_ERR_INVALID_ARGUMENT
    bad = [
        [(10, (48, 64, 64), 1)],          # dim_x not a multiple of 32
        [(10, (64, 0, 64), 1)],           # empty side
        [(10, (64, 64, 64), 2)],          # unknown flag
        [(-1, (64, 64, 64), 1)],          # negative n
        [(10, (32768, 32, 32), 1)],       # side beyond the brick path
    ]
    for specs in bad:
        a = scene_array(specs)
        assert lib.vox_batch_plan(a, 1, None, 0, ctypes.byref(launch)) == \
            binding.VOX_ERR_INVALID_ARGUMENT, specs
    a = scene_array([(10, (64, 64, 64), 1), (10, (64, 64, 64), 1)])
    a[1].grid = (1 << 40) + 4                                    # misaligned grid
    assert lib.vox_batch_plan(a, 2, None, 0, ctypes.byref(launch)) == binding.VOX_ERR_INVALID_ARGUMENT
    assert b"scene 1" in lib.vox_last_error()
    a = scene_array([(10, (64, 64, 64), 1)])
    a[0].segs = (1 << 30) + 4                                    # only 4-byte aligned
    assert lib.vox_batch_plan(a, 1, None, 0, ctypes.byref(launch)) == binding.VOX_ERR_INVALID_ARGUMENT
    assert b"8-byte" in lib.vox_last_error()
    a = scene_array([(10, (64, 64, 64), 1)])
    a[0].segs = 0                                                # n > 0 without segments
    assert lib.vox_batch_plan(a, 1, None, 0, ctypes.byref(launch)) == binding.VOX_ERR_INVALID_ARGUMENT
    a = scene_array([(10, (64, 64, 64), 1)])
    assert lib.vox_batch_plan(a, 1, None, 0, ctypes.byref(launch)) == binding.VOX_OK
    small = np.zeros(launch.table_bytes - 1, dtype=np.uint8)
    assert lib.vox_batch_plan(a, 1, ctypes.c_void_p(small.ctypes.data), small.nbytes,
                              ctypes.byref(launch)) == binding.VOX_ERR_INVALID_ARGUMENT


def test_launch_cover(lib):
    _, a = plan(lib, [(1000, (512, 512, 512), 1)])
    _, b = plan(lib, [(10**5, (256, 256, 256), 1), (10, (64, 64, 64), 1)])
    bound = binding.VoxBatchLaunch()
    binding.vox_batch_launch_cover(bound, a)
    binding.vox_batch_launch_cover(bound, b)
    for f in ("rows", "bricks", "max_scene_bricks", "work_bytes", "table_bytes"):
        assert getattr(bound, f) == max(getattr(a, f), getattr(b, f)), f
    assert tuple(bound.brick_lg) == (8, 6, 5)
    binding.vox_set_tuning((8, 6, 6))
    _, c = plan(lib, [(10, (64, 64, 64), 1)])
    with pytest.raises(binding.VoxError):
        binding.vox_batch_launch_cover(bound, c)


def test_batch_scenes_host_errors(lib):
    _, launch = plan(lib, [(10, (64, 64, 64), 1)])
    P = ctypes.c_void_p
    fake = P(1 << 20)
    L = ctypes.byref(launch)
    assert lib.vox_batch_scenes(None, L, fake, 1 << 30, None) == binding.VOX_ERR_INVALID_ARGUMENT
    assert lib.vox_batch_scenes(P((1 << 20) + 8), L, fake, 1 << 30, None) == \
        binding.VOX_ERR_INVALID_ARGUMENT
    assert lib.vox_batch_scenes(fake, None, fake, 1 << 30, None) == binding.VOX_ERR_INVALID_ARGUMENT
    assert lib.vox_batch_scenes(fake, L, fake, launch.work_bytes - 1, None) == binding.VOX_ERR_WORKSPACE
    assert lib.vox_batch_scenes(fake, L, P((1 << 20) + 64), 1 << 30, None) == binding.VOX_ERR_WORKSPACE
    bad = binding.VoxBatchLaunch.from_buffer_copy(launch)
    bad.brick_lg[2] = 4
    assert lib.vox_batch_scenes(fake, ctypes.byref(bad), fake, 1 << 30, None) == \
        binding.VOX_ERR_INVALID_ARGUMENT
    bad = binding.VoxBatchLaunch.from_buffer_copy(launch)
    bad.rows = 0
    assert lib.vox_batch_scenes(fake, ctypes.byref(bad), fake, 1 << 30, None) == \
        binding.VOX_ERR_INVALID_ARGUMENT
