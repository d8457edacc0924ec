"""Batch planning on the CPU: the per-scene rule the plan kernel applies
(which scenes the LDS brick kernels serve, which the direct kernels serve,
histogram rows, brick counts, the argument rules), the batch workspace
query, the host-side checks of vox_batch_scenes, the autotune cache and the
status-word address.  No call here reaches the GPU."""

import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2009_09500_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "cpp", "plan_check.cpp")
CLEAR, EUCLID = 1, 2
F_CLEAR, F_DIRECT, F_EUCLID, F_A8 = 1, 2, 4, 8
SEGS, GRID = 1 << 30, 1 << 40          # fake 256-aligned device addresses


@pytest.fixture(scope="module")
def lib():
    return binding.load()


@pytest.fixture(scope="module")
def planner(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("plan") / "plan_check")
    subprocess.check_call([hipcc, "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2009_09500_amd", "csrc"), "-o", out, SRC])

    def run(lg, scenes, per_row=4096):
        """scenes: dicts with n, dims and optional flags, segs, grid, counts;
        per_row: segments per histogram row (4096 in batches, 512 in plain
        calls)."""
        lines = ["%d %d %d %d %d" % (lg[0], lg[1], lg[2], per_row, len(scenes))]
        for sc in scenes:
            lines.append("%d %d %d %d %d %d %d %d" % (
                sc.get("segs", SEGS), sc["n"], sc["dims"][0], sc["dims"][1], sc["dims"][2],
                sc.get("flags", CLEAR), sc.get("grid", GRID), sc.get("counts", 0)))
        r = subprocess.run([out], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True)
        res = []
        for ln in r.stdout.split("\n"):
            if ln.strip():
                v = [int(x) for x in ln.split()]
                res.append(dict(valid=bool(v[0]), flags=v[1], rows=v[2], nbricks=v[3], nb=tuple(v[4:7]),
                                dim=tuple(v[7:10]), n=v[10]))
        return res
    return run


def expected_rows(n, per_row=4096):
    return min(256, max(1, -(-n // per_row)))


def test_brick_scenes(planner):
    lg = (8, 6, 5)
    specs = [dict(n=1000, dims=(64, 64, 64)), dict(n=0, dims=(128, 96, 64), flags=0),
             dict(n=200000, dims=(512, 512, 512)), dict(n=5000, dims=(256, 128, 256)),
             dict(n=4096 * 300, dims=(2048, 2048, 2048))]
    for sc, out in zip(specs, planner(lg, specs)):
        nb = tuple(-(-d // (1 << l)) for d, l in zip(sc["dims"], lg))
        assert out["valid"] and out["nb"] == nb and out["nbricks"] == nb[0] * nb[1] * nb[2]
        assert out["flags"] == (F_CLEAR if sc.get("flags", CLEAR) else 0) | F_A8
        assert out["rows"] == expected_rows(sc["n"]) and out["dim"] == sc["dims"] and out["n"] == sc["n"]
    # Plain calls: rows of 512 segments, at most 256.
    plain = planner(lg, specs, per_row=512)
    assert [o["rows"] for o in plain] == [2, 1, 256, 10, 256]


def test_direct_scenes(planner):
    """Scenes the bricks cannot serve go to the direct kernels: rows not
    whole words, sides beyond 16384, too many bricks, the Euclidean N in a
    volume whose diagonal reaches 16385 (N up to 16384 keeps 2N within the
    fill's 16-bit halves), a segment array that is only 4-byte aligned."""
    lg = (8, 6, 5)
    specs = [dict(n=10, dims=(48, 64, 64)), dict(n=10, dims=(32768, 32, 32)),
             dict(n=10, dims=(16384, 16384, 64)), dict(n=10, dims=(16384, 512, 64), flags=CLEAR | EUCLID),
             dict(n=10, dims=(64, 64, 64), segs=SEGS + 4)]
    res = planner(lg, specs)
    for sc, out in zip(specs, res):
        assert out["valid"] and out["flags"] & F_DIRECT and out["rows"] == 0 and out["nbricks"] == 0, sc
        assert out["dim"] == sc["dims"] and out["n"] == 10
    assert res[3]["flags"] & F_EUCLID and res[3]["flags"] & F_A8
    assert not res[4]["flags"] & F_A8


def test_euclid_brick_scenes(planner):
    """The Euclidean N takes the bricks while the volume's diagonal
    (sqrt of the sum of (side - 1)^2) stays below 16385; the same volumes
    with the Chebyshev N take them regardless."""
    lg = (8, 6, 5)
    # 16383^2 + 127^2 + 63^2 < 16385^2 <= 16383^2 + 511^2 + 63^2
    specs = [dict(n=10, dims=(64, 64, 64), flags=CLEAR | EUCLID), dict(n=10, dims=(16384, 128, 64), flags=EUCLID),
             dict(n=10, dims=(16384, 512, 64), flags=EUCLID), dict(n=10, dims=(16384, 512, 64), flags=0)]
    res = planner(lg, specs)
    assert [bool(o["flags"] & F_DIRECT) for o in res] == [False, False, True, False]
    assert res[0]["flags"] == F_CLEAR | F_EUCLID | F_A8 and res[0]["rows"] == expected_rows(10)
    assert res[1]["flags"] == F_EUCLID | F_A8 and res[1]["nb"] == (64, 2, 2)


def test_invalid_scenes(planner):
    bad = [dict(n=-1, dims=(64, 64, 64)), dict(n=10, dims=(64, 0, 64)), dict(n=10, dims=(1 << 21, 8, 8)),
           dict(n=10, dims=(64, 64, 64), flags=4), dict(n=10, dims=(64, 64, 64), segs=0),
           dict(n=10, dims=(64, 64, 64), segs=SEGS + 2), dict(n=10, dims=(64, 64, 64), grid=GRID + 4),
           dict(n=10, dims=(64, 64, 64), grid=0), dict(n=10, dims=(64, 64, 64), counts=GRID + 2),
           dict(n=1 << 31, dims=(64, 64, 64)), dict(n=10, dims=(1 << 20, 1 << 20, 1 << 0))]
    res = planner((8, 6, 5), bad[:-1] + [dict(n=10, dims=(1 << 19, 1 << 19, 2))])
    for sc, out in zip(bad, res):
        assert not out["valid"], sc
        assert out["n"] == 0 and out["flags"] & F_DIRECT      # no segment is ever read
    ok = planner((8, 6, 5), [dict(n=0, dims=(64, 64, 64), segs=0), dict(n=10, dims=(1 << 20, 1 << 18, 1))])
    assert all(o["valid"] for o in ok)


def test_shape_changes_bricks(planner):
    for lg in ((8, 6, 6), (7, 6, 6), (7, 7, 6)):
        out = planner(lg, [dict(n=100, dims=(512, 512, 512))])[0]
        nb = tuple(512 >> l for l in lg)
        assert out["nb"] == nb and not out["flags"] & F_DIRECT


def test_batch_workspace_query(lib):
    w = lambda n, s: lib.vox_workspace_bytes(binding.VOX_OP_BATCH, n, s)
    assert 0 < w(1000, 1) < w(10**6, 1) < w(10**6, 32)
    assert w(10**6, 1) >= 16 * 16 * 10**6                 # 16 records of 16 bytes a segment
    assert w(-1, 1) == 0 and w(10, 0) == 0 and w(10, 65537) == 0
    assert lib.vox_workspace_bytes(99, 10, 1) == 0


def test_grid_compact_workspace_query(lib):
    """The compact grid workspace is the one-scene batch workspace; it is far
    below the worst case for the arbitrary-length workload's shape, and a
    workspace below its table and histogram part is refused before any
    launch."""
    g = lambda n: lib.vox_workspace_bytes(binding.VOX_OP_GRID, n, 1)
    assert g(10**6) == lib.vox_workspace_bytes(binding.VOX_OP_BATCH, 10**6, 1)
    assert lib.vox_workspace_bytes(binding.VOX_OP_GRID, 10**6, 2) == 0
    n, dims = 4194304, (2048, 2048, 2048)
    full = lib.vox_grid_workspace_bytes(n, *dims)
    assert 0 < g(n) < full / 4
    P = ctypes.c_void_p
    fake = P(1 << 20)
    st = lib.vox_segments_to_grid(fake, n, *dims, fake, None, binding.VOX_GRID_CLEAR, fake, 1 << 20, None)
    assert st == binding.VOX_ERR_WORKSPACE


def test_batch_host_errors(lib):
    P = ctypes.c_void_p
    fake = P(1 << 20)
    big = 1 << 40
    T = ctypes.byref
    assert lib.vox_batch_scenes(None, 1, 10, None, fake, big, None) == binding.VOX_ERR_INVALID_ARGUMENT
    assert lib.vox_batch_scenes(P((1 << 20) + 4), 1, 10, None, fake, big, None) == binding.VOX_ERR_INVALID_ARGUMENT
    assert lib.vox_batch_scenes(fake, 0, 10, None, fake, big, None) == binding.VOX_ERR_INVALID_ARGUMENT
    assert lib.vox_batch_scenes(fake, 65537, 10, None, fake, big, None) == binding.VOX_ERR_INVALID_ARGUMENT
    assert lib.vox_batch_scenes(fake, 1, -1, None, fake, big, None) == binding.VOX_ERR_INVALID_ARGUMENT
    for t in (binding.make_tuning((8, 6, 4)), binding.make_tuning((8, 6, 6), 2), binding.make_tuning(None, 3)):
        assert lib.vox_batch_scenes(fake, 1, 10, T(t), fake, big, None) == binding.VOX_ERR_INVALID_ARGUMENT
    t = binding.make_tuning((8, 6, 5))
    t.reserved[2] = 1
    assert lib.vox_batch_scenes(fake, 1, 10, T(t), fake, big, None) == binding.VOX_ERR_INVALID_ARGUMENT
    assert lib.vox_batch_scenes(fake, 1, 10, None, None, big, None) == binding.VOX_ERR_WORKSPACE
    assert lib.vox_batch_scenes(fake, 1, 10, None, P((1 << 20) + 64), big, None) == binding.VOX_ERR_WORKSPACE
    assert lib.vox_batch_scenes(fake, 1, 10, None, fake, 1024, None) == binding.VOX_ERR_WORKSPACE
    assert b"workspace" in lib.vox_last_error()


def test_tuning_cache(lib):
    binding.vox_tuning_cache_clear()
    try:
        assert binding.vox_tuning_cache_get((512, 512, 512), 100_000) is None
        binding.vox_tuning_cache_set((512, 512, 512), 100_000, binding.make_tuning((7, 6, 6), 1))
        t = binding.vox_tuning_cache_get((512, 512, 512), 120_000)       # same power-of-two bucket
        assert tuple(t.brick_lg) == (7, 6, 6) and t.fill_wgs_per_cu == 1
        assert binding.vox_tuning_cache_get((512, 512, 512), 300_000) is None
        assert binding.vox_tuning_cache_get((512, 512, 256), 100_000) is None
        # The plain call's workspace follows the cached shape (brick path: > 16384 segments).
        before = lib.vox_grid_workspace_bytes(100_000, 512, 512, 512)
        binding.vox_tuning_cache_set((512, 512, 512), 100_000, binding.make_tuning((8, 6, 6)))
        assert lib.vox_grid_workspace_bytes(100_000, 512, 512, 512) != before
        binding.vox_tuning_cache_set((512, 512, 512), 100_000, None)
        assert binding.vox_tuning_cache_get((512, 512, 512), 100_000) is None
        with pytest.raises(binding.VoxError):
            binding.vox_tuning_cache_set((512, 512, 512), 10, binding.make_tuning((9, 9, 9)))
        binding.vox_tuning_cache_set((0, 0, 0), 1 << 20, binding.make_tuning((8, 6, 6)))
        assert tuple(binding.vox_tuning_cache_get((0, 0, 0), 1 << 20).brick_lg) == (8, 6, 6)
    finally:
        binding.vox_tuning_cache_clear()


def test_device_status_address(lib):
    assert lib.vox_device_status(ctypes.c_void_p(1 << 24)) == 1 << 24
    assert not lib.vox_device_status(None)
