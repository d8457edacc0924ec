"""Thin Python binding over the C ABI of libvox.so (include/vox.h).

Argument marshalling only: torch tensors supply device memory and the HIP
stream; every step of the voxelization runs in the library's HIP kernels.
The functions named like the C entry points take tensors and pass their
data pointers; `segments_to_list` / `segments_to_grid` are conveniences that
also allocate the outputs and the workspace with torch.

There is no fallback: if libvox.so is missing or cannot be loaded, `load()`
raises.
"""

from __future__ import annotations

import ctypes
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
LIBRARY = os.path.join(PKG, "libvox.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "vox.h")

VOX_OK = 0
VOX_ERR_INVALID_ARGUMENT = 1
VOX_ERR_OUT_OF_RANGE = 2
VOX_ERR_CAPACITY = 3
VOX_ERR_DEVICE = 4
VOX_ERR_WORKSPACE = 5
VOX_ERR_BATCH_MISMATCH = 6
VOX_GRID_CLEAR = 1
VOX_GRID_EUCLID = 2

_lib = None


class VoxError(RuntimeError):
    """A vox_* call returned a status other than VOX_OK."""

    def __init__(self, status: int, message: str):
        super().__init__("%s (status %d)" % (message, status))
        self.status = status


class VoxTuning(ctypes.Structure):
    """struct vox_tuning of include/vox.h."""
    _fields_ = [("brick_lg", ctypes.c_int32 * 3), ("fill_wgs_per_cu", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 4)]


def make_tuning(brick_lg=None, fill_wgs_per_cu: int = 0) -> VoxTuning:
    t = VoxTuning()
    if brick_lg is not None:
        for a in range(3):
            t.brick_lg[a] = int(brick_lg[a])
    t.fill_wgs_per_cu = int(fill_wgs_per_cu)
    return t


class VoxScene(ctypes.Structure):
    """struct vox_scene of include/vox.h (48 bytes)."""
    _fields_ = [
        ("segs", ctypes.c_void_p),
        ("n", ctypes.c_int64),
        ("dim_x", ctypes.c_int32),
        ("dim_y", ctypes.c_int32),
        ("dim_z", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("grid", ctypes.c_void_p),
        ("counts", ctypes.c_void_p),
    ]


VOX_OP_GRID = 2
VOX_OP_BATCH = 3
VOX_DEVICE_STATUS_OUT_OF_RANGE = 1
VOX_DEVICE_STATUS_CAPACITY = 2
VOX_DEVICE_STATUS_MISMATCH = 4
VOX_DEVICE_STATUS_INVALID = 8


def load(path: str | None = None):
    """Load libvox.so (built by `python -m paper_2009_09500_amd.build`)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIBRARY
    if not os.path.exists(p):
        raise RuntimeError("libvox.so not found at %s: build it with "
                           "`python -m paper_2009_09500_amd.build`" % p)
    # torch first: its HIP libraries ask for the HIP runtime by its bare file
    # name, libvox.so by its versioned soname.  Loaded in this order, libvox.so
    # binds to torch's runtime; the other way round the process would hold two
    # HIP runtimes, and the second to touch the GPU finds no device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(p)
    P, i64, i32, u32, sz = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                            ctypes.c_uint32, ctypes.c_size_t)
    lib.vox_abi_version.argtypes = []
    lib.vox_abi_version.restype = ctypes.c_int
    lib.vox_last_error.argtypes = []
    lib.vox_last_error.restype = ctypes.c_char_p
    lib.vox_status_string.argtypes = [ctypes.c_int]
    lib.vox_status_string.restype = ctypes.c_char_p
    lib.vox_list_workspace_bytes.argtypes = [i64, i64]
    lib.vox_list_workspace_bytes.restype = sz
    lib.vox_segments_to_list.argtypes = [P, i64, P, P, i64, P, P, sz, P]
    lib.vox_segments_to_list.restype = ctypes.c_int
    lib.vox_segments_to_list_euclid.argtypes = [P, i64, P, P, i64, P, P, sz, P]
    lib.vox_segments_to_list_euclid.restype = ctypes.c_int
    lib.vox_segments_to_list32.argtypes = [P, i64, P, P, i64, P, P, sz, P]
    lib.vox_segments_to_list32.restype = ctypes.c_int
    lib.vox_segments_to_list_noalloc.argtypes = [P, i64, P, P, i64, P, P]
    lib.vox_segments_to_list_noalloc.restype = ctypes.c_int
    lib.vox_grid_workspace_bytes.argtypes = [i64, i32, i32, i32]
    lib.vox_grid_workspace_bytes.restype = sz
    lib.vox_segments_to_grid.argtypes = [P, i64, i32, i32, i32, P, P, u32, P, sz, P]
    lib.vox_segments_to_grid.restype = ctypes.c_int
    TP = ctypes.POINTER(VoxTuning)
    lib.vox_workspace_bytes.argtypes = [ctypes.c_int, i64, i32]
    lib.vox_workspace_bytes.restype = sz
    lib.vox_batch_scenes.argtypes = [P, i32, i64, TP, P, sz, P]
    lib.vox_batch_scenes.restype = ctypes.c_int
    lib.vox_device_status.argtypes = [P]
    lib.vox_device_status.restype = ctypes.c_void_p
    lib.vox_read_status.argtypes = [P, ctypes.POINTER(i32), P]
    lib.vox_read_status.restype = ctypes.c_int
    lib.vox_read_batch_info.argtypes = [P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(i32), P]
    lib.vox_read_batch_info.restype = ctypes.c_int
    lib.vox_tuning_cache_set.argtypes = [i32, i32, i32, i64, TP]
    lib.vox_tuning_cache_set.restype = ctypes.c_int
    lib.vox_tuning_cache_get.argtypes = [i32, i32, i32, i64, TP, ctypes.POINTER(i32)]
    lib.vox_tuning_cache_get.restype = ctypes.c_int
    lib.vox_tuning_cache_clear.argtypes = []
    lib.vox_tuning_cache_clear.restype = None
    lib.vox_profile_enable.argtypes = [ctypes.c_int]
    lib.vox_profile_enable.restype = ctypes.c_int
    lib.vox_profile_reset.argtypes = []
    lib.vox_profile_reset.restype = None
    lib.vox_profile_count.argtypes = []
    lib.vox_profile_count.restype = ctypes.c_int
    lib.vox_profile_read.argtypes = [ctypes.c_int, ctypes.c_char_p, sz,
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    lib.vox_profile_read.restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def header_functions(header: str = HEADER) -> list:
    """Names of the functions declared in include/vox.h."""
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vox_[a-z0-9_]+)\s*\(", text)))


def _check(lib, status: int):
    if status != VOX_OK:
        raise VoxError(status, lib.vox_last_error().decode() or
                       lib.vox_status_string(status).decode())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _check_segs(segs):
    import torch
    if segs.dtype != torch.int32 or segs.dim() != 2 or segs.shape[1] != 6:
        raise ValueError("segments must be an int32 tensor of shape [n, 6]")
    if not segs.is_cuda or not segs.is_contiguous():
        raise ValueError("segments must be a contiguous device tensor")


# ------------------------------------------------------- entry-point names

def vox_list_workspace_bytes(n: int, capacity: int) -> int:
    return int(load().vox_list_workspace_bytes(n, capacity))


def vox_grid_workspace_bytes(n: int, dims) -> int:
    return int(load().vox_grid_workspace_bytes(n, *[int(d) for d in dims]))


def vox_segments_to_list(segs, offsets, voxels, capacity: int, work, want_total: bool = False,
                         stream=None, euclid: bool = False, wide: bool = False):
    """Calls vox_segments_to_list (vox_segments_to_list_euclid if euclid,
    vox_segments_to_list32 if wide); returns the total if want_total."""
    if euclid and wide:
        raise ValueError("the int32 lists use the Chebyshev length")
    lib = load()
    _check_segs(segs)
    total = ctypes.c_int64(-1)
    fn = (lib.vox_segments_to_list_euclid if euclid else
          lib.vox_segments_to_list32 if wide else lib.vox_segments_to_list)
    st = fn(_ptr(segs), segs.shape[0], _ptr(offsets), _ptr(voxels),
            int(capacity), ctypes.byref(total) if want_total else None,
            _ptr(work), work.numel() * work.element_size(), _stream(stream))
    if want_total and st in (VOX_ERR_CAPACITY, VOX_ERR_OUT_OF_RANGE):
        raise VoxError(st, lib.vox_last_error().decode())
    _check(lib, st)
    return int(total.value) if want_total else None


def vox_segments_to_list_noalloc(segs, offsets, voxels, capacity: int, want_total: bool = False,
                                 stream=None):
    """Calls vox_segments_to_list_noalloc (no workspace argument); returns
    the total if want_total."""
    lib = load()
    _check_segs(segs)
    total = ctypes.c_int64(-1)
    st = lib.vox_segments_to_list_noalloc(_ptr(segs), segs.shape[0], _ptr(offsets), _ptr(voxels),
                                          int(capacity), ctypes.byref(total) if want_total else None,
                                          _stream(stream))
    if want_total and st in (VOX_ERR_CAPACITY, VOX_ERR_OUT_OF_RANGE):
        raise VoxError(st, lib.vox_last_error().decode())
    _check(lib, st)
    return int(total.value) if want_total else None


def vox_segments_to_grid(segs, dims, grid, counts, flags: int, work, stream=None):
    lib = load()
    _check_segs(segs)
    dx, dy, dz = (int(d) for d in dims)
    st = lib.vox_segments_to_grid(_ptr(segs), segs.shape[0], dx, dy, dz, _ptr(grid), _ptr(counts),
                                  int(flags), _ptr(work), work.numel() * work.element_size(),
                                  _stream(stream))
    _check(lib, st)


def scene_table(scenes):
    """Host image (numpy uint8, 48 bytes a scene) of a vox_scene array from
    (segs, dims, grid, counts, flags) tuples of device tensors (counts may be
    None); copy it to device memory for vox_batch_scenes."""
    import numpy as np
    arr = (VoxScene * len(scenes))()
    for i, (segs, dims, grid, counts, flags) in enumerate(scenes):
        _check_segs(segs)
        sc = arr[i]
        sc.segs = segs.data_ptr() if segs.shape[0] > 0 else 0
        sc.n = segs.shape[0]
        sc.dim_x, sc.dim_y, sc.dim_z = (int(d) for d in dims)
        sc.flags = int(flags)
        sc.grid = grid.data_ptr()
        sc.counts = counts.data_ptr() if counts is not None else 0
    return np.frombuffer(bytes(arr), dtype=np.uint8).copy()


def vox_workspace_bytes(op: int, n_segments: int, n_scenes: int) -> int:
    return int(load().vox_workspace_bytes(int(op), int(n_segments), int(n_scenes)))


def batch_workspace_bytes(total_segments: int, n_scenes: int) -> int:
    return vox_workspace_bytes(VOX_OP_BATCH, total_segments, n_scenes)


def vox_batch_scenes(d_scenes, n_scenes: int, total_segments: int, work, tuning=None, stream=None):
    """Calls vox_batch_scenes; d_scenes is a device uint8 tensor holding a
    vox_scene array (scene_table), tuning a VoxTuning or None."""
    lib = load()
    st = lib.vox_batch_scenes(_ptr(d_scenes), int(n_scenes), int(total_segments),
                              ctypes.byref(tuning) if tuning is not None else None, _ptr(work),
                              work.numel() * work.element_size(), _stream(stream))
    _check(lib, st)


def vox_read_batch_info(work, stream=None):
    """(piece records needed, whether the direct kernels served every scene)
    of the last brick-path call on `work` (synchronises)."""
    lib = load()
    pieces = ctypes.c_uint64(0)
    direct_all = ctypes.c_int32(0)
    _check(lib, lib.vox_read_batch_info(_ptr(work), ctypes.byref(pieces), ctypes.byref(direct_all),
                                        _stream(stream)))
    return int(pieces.value), bool(direct_all.value)


def vox_device_status(work) -> int:
    """Device address of the workspace's status word."""
    return int(load().vox_device_status(_ptr(work)) or 0)


def vox_read_status(work, stream=None) -> int:
    lib = load()
    out = ctypes.c_int32(-1)
    _check(lib, lib.vox_read_status(_ptr(work), ctypes.byref(out), _stream(stream)))
    return int(out.value)


def vox_tuning_cache_set(dims, n_segments: int, tuning):
    """Autotune cache entry for (dims, n_segments); dims (0, 0, 0) keys
    batches by their total segment count; tuning None removes it."""
    lib = load()
    _check(lib, lib.vox_tuning_cache_set(*[int(d) for d in dims], int(n_segments),
                                         ctypes.byref(tuning) if tuning is not None else None))


def vox_tuning_cache_get(dims, n_segments: int):
    """The cache entry as a VoxTuning, or None."""
    lib = load()
    t = VoxTuning()
    found = ctypes.c_int32(0)
    _check(lib, lib.vox_tuning_cache_get(*[int(d) for d in dims], int(n_segments), ctypes.byref(t),
                                         ctypes.byref(found)))
    return t if found.value else None


def vox_tuning_cache_clear():
    load().vox_tuning_cache_clear()


def vox_profile_enable(enable: bool = True):
    load().vox_profile_enable(1 if enable else 0)


def vox_profile_reset():
    load().vox_profile_reset()


def vox_profile_records() -> dict:
    """{kernel name: (total ms, launches)} of the library's kernel timing."""
    lib = load()
    out = {}
    buf = ctypes.create_string_buffer(128)
    for i in range(lib.vox_profile_count()):
        ms = ctypes.c_double(0)
        cnt = ctypes.c_int64(0)
        _check(lib, lib.vox_profile_read(i, buf, 128, ctypes.byref(ms), ctypes.byref(cnt)))
        out[buf.value.decode()] = (float(ms.value), int(cnt.value))
    return out


# ------------------------------------------------------------- conveniences

def workspace(nbytes: int, device):
    """A 256-byte-aligned device workspace of at least nbytes (torch
    allocations are 256-byte aligned)."""
    import torch
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def segments_to_list(segs, stream=None, euclid: bool = False, wide: bool = False):
    """(offsets int64 [n+1], voxels int16 [total, 3]) for a device segment
    tensor; two library calls (size query, then generation).  euclid: the
    paper's eq. (1) length (vox_segments_to_list_euclid); wide: int32
    coordinates (vox_segments_to_list32)."""
    import torch
    _check_segs(segs)
    n = segs.shape[0]
    offsets = torch.empty(n + 1, dtype=torch.int64, device=segs.device)
    work = workspace(vox_list_workspace_bytes(n, 0), segs.device)
    total = vox_segments_to_list(segs, offsets, None, 0, work, want_total=True, stream=stream, euclid=euclid,
                                 wide=wide)
    voxels = torch.empty((max(total, 1), 3), dtype=torch.int32 if wide else torch.int16, device=segs.device)
    work = workspace(vox_list_workspace_bytes(n, total), segs.device)
    vox_segments_to_list(segs, offsets, voxels, total, work, stream=stream, euclid=euclid, wide=wide)
    return offsets, voxels[:total]


def grid_words(dims) -> int:
    dx, dy, dz = (int(d) for d in dims)
    return (dx * dy * dz + 31) // 32


def segments_to_grid(segs, dims, grid=None, want_counts: bool = False, stream=None, euclid: bool = False):
    """Packed uint32 bit-volume (as int32 storage) of the segments; a new
    cleared volume unless `grid` is given (then ORed into it).  euclid: the
    paper's eq. (1) length (VOX_GRID_EUCLID)."""
    import torch
    _check_segs(segs)
    flags = VOX_GRID_EUCLID if euclid else 0
    if grid is None:
        grid = torch.empty(grid_words(dims), dtype=torch.int32, device=segs.device)
        flags |= VOX_GRID_CLEAR
    counts = torch.empty(segs.shape[0], dtype=torch.int32, device=segs.device) if want_counts else None
    work = workspace(vox_grid_workspace_bytes(segs.shape[0], dims), segs.device)
    vox_segments_to_grid(segs, dims, grid, counts, flags, work, stream=stream)
    status = vox_read_status(work, stream=stream)
    if status != VOX_OK:
        raise VoxError(status, load().vox_status_string(status).decode())
    return (grid, counts) if want_counts else grid


def batch_to_grids(scenes, stream=None, tuning=None):
    """Cleared bit-volumes of several scenes in one batched launch sequence.
    `scenes` holds (segs, dims) pairs of device tensors; returns the grids
    (int32 storage of the packed words)."""
    import torch
    if not scenes:
        return []
    dev = scenes[0][0].device
    grids = [torch.empty(grid_words(d), dtype=torch.int32, device=dev) for _, d in scenes]
    table = scene_table([(s, d, g, None, VOX_GRID_CLEAR) for (s, d), g in zip(scenes, grids)])
    d_scenes = torch.from_numpy(table).to(dev)
    total = sum(int(s.shape[0]) for s, _ in scenes)
    work = workspace(batch_workspace_bytes(total, len(scenes)), dev)
    vox_batch_scenes(d_scenes, len(scenes), total, work, tuning=tuning, stream=stream)
    status = vox_read_status(work, stream=stream)
    if status != VOX_OK:
        raise VoxError(status, load().vox_status_string(status).decode())
    return grids
