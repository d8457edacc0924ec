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
    _fields_ = [("brick_lg", ctypes.c_int32 * 3)]


class VoxScene(ctypes.Structure):
    """struct vox_scene of include/vox.h."""
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


class VoxBatchLaunch(ctypes.Structure):
    """struct vox_batch_launch of include/vox.h."""
    _fields_ = [
        ("rows", ctypes.c_int64),
        ("bricks", ctypes.c_int64),
        ("brick_lg", ctypes.c_int32 * 3),
        ("max_scene_bricks", ctypes.c_int32),
        ("work_bytes", ctypes.c_uint64),
        ("table_bytes", ctypes.c_uint64),
    ]

    def as_dict(self) -> dict:
        return {"rows": int(self.rows), "bricks": int(self.bricks),
                "brick_lg": tuple(int(v) for v in self.brick_lg),
                "max_scene_bricks": int(self.max_scene_bricks),
                "work_bytes": int(self.work_bytes), "table_bytes": int(self.table_bytes)}


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
    lib.vox_grid_workspace_bytes.argtypes = [i64, i32, i32, i32]
    lib.vox_grid_workspace_bytes.restype = sz
    lib.vox_segments_to_grid.argtypes = [P, i64, i32, i32, i32, P, P, u32, P, sz, P]
    lib.vox_segments_to_grid.restype = ctypes.c_int
    LP = ctypes.POINTER(VoxBatchLaunch)
    lib.vox_batch_plan.argtypes = [ctypes.POINTER(VoxScene), i32, P, sz, LP]
    lib.vox_batch_plan.restype = ctypes.c_int
    lib.vox_batch_launch_cover.argtypes = [LP, LP]
    lib.vox_batch_launch_cover.restype = ctypes.c_int
    lib.vox_batch_scenes.argtypes = [P, LP, P, sz, P]
    lib.vox_batch_scenes.restype = ctypes.c_int
    lib.vox_read_status.argtypes = [P, ctypes.POINTER(i32), P]
    lib.vox_read_status.restype = ctypes.c_int
    lib.vox_set_tuning.argtypes = [ctypes.POINTER(VoxTuning)]
    lib.vox_set_tuning.restype = ctypes.c_int
    lib.vox_get_tuning.argtypes = [ctypes.POINTER(VoxTuning)]
    lib.vox_get_tuning.restype = ctypes.c_int
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


def vox_segments_to_grid(segs, dims, grid, counts, flags: int, work, stream=None):
    lib = load()
    _check_segs(segs)
    dx, dy, dz = (int(d) for d in dims)
    st = lib.vox_segments_to_grid(_ptr(segs), segs.shape[0], dx, dy, dz, _ptr(grid), _ptr(counts),
                                  int(flags), _ptr(work), work.numel() * work.element_size(),
                                  _stream(stream))
    _check(lib, st)


def _scene_array(scenes):
    """ctypes array of vox_scene from (segs, dims, grid, counts, flags) tuples
    of device tensors (counts may be None)."""
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
    return arr


def vox_batch_plan(scenes):
    """Plans a batch of (segs, dims, grid, counts, flags) scenes.  Returns
    (table image as a numpy uint8 array, VoxBatchLaunch)."""
    import numpy as np
    lib = load()
    arr = _scene_array(scenes)
    launch = VoxBatchLaunch()
    _check(lib, lib.vox_batch_plan(arr, len(scenes), None, 0, ctypes.byref(launch)))
    table = np.zeros(int(launch.table_bytes), dtype=np.uint8)
    _check(lib, lib.vox_batch_plan(arr, len(scenes), ctypes.c_void_p(table.ctypes.data),
                                   table.nbytes, ctypes.byref(launch)))
    return table, launch


def vox_batch_launch_cover(bound: VoxBatchLaunch, launch: VoxBatchLaunch) -> VoxBatchLaunch:
    """Widens `bound` in place to cover `launch`; returns it."""
    lib = load()
    _check(lib, lib.vox_batch_launch_cover(ctypes.byref(bound), ctypes.byref(launch)))
    return bound


def vox_batch_scenes(d_table, launch: VoxBatchLaunch, work, stream=None):
    """Runs a planned batch; d_table is a device uint8 tensor holding the
    table image."""
    lib = load()
    st = lib.vox_batch_scenes(_ptr(d_table), ctypes.byref(launch), _ptr(work),
                              work.numel() * work.element_size(), _stream(stream))
    _check(lib, st)


def vox_read_status(work, stream=None) -> int:
    lib = load()
    out = ctypes.c_int32(-1)
    _check(lib, lib.vox_read_status(_ptr(work), ctypes.byref(out), _stream(stream)))
    return int(out.value)


def vox_set_tuning(brick_lg=None):
    """Process-wide brick shape (log2 per axis) for grid calls; None = default."""
    lib = load()
    if brick_lg is None:
        _check(lib, lib.vox_set_tuning(None))
    else:
        t = VoxTuning()
        for a in range(3):
            t.brick_lg[a] = int(brick_lg[a])
        _check(lib, lib.vox_set_tuning(ctypes.byref(t)))


def vox_get_tuning():
    lib = load()
    t = VoxTuning()
    _check(lib, lib.vox_get_tuning(ctypes.byref(t)))
    return tuple(int(v) for v in t.brick_lg)


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


def batch_to_grids(scenes, stream=None):
    """Cleared bit-volumes of several scenes in one batched launch sequence.
    `scenes` holds (segs, dims) pairs of device tensors; returns the grids
    (int32 storage of the packed words)."""
    import torch
    if not scenes:
        return []
    dev = scenes[0][0].device
    grids = [torch.empty(grid_words(d), dtype=torch.int32, device=dev) for _, d in scenes]
    table, launch = vox_batch_plan([(s, d, g, None, VOX_GRID_CLEAR)
                                    for (s, d), g in zip(scenes, grids)])
    d_table = torch.from_numpy(table).to(dev)
    work = workspace(launch.work_bytes, dev)
    vox_batch_scenes(d_table, launch, work, stream=stream)
    status = vox_read_status(work, stream=stream)
    if status != VOX_OK:
        raise VoxError(status, load().vox_status_string(status).decode())
    return grids
