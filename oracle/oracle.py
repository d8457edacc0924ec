"""Python access to the CPU oracle in vox_oracle.c.

TEST INFRASTRUCTURE ONLY: the tests, the package smoke check and the
benchmark's CPU-baseline leg use this module to compute the expected output of
the parametric voxelization (arXiv 2009.09500, Section 3, eq. (2)-(3) and the
algorithm of Fig. 3, with N = max|d_a| and round-half-up voxel rounding).  The
product path never imports it.  It shares no code with the HIP library.
The `*_euclid` functions state the paper's literal variant with the
Euclidean N of eq. (1) (N = int(|E - S|), consecutive duplicates removed).

The C source is compiled with gcc into oracle/liboracle.so by `build()`
(called by the package build step and on first use).  `Oracle(path)` wraps
any build of the same source, which lets the tests check that their pins
reject deliberately broken builds of it.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "vox_oracle.c")
LIBRARY = os.path.join(_HERE, "liboracle.so")


def compile_source(src: str, out: str) -> str:
    """gcc -O2, single-threaded, no vectorisation flags beyond -O2."""
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Werror", "-shared",
                           "-fPIC", "-o", tmp, src])
    os.replace(tmp, out)
    return out


NATIVE_LIBRARY = os.path.join(_HERE, "liboracle_native.so")


def compile_native(src: str, out: str) -> str:
    """gcc -O2 -march=native: the same source tuned for the host it is built
    on (the benchmark's CPU-baseline leg builds it where it runs)."""
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-march=native", "-std=c99", "-Wall", "-Werror", "-shared",
                           "-fPIC", "-o", tmp, src])
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile vox_oracle.c into oracle/liboracle.so."""
    if force or not os.path.exists(LIBRARY) or \
            os.path.getmtime(LIBRARY) < os.path.getmtime(SOURCE):
        compile_source(SOURCE, LIBRARY)
    return LIBRARY


def _segs(segs) -> np.ndarray:
    a = np.ascontiguousarray(segs, dtype=np.int32)
    if a.ndim != 2 or a.shape[1] != 6:
        raise ValueError("segments must have shape [n, 6]")
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Oracle:
    """numpy front end over one build of vox_oracle.c."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        P, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        lib.vox_oracle_length.argtypes = [P]
        lib.vox_oracle_length.restype = i64
        lib.vox_oracle_voxel.argtypes = [P, i64, P]
        lib.vox_oracle_voxel.restype = None
        lib.vox_oracle_counts.argtypes = [P, i64, P]
        lib.vox_oracle_counts.restype = None
        lib.vox_oracle_offsets.argtypes = [P, i64, P]
        lib.vox_oracle_offsets.restype = i64
        lib.vox_oracle_list.argtypes = [P, i64, P, i64]
        lib.vox_oracle_list.restype = i64
        lib.vox_oracle_list32.argtypes = [P, i64, P, i64]
        lib.vox_oracle_list32.restype = i64
        lib.vox_oracle_grid.argtypes = [P, i64, i32, i32, i32, P, ctypes.c_int]
        lib.vox_oracle_grid.restype = i64
        lib.vox_oracle_length_euclid.argtypes = [P]
        lib.vox_oracle_length_euclid.restype = i64
        lib.vox_oracle_sample_euclid.argtypes = [P, i64, P]
        lib.vox_oracle_sample_euclid.restype = None
        lib.vox_oracle_counts_euclid.argtypes = [P, i64, P]
        lib.vox_oracle_counts_euclid.restype = None
        lib.vox_oracle_offsets_euclid.argtypes = [P, i64, P]
        lib.vox_oracle_offsets_euclid.restype = i64
        lib.vox_oracle_list_euclid.argtypes = [P, i64, P, i64]
        lib.vox_oracle_list_euclid.restype = i64
        lib.vox_oracle_grid_euclid.argtypes = [P, i64, i32, i32, i32, P, ctypes.c_int]
        lib.vox_oracle_grid_euclid.restype = i64
        self._lib = lib
        self.path = path

    def counts(self, segs) -> np.ndarray:
        """int32 [n]: N_i + 1 voxels per segment."""
        s = _segs(segs)
        out = np.empty(s.shape[0], dtype=np.int32)
        self._lib.vox_oracle_counts(_ptr(s), s.shape[0], _ptr(out))
        return out

    def offsets(self, segs) -> np.ndarray:
        """int64 [n+1]: exclusive prefix sum of the counts; last = total."""
        s = _segs(segs)
        out = np.empty(s.shape[0] + 1, dtype=np.int64)
        self._lib.vox_oracle_offsets(_ptr(s), s.shape[0], _ptr(out))
        return out

    def voxel(self, seg, k: int) -> tuple:
        """Voxel k (0 <= k <= N) of one segment."""
        s = _segs(np.asarray(seg).reshape(1, 6))
        out = np.empty(3, dtype=np.int64)
        self._lib.vox_oracle_voxel(_ptr(s), int(k), _ptr(out))
        return tuple(int(v) for v in out)

    def voxel_list(self, segs) -> np.ndarray:
        """int16 [total, 3]: every segment's voxels, S to E, in input order."""
        s = _segs(segs)
        total = int(self.offsets(s)[-1])
        out = np.empty((max(total, 0), 3), dtype=np.int16)
        got = self._lib.vox_oracle_list(_ptr(s), s.shape[0], _ptr(out), total)
        if got < 0:
            raise ValueError("end point outside the int16 range")
        return out

    def voxel_list32(self, segs) -> np.ndarray:
        """int32 [total, 3]: the same lists with int32 coordinates, for
        segments with every |P1_a - P0_a| < 2^30."""
        s = _segs(segs)
        total = int(self.offsets(s)[-1])
        out = np.empty((max(total, 0), 3), dtype=np.int32)
        got = self._lib.vox_oracle_list32(_ptr(s), s.shape[0], _ptr(out), total)
        if got < 0:
            raise ValueError("a segment spans 2^30 or more along an axis")
        return out

    def grid(self, segs, dims, base=None) -> np.ndarray:
        """uint32 [ceil(dx*dy*dz/32)] packed bit-volume (bit (z*dy+y)*dx+x,
        LSB first).  base=None starts empty; otherwise ORs into a copy."""
        s = _segs(segs)
        dx, dy, dz = (int(v) for v in dims)
        nwords = (dx * dy * dz + 31) // 32
        if base is None:
            out = np.empty(nwords, dtype=np.uint32)
            clear = 1
        else:
            out = np.array(base, dtype=np.uint32, copy=True).reshape(-1)
            if out.size != nwords:
                raise ValueError("base has the wrong size")
            clear = 0
        got = self._lib.vox_oracle_grid(_ptr(s), s.shape[0], dx, dy, dz, _ptr(out), clear)
        if got < 0:
            raise ValueError("end point outside the volume")
        return out

    # Euclidean-length variant (eq. (1): N = int(|E - S|), consecutive
    # duplicates removed).

    def length_euclid(self, seg) -> int:
        s = _segs(np.asarray(seg).reshape(1, 6))
        return int(self._lib.vox_oracle_length_euclid(_ptr(s)))

    def sample_euclid(self, seg, k: int) -> tuple:
        """Voxel of sample k (0 <= k <= N_e), before duplicates are removed."""
        s = _segs(np.asarray(seg).reshape(1, 6))
        out = np.empty(3, dtype=np.int64)
        self._lib.vox_oracle_sample_euclid(_ptr(s), int(k), _ptr(out))
        return tuple(int(v) for v in out)

    def counts_euclid(self, segs) -> np.ndarray:
        s = _segs(segs)
        out = np.empty(s.shape[0], dtype=np.int32)
        self._lib.vox_oracle_counts_euclid(_ptr(s), s.shape[0], _ptr(out))
        return out

    def offsets_euclid(self, segs) -> np.ndarray:
        s = _segs(segs)
        out = np.empty(s.shape[0] + 1, dtype=np.int64)
        self._lib.vox_oracle_offsets_euclid(_ptr(s), s.shape[0], _ptr(out))
        return out

    def voxel_list_euclid(self, segs) -> np.ndarray:
        s = _segs(segs)
        total = int(self.offsets_euclid(s)[-1])
        out = np.empty((max(total, 0), 3), dtype=np.int16)
        got = self._lib.vox_oracle_list_euclid(_ptr(s), s.shape[0], _ptr(out), total)
        if got < 0:
            raise ValueError("end point outside the int16 range")
        return out

    def grid_euclid(self, segs, dims, base=None) -> np.ndarray:
        s = _segs(segs)
        dx, dy, dz = (int(v) for v in dims)
        nwords = (dx * dy * dz + 31) // 32
        if base is None:
            out = np.empty(nwords, dtype=np.uint32)
            clear = 1
        else:
            out = np.array(base, dtype=np.uint32, copy=True).reshape(-1)
            if out.size != nwords:
                raise ValueError("base has the wrong size")
            clear = 0
        got = self._lib.vox_oracle_grid_euclid(_ptr(s), s.shape[0], dx, dy, dz, _ptr(out), clear)
        if got < 0:
            raise ValueError("end point outside the volume")
        return out


_default = None


def native() -> Oracle:
    """The oracle built with -march=native on this host (for timing only;
    always rebuilt, since the tree may have been built on another host)."""
    return Oracle(compile_native(SOURCE, NATIVE_LIBRARY))


def default() -> Oracle:
    global _default
    if _default is None:
        if not os.path.exists(LIBRARY) or \
                os.path.getmtime(LIBRARY) < os.path.getmtime(SOURCE):
            build(force=True)
        _default = Oracle(LIBRARY)
    return _default


def counts(segs):
    return default().counts(segs)


def offsets(segs):
    return default().offsets(segs)


def voxel(seg, k):
    return default().voxel(seg, k)


def voxel_list(segs):
    return default().voxel_list(segs)


def voxel_list32(segs):
    return default().voxel_list32(segs)


def grid(segs, dims, base=None):
    return default().grid(segs, dims, base)


def counts_euclid(segs):
    return default().counts_euclid(segs)


def offsets_euclid(segs):
    return default().offsets_euclid(segs)


def voxel_list_euclid(segs):
    return default().voxel_list_euclid(segs)


def grid_euclid(segs, dims, base=None):
    return default().grid_euclid(segs, dims, base)
