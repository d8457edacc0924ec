"""Seeded synthetic segment sets for the five workloads.

The paper measures on synthetic segment sets only: one segment of a given
length, 1024 segments of one fixed length, and 1024 segments of arbitrary
lengths (Section 5, experiments 1-3).  The sets below keep that character at
MI355X scale: a small uniform set with a 256^3 volume, 1 M fixed-length
segments, 4 M arbitrary-length segments in a 2048^3 volume, 256 scenes of mixed
volume size, and icosphere wireframes for the request stream.  No dataset is
involved.

This module is shared by the tests, the benchmark and the serving driver.  It
only draws endpoints: it holds none of the voxelization arithmetic, and it
imports nothing from the HIP binding or from the CPU oracle.

Every generator returns int32 arrays of shape [n, 6] laid out x0,y0,z0,x1,y1,z1
(start point S, end point E).  "Direction uniform on the sphere" is a 3D
standard normal u scaled by 1/max|u_a|, so its dominant component is exactly
+-1 and a length L along it gives a Chebyshev length of exactly L.
"""

from __future__ import annotations

import math

import numpy as np

SEED_SMALL = 1001
SEED_FIXED = 1002
SEED_ARBITRARY = 1003
SEED_SCENES = 1004
SEED_REQUEST0 = 1005

SEED_PAPER = 1006

N_SMALL = 1000
N_FIXED = 1 << 20
N_ARBITRARY = 1 << 22
N_SCENES = 256


def _chebyshev_directions(rng: np.random.Generator, n: int) -> np.ndarray:
    """n directions uniform on the sphere, scaled so max |v_a| == 1 exactly."""
    u = rng.standard_normal((n, 3))
    m = np.max(np.abs(u), axis=1, keepdims=True)
    m[m == 0] = 1.0
    v = u / m
    # Division by the max can leave the dominant entry at 1 - ulp; pin it.
    dom = np.argmax(np.abs(u), axis=1)
    rows = np.arange(n)
    v[rows, dom] = np.sign(u[rows, dom])
    return v


def small_uniform(n: int = N_SMALL, seed: int = SEED_SMALL, volume: int = 256):
    """Both endpoints uniform in [0, volume)^3; lengths 0..volume-1 voxels."""
    rng = np.random.default_rng(seed)
    p0 = rng.integers(0, volume, size=(n, 3))
    p1 = rng.integers(0, volume, size=(n, 3))
    segs = np.concatenate([p0, p1], axis=1).astype(np.int32)
    return {"segs": segs, "dims": (volume, volume, volume)}


def single_diagonal(volume: int = 256):
    """One segment along the main diagonal of the volume: volume voxels."""
    segs = np.array([[0, 0, 0, volume - 1, volume - 1, volume - 1]], dtype=np.int32)
    return {"segs": segs, "dims": (volume, volume, volume)}


def fixed_length(n: int = N_FIXED, seed: int = SEED_FIXED, length: int = 64,
                 start_range: int = 960):
    """Start uniform in [0, start_range)^3, direction uniform on the sphere,
    end = start + rint(length * v): every segment has Chebyshev length
    `length` (length + 1 voxels).  Coordinates span [-length, start_range +
    length) and are kept as drawn, negative values included."""
    rng = np.random.default_rng(seed)
    start = rng.integers(0, start_range, size=(n, 3))
    v = _chebyshev_directions(rng, n)
    d = np.rint(length * v).astype(np.int64)
    segs = np.concatenate([start, start + d], axis=1).astype(np.int32)
    return {"segs": segs}


def arbitrary_length(n: int = N_ARBITRARY, seed: int = SEED_ARBITRARY,
                     volume: int = 2048):
    """Start uniform in [0, volume)^3, direction uniform on the sphere, length
    L log-uniform in [1, volume], clipped along the direction so the end point
    stays inside the volume:
        L' = floor(min(L, min_a floor(bound_a / |v_a|))),
        bound_a = volume-1-s_a if v_a > 0 else s_a,
    d = rint(L' * v), so the Chebyshev length is exactly L' (0 allowed)."""
    rng = np.random.default_rng(seed)
    start = rng.integers(0, volume, size=(n, 3))
    L = np.exp(rng.uniform(0.0, math.log(volume), size=n))
    v = _chebyshev_directions(rng, n)
    bound = np.where(v > 0, (volume - 1) - start, start).astype(np.float64)
    av = np.abs(v)
    with np.errstate(divide="ignore"):
        lim = np.where(av > 0, np.floor(bound / np.where(av > 0, av, 1.0)), np.inf)
    Lc = np.floor(np.minimum(L, lim.min(axis=1)))
    d = np.rint(Lc[:, None] * v).astype(np.int64)
    segs = np.concatenate([start, start + d], axis=1).astype(np.int32)
    return {"segs": segs, "dims": (volume, volume, volume)}


def paper_segments(lengths, seed: int = SEED_PAPER, start_bound: int = 1 << 29):
    """The paper's experiment shapes (Section 5) with int32 coordinates: one
    segment per entry of `lengths` (voxels per segment, >= 1), start uniform
    in [-start_bound, start_bound)^3, direction uniform on the sphere,
    end = start + rint((length - 1) * v), so segment i has exactly lengths[i]
    voxels under the Chebyshev length.  Every axis difference stays below
    2^30 for lengths up to 2^30."""
    L = np.asarray(lengths, dtype=np.int64).reshape(-1)
    rng = np.random.default_rng(seed)
    start = rng.integers(-start_bound, start_bound, size=(L.size, 3))
    v = _chebyshev_directions(rng, L.size)
    d = np.rint((L[:, None] - 1) * v).astype(np.int64)
    segs = np.concatenate([start, start + d], axis=1).astype(np.int32)
    return {"segs": segs}


def paper_arbitrary_lengths(n: int = 1024, total: int = 10 ** 9, seed: int = SEED_PAPER + 1):
    """Experiment 3's lengths: n segments of arbitrary length totalling
    `total` voxels: lengths uniform in [1, 2 total / n], rescaled to the
    total, the rounding remainder on the last segment."""
    rng = np.random.default_rng(seed)
    w = rng.uniform(1.0, 2.0 * total / n, size=n)
    L = np.maximum(1, np.floor(w * (total / w.sum()))).astype(np.int64)
    L[-1] += total - int(L.sum())
    return L


def scenes(n_scenes: int = N_SCENES, seed: int = SEED_SCENES,
           volumes=(64, 128, 256, 512), n_lo: float = 1e3, n_hi: float = 2e5):
    """Independent scenes: volume V_s drawn from `volumes` (cubic), segment
    count floor(exp(uniform(ln n_lo, ln n_hi))), both endpoints uniform in
    [0, V_s)^3.  Returns a list of {"segs", "dims"}."""
    rng = np.random.default_rng(seed)
    vol = rng.choice(np.asarray(volumes), size=n_scenes)
    counts = np.floor(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi),
                                         size=n_scenes))).astype(np.int64)
    out = []
    for s in range(n_scenes):
        V = int(vol[s])
        segs = rng.integers(0, V, size=(int(counts[s]), 6)).astype(np.int32)
        out.append({"segs": segs, "dims": (V, V, V)})
    return out


# ---------------------------------------------------------------- wireframes

_ICO_T = (1.0 + 5.0 ** 0.5) / 2.0
_ICO_VERTS = np.array([
    (-1, _ICO_T, 0), (1, _ICO_T, 0), (-1, -_ICO_T, 0), (1, -_ICO_T, 0),
    (0, -1, _ICO_T), (0, 1, _ICO_T), (0, -1, -_ICO_T), (0, 1, -_ICO_T),
    (_ICO_T, 0, -1), (_ICO_T, 0, 1), (-_ICO_T, 0, -1), (-_ICO_T, 0, 1),
], dtype=np.float64)
_ICO_FACES = np.array([
    (0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
    (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
    (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
    (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1),
], dtype=np.int64)


def geodesic_icosphere(m: int):
    """Class-I geodesic subdivision of frequency m of the unit icosahedron.

    Returns (unit vertices float64 [V,3], undirected edges int64 [E,2] with
    a < b, face count F).  V = 10 m^2 + 2, E = 30 m^2, F = 20 m^2.
    Vertices shared by neighbouring faces are merged on their exact integer
    barycentric key (icosahedron vertex ids with weights summing to m)."""
    if m < 1:
        raise ValueError("frequency must be >= 1")
    ii, jj = np.meshgrid(np.arange(m + 1), np.arange(m + 1), indexing="ij")
    keep = (ii + jj) <= m
    ii, jj = ii[keep], jj[keep]                     # local grid points of a face
    P = ii.size
    local = -np.ones((m + 1, m + 1), dtype=np.int64)
    local[ii, jj] = np.arange(P)
    F0 = _ICO_FACES.shape[0]
    # Weights on (A, B, C) of each face for every local point.
    w = np.stack([m - ii - jj, ii, jj], axis=1)      # [P,3]
    vid = np.broadcast_to(_ICO_FACES[:, None, :], (F0, P, 3))
    ww = np.broadcast_to(w[None, :, :], (F0, P, 3))
    vid = np.where(ww > 0, vid, 12)                  # 12 sorts after real ids
    order = np.argsort(vid, axis=2, kind="stable")
    vid_s = np.take_along_axis(vid, order, axis=2)
    ww_s = np.take_along_axis(ww, order, axis=2)
    # One int64 per key, packed so that integer order is the lexicographic
    # order of (ids, weights): ids < 16 take 4 bits, weights <= m < 2^16 take
    # 16 bits each (52 bits in all).
    keys = np.concatenate([vid_s, ww_s], axis=2).reshape(F0 * P, 6).astype(np.int64)
    packed = np.zeros(F0 * P, dtype=np.int64)
    for c in range(3):
        packed = (packed << 4) | keys[:, c]
    for c in range(3):
        packed = (packed << 16) | keys[:, 3 + c]
    uniq_p, first, inv = np.unique(packed, return_index=True, return_inverse=True)
    uniq = keys[first]
    inv = inv.reshape(F0, P)
    # Positions from the unique keys.
    pos = np.zeros((uniq.shape[0], 3))
    for c in range(3):
        vv = uniq[:, c]
        wc = uniq[:, 3 + c].astype(np.float64)
        valid = vv < 12
        pos[valid] += wc[valid, None] * _ICO_VERTS[vv[valid]]
    pos /= np.linalg.norm(pos, axis=1, keepdims=True)
    # Triangles of the subdivided face: up (i,j),(i+1,j),(i,j+1) and
    # down (i+1,j),(i+1,j+1),(i,j+1).
    tris = []
    ui, uj = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    up = (ui + uj) <= m - 1
    a, b = ui[up], uj[up]
    tris.append(np.stack([local[a, b], local[a + 1, b], local[a, b + 1]], axis=1))
    dn = (ui + uj) <= m - 2
    a, b = ui[dn], uj[dn]
    tris.append(np.stack([local[a + 1, b], local[a + 1, b + 1], local[a, b + 1]], axis=1))
    tri_local = np.concatenate(tris, axis=0)         # [m^2, 3]
    tri = inv[:, tri_local].reshape(-1, 3)           # [20 m^2, 3]
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]], axis=0)
    e = np.sort(e, axis=1).astype(np.int64)
    # Unique rows (a, b), a < b, in row order, as unique int64 (a << 32 | b).
    pe = np.unique((e[:, 0] << 32) | e[:, 1])
    edges = np.stack([pe >> 32, pe & 0xFFFFFFFF], axis=1)
    return pos, edges, tri.shape[0]


def wireframe_request(r: int, seed0: int = SEED_REQUEST0, volume: int = 512,
                      e_lo: float = 1e4, e_hi: float = 1e6):
    """Request r of the serving stream: the edge set of a jittered geodesic
    icosphere quantized into [0, volume)^3.

    Target edge count E* log-uniform in [e_lo, e_hi], frequency
    m = round(sqrt(E*/30)); radius uniform in [64, 240]; centre volume/2 - 0.5;
    per-vertex radial jitter factor 1 + 0.05 N(0,1); coordinates
    clip(floor(p + 0.5), 0, volume-1).  Each undirected edge (a < b) becomes
    one segment from vertex a to vertex b."""
    rng = np.random.default_rng(seed0 + r)
    e_star = math.exp(rng.uniform(math.log(e_lo), math.log(e_hi)))
    m = max(1, int(round(math.sqrt(e_star / 30.0))))
    radius = rng.uniform(64.0, 240.0)
    pos, edges, n_faces = geodesic_icosphere(m)
    jitter = 1.0 + 0.05 * rng.standard_normal(pos.shape[0])
    centre = volume / 2.0 - 0.5
    p = centre + radius * jitter[:, None] * pos
    q = np.clip(np.floor(p + 0.5), 0, volume - 1).astype(np.int32)
    segs = np.concatenate([q[edges[:, 0]], q[edges[:, 1]]], axis=1).astype(np.int32)
    return {"segs": segs, "dims": (volume, volume, volume), "frequency": m,
            "n_vertices": pos.shape[0], "n_faces": n_faces}
