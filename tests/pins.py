"""Checks that pin the CPU oracle to definitions other than its own formula.

The oracle computes voxel k of segment (P0, P1) as P0 + floor((2 k d + N) / 2N)
per axis (eq. (3) with round-half-up).  The checks below state the same result
in other ways, none of which evaluates that expression:

* nearest centre, by exhaustive search: in the slice of the dominant axis
  that holds G_k = P0 + k d / N, the voxel is the candidate centre c with
  |c - x| < 1/2, or |c - x| == 1/2 and c > x, searched over every integer of
  the segment's bounding box (exact integer comparisons on 2N (c - x));
* the same with Python `fractions.Fraction` and min |c - x|;
* brute-force bit-volume: every voxel of a small volume tested for
  membership, packed with numpy's little-endian bit order;
* invariants the method guarantees exactly (count N+1, both end points,
  26-adjacency, one voxel per dominant slice, per-axis monotonicity, thinness,
  reversal, axis permutation, integer translation);
* closed forms (axis-aligned lines, pure diagonals);
* fp64 evaluation of floor(P0 + k d / N + 1/2), exact for N < 2^20.

Each `check_*` returns None on success or a string naming the failure, so the
same checks can be run against deliberately broken builds of the oracle.
"""

from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np


def _len(seg):
    return max(abs(int(seg[3 + a]) - int(seg[a])) for a in range(3))


# ----------------------------------------------------------- independent defs

def nearest_centre_list(segs: np.ndarray) -> np.ndarray:
    """Voxel lists by exhaustive candidate search (vectorised, exact ints).

    For segment i, k in 0..N and axis a, keep the integers c in the bounding
    box [min(P0_a,P1_a), max(P0_a,P1_a)] with  -N < 2N(c - P0_a) - 2 k d_a <= N,
    i.e. |c - x| < 1/2 or c - x == +1/2.  Exactly one must qualify."""
    segs = np.asarray(segs, dtype=np.int64)
    p0, p1 = segs[:, :3], segs[:, 3:]
    d = p1 - p0
    N = np.abs(d).max(axis=1)
    out = []
    lo = np.minimum(p0, p1)
    hi = np.maximum(p0, p1)
    span = int((hi - lo).max()) + 1 if len(segs) else 1
    cand = np.arange(span)                                   # offsets from lo
    kmax = int(N.max()) if len(segs) else 0
    ks = np.arange(kmax + 1)
    # [n, K, 3, C]
    c = lo[:, None, :, None] + cand[None, None, None, :]
    Nn = np.maximum(N, 1)[:, None, None, None]
    t = 2 * Nn * (c - p0[:, None, :, None]) - 2 * ks[None, :, None, None] * d[:, None, :, None]
    ok = (t > -Nn) & (t <= Nn) & (c <= hi[:, None, :, None])
    zero = (N == 0)
    if zero.any():
        ok[zero] = (c[zero] == p0[zero][:, None, :, None])
    nok = ok.sum(axis=3)
    valid_k = ks[None, :] <= N[:, None]
    if not np.all(nok[valid_k] == 1):
        raise AssertionError("nearest-centre search found no unique voxel")
    idx = np.argmax(ok, axis=3)
    vox = lo[:, None, :] + idx                                  # [n, K, 3]
    return vox[valid_k].astype(np.int16)


def fraction_list(seg) -> list:
    """One segment by Fraction arithmetic: argmin |c - x|, ties to larger c."""
    p0 = [int(v) for v in seg[:3]]
    p1 = [int(v) for v in seg[3:]]
    N = _len(seg)
    res = []
    for k in range(N + 1):
        v = []
        for a in range(3):
            x = Fraction(p0[a]) if N == 0 else Fraction(p0[a]) + Fraction(k * (p1[a] - p0[a]), N)
            f = x.numerator // x.denominator
            best = None
            for c in (f - 1, f, f + 1, f + 2):
                dist = abs(Fraction(c) - x)
                if best is None or dist < best[0] or (dist == best[0] and c > best[1]):
                    best = (dist, c)
            v.append(best[1])
        res.append(tuple(v))
    return res


def brute_grid(segs: np.ndarray, dims) -> np.ndarray:
    """bool [dz, dy, dx]: every voxel of the volume tested for membership in
    some segment (exists k with all three axes passing the nearest-centre
    test)."""
    dx, dy, dz = dims
    zz, yy, xx = np.meshgrid(np.arange(dz), np.arange(dy), np.arange(dx), indexing="ij")
    V = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1).astype(np.int64)  # [M,3]
    occ = np.zeros(V.shape[0], dtype=bool)
    for seg in np.asarray(segs, dtype=np.int64):
        p0, d = seg[:3], seg[3:] - seg[:3]
        N = int(np.abs(d).max())
        if N == 0:
            occ |= np.all(V == p0, axis=1)
            continue
        k = np.arange(N + 1)
        t = 2 * N * (V[:, None, :] - p0[None, None, :]) - 2 * k[None, :, None] * d[None, None, :]
        occ |= np.any(np.all((t > -N) & (t <= N), axis=2), axis=1)
    return occ.reshape(dz, dy, dx)


def unpack_grid(words: np.ndarray, dims) -> np.ndarray:
    """bool [dz, dy, dx] from packed words: bit b = (z*dy + y)*dx + x, word
    b // 32, bit b % 32, least significant bit first."""
    dx, dy, dz = dims
    bits = np.unpackbits(np.ascontiguousarray(words, dtype="<u4").view(np.uint8),
                         bitorder="little")
    return bits[: dx * dy * dz].reshape(dz, dy, dx).astype(bool)


# ---------------------------------------------------------------- segment sets

def exhaustive(lo: int, hi: int) -> np.ndarray:
    """Every ordered endpoint pair with coordinates in [lo, hi]."""
    r = np.arange(lo, hi + 1)
    pts = np.array(list(itertools.product(r, r, r)), dtype=np.int32)
    i, j = np.meshgrid(np.arange(len(pts)), np.arange(len(pts)), indexing="ij")
    return np.concatenate([pts[i.ravel()], pts[j.ravel()]], axis=1)


def random_segments(n: int, seed: int, lo: int = -300, hi: int = 300) -> np.ndarray:
    rng = np.random.default_rng(seed)
    a = rng.integers(lo, hi, size=(n, 3))
    # Mix of lengths: short, long, axis-aligned, diagonal-ish.
    L = np.exp(rng.uniform(0, np.log(hi - lo), size=n)).astype(np.int64)
    d = rng.integers(-1, 2, size=(n, 3)) * L[:, None] + rng.integers(-3, 4, size=(n, 3))
    return np.concatenate([a, a + d], axis=1).astype(np.int32)


# ----------------------------------------------------------------------- checks

def check_nearest_centre(o, segs) -> str | None:
    got = o.voxel_list(segs)
    exp = nearest_centre_list(segs)
    if got.shape != exp.shape:
        return "nearest-centre: shape %s vs %s" % (got.shape, exp.shape)
    if not np.array_equal(got, exp):
        bad = np.argwhere(np.any(got != exp, axis=1))[0, 0]
        return "nearest-centre: first mismatch at voxel %d: %s vs %s" % (
            bad, got[bad].tolist(), exp[bad].tolist())
    return None


def check_fraction(o, segs) -> str | None:
    for seg in segs:
        got = [tuple(int(c) for c in v) for v in o.voxel_list(seg[None, :])]
        exp = fraction_list(seg)
        if got != exp:
            return "fraction: segment %s gives %s, expected %s" % (seg.tolist(), got, exp)
    return None


def check_invariants(o, segs) -> str | None:
    segs = np.asarray(segs, dtype=np.int32)
    offs = o.offsets(segs)
    cnt = o.counts(segs)
    lst = o.voxel_list(segs).astype(np.int64)
    s64 = segs.astype(np.int64)
    N = np.abs(s64[:, 3:] - s64[:, :3]).max(axis=1)
    if not np.array_equal(cnt, N + 1):
        return "invariant: counts != N+1"
    if offs[0] != 0 or not np.array_equal(np.diff(offs), cnt) or lst.shape[0] != offs[-1]:
        return "invariant: offsets are not the prefix sum of counts"
    for i in range(len(segs)):
        v = lst[offs[i]:offs[i + 1]]
        if not np.array_equal(v[0], s64[i, :3]) or not np.array_equal(v[-1], s64[i, 3:]):
            return "invariant: end points of segment %d" % i
        if len(v) > 1:
            step = np.diff(v, axis=0)
            if np.abs(step).max() > 1:
                return "invariant: not 26-adjacent in segment %d" % i
            m = int(np.argmax(np.abs(s64[i, 3:] - s64[i, :3])))
            sgn = np.sign(s64[i, 3 + m] - s64[i, m])
            if not np.all(step[:, m] == sgn):
                return "invariant: dominant axis does not step by 1 in segment %d" % i
            for a in range(3):
                sa = np.sign(s64[i, 3 + a] - s64[i, a])
                if np.any(step[:, a] * sa < 0):
                    return "invariant: axis %d not monotone in segment %d" % (a, i)
            # Thinness: an interior voxel has exactly two 26-neighbours in its
            # own list (the previous and the next one).
            if len(v) > 2:
                cheb = np.abs(v[:, None, :] - v[None, :, :]).max(axis=2)
                nb = ((cheb == 1)).sum(axis=1)
                if not (np.all(nb[1:-1] == 2) and nb[0] == 1 and nb[-1] == 1):
                    return "invariant: list of segment %d is not thin" % i
    return None


def check_distance(o, segs) -> str | None:
    """|v_a - x_a| <= 1/2 with equality only when v_a > x_a (exact ints)."""
    segs = np.asarray(segs, dtype=np.int64)
    offs = o.offsets(segs)
    lst = o.voxel_list(segs).astype(np.int64)
    for i, s in enumerate(segs):
        N = int(np.abs(s[3:] - s[:3]).max())
        if N == 0:
            continue
        k = np.arange(N + 1)[:, None]
        v = lst[offs[i]:offs[i + 1]]
        t = 2 * N * (v - s[None, :3]) - 2 * k * (s[None, 3:] - s[None, :3])
        if np.any(t <= -N) or np.any(t > N):
            return "distance: segment %d leaves the half-voxel band" % i
    return None


def check_symmetries(o, segs) -> str | None:
    segs = np.asarray(segs, dtype=np.int32)
    offs = o.offsets(segs)
    lst = o.voxel_list(segs)
    rev = np.concatenate([segs[:, 3:], segs[:, :3]], axis=1)
    lst_r = o.voxel_list(rev)
    for i in range(len(segs)):
        if not np.array_equal(lst_r[offs[i]:offs[i + 1]], lst[offs[i]:offs[i + 1]][::-1]):
            return "reversal: segment %d" % i
    for perm in ((1, 2, 0), (2, 0, 1), (0, 2, 1), (1, 0, 2)):
        p = list(perm) + [3 + q for q in perm]
        if not np.array_equal(o.voxel_list(segs[:, p]), lst[:, list(perm)]):
            return "permutation %s" % (perm,)
    shift = np.array([7, -5, 3], dtype=np.int32)
    sh = segs + np.concatenate([shift, shift])
    if not np.array_equal(o.voxel_list(sh), lst + shift.astype(np.int16)):
        return "translation"
    return None


def check_mirror_ties(o, segs) -> str | None:
    """x -> -x changes a voxel only at ties 2 k d_a == N (mod 2N)."""
    segs = np.asarray(segs, dtype=np.int64)
    offs = o.offsets(segs)
    lst = o.voxel_list(segs).astype(np.int64)
    mir = segs.copy()
    mir[:, 0] *= -1
    mir[:, 3] *= -1
    lst_m = o.voxel_list(mir).astype(np.int64)
    for i, s in enumerate(segs):
        N = int(np.abs(s[3:] - s[:3]).max())
        v = lst[offs[i]:offs[i + 1], 0]
        w = -lst_m[offs[i]:offs[i + 1], 0]
        k = np.arange(N + 1)
        tie = ((2 * k * (s[3] - s[0]) - N) % (2 * N) == 0) if N else np.zeros(1, bool)
        if np.any((v != w) & ~tie):
            return "mirror: segment %d differs away from a tie" % i
        if np.any((v == w) & tie):
            return "mirror: segment %d agrees at a tie" % i
    return None


def check_closed_forms(o) -> str | None:
    cases = []
    for a in range(3):
        for sgn in (1, -1):
            for L in (0, 1, 2, 5, 31, 64, 300):
                p0 = np.array([11, -4, 9])
                e = np.zeros(3, dtype=np.int64)
                e[a] = sgn
                cases.append((p0, e, L))
    for sx, sy, sz in itertools.product((1, -1), repeat=3):
        for L in (1, 3, 17):
            cases.append((np.array([2, 3, -7]), np.array([sx, sy, sz]), L))
    for p0, e, L in cases:
        seg = np.concatenate([p0, p0 + L * e]).astype(np.int32)[None, :]
        exp = (p0[None, :] + np.arange(L + 1)[:, None] * e[None, :]).astype(np.int16)
        got = o.voxel_list(seg)
        if not np.array_equal(got, exp):
            return "closed form: %s" % seg.tolist()
    # Two-voxel-wide ties: (0,0,0)->(2,1,0): x = 0,1,2; y = 0, 1/2 -> 1, 1.
    got = o.voxel_list(np.array([[0, 0, 0, 2, 1, 0]], dtype=np.int32))
    if got.tolist() != [[0, 0, 0], [1, 1, 0], [2, 1, 0]]:
        return "closed form: tie rounds half up"
    got = o.voxel_list(np.array([[0, 0, 0, 2, -1, 0]], dtype=np.int32))
    if got.tolist() != [[0, 0, 0], [1, 0, 0], [2, -1, 0]]:
        return "closed form: negative tie rounds half up (toward +inf)"
    return None


def nearest_centre_at(seg, k: int) -> tuple:
    """Voxel of sample k by exact rational arithmetic: the centre c nearest to
    x = P0 + k d / N on each axis, ties to the larger c."""
    p0 = [int(v) for v in seg[:3]]
    p1 = [int(v) for v in seg[3:]]
    N = _len(seg)
    v = []
    for a in range(3):
        x = Fraction(p0[a]) if N == 0 else Fraction(p0[a]) + Fraction(k * (p1[a] - p0[a]), N)
        f = x.numerator // x.denominator
        best = None
        for c in (f - 1, f, f + 1, f + 2):
            dist = abs(Fraction(c) - x)
            if best is None or dist < best[0] or (dist == best[0] and c > best[1]):
                best = (dist, c)
        v.append(best[1])
    return tuple(v)


def check_list32(o) -> str | None:
    """int32 lists beyond the int16 range: closed forms of long axis and
    diagonal segments far from the origin, a half-slope closed form, and
    exact nearest-centre voxels at sampled k of random long segments with
    end points near +-2^30."""
    for p0, e, L in (((10 ** 9, -5, 7), (1, 0, 0), 10 ** 6), ((3, -(10 ** 9), 0), (0, -1, 0), 123457),
                     ((-(2 ** 30), 2 ** 30, 40000), (1, -1, 1), 70001), ((0, 0, 2 ** 31 - 1), (0, 0, -1), 99999)):
        p0, e = np.array(p0, np.int64), np.array(e, np.int64)
        seg = np.concatenate([p0, p0 + L * e]).astype(np.int32)[None, :]
        exp = p0[None, :] + np.arange(L + 1)[:, None] * e[None, :]
        if not np.array_equal(o.voxel_list32(seg).astype(np.int64), exp):
            return "list32 closed form %s" % seg.tolist()
    # (0,0,0) -> (2m, m, 0): y_k = round_half_up(k / 2) = (k + 1) // 2.
    m = 60000
    got = o.voxel_list32(np.array([[0, 0, 0, 2 * m, m, 0]], np.int32)).astype(np.int64)
    k = np.arange(2 * m + 1)
    if not np.array_equal(got, np.stack([k, (k + 1) // 2, 0 * k], 1)):
        return "list32 half-slope ties"
    rng = np.random.default_rng(7)
    p0 = rng.integers(-(2 ** 30), 2 ** 30, (6, 3))
    d = rng.integers(-200000, 200001, (6, 3))
    segs = np.concatenate([p0, p0 + d], 1).astype(np.int32)
    got = o.voxel_list32(segs).astype(np.int64)
    j = 0
    for seg in segs:
        N = _len(seg)
        for kk in sorted({0, 1, N // 3, N // 2, N - 1, N} | set(rng.integers(0, N + 1, 40).tolist())):
            if kk < 0 or kk > N:
                continue
            if tuple(got[j + kk]) != nearest_centre_at(seg, kk):
                return "list32 sample %d of %s" % (kk, seg.tolist())
        j += N + 1
    if j != len(got):
        return "list32 total"
    return None


def check_fp64(o, segs) -> str | None:
    """floor(P0 + k d / N + 1/2) in fp64 (exact for N < 2^20)."""
    segs = np.asarray(segs, dtype=np.int64)
    lst = o.voxel_list(segs).astype(np.int64)
    offs = o.offsets(segs)
    for i, s in enumerate(segs):
        N = int(np.abs(s[3:] - s[:3]).max())
        k = np.arange(N + 1, dtype=np.float64)[:, None]
        if N == 0:
            exp = s[None, :3]
        else:
            exp = np.floor(s[None, :3] + k * (s[None, 3:] - s[None, :3]) / N + 0.5).astype(np.int64)
        if not np.array_equal(lst[offs[i]:offs[i + 1]], exp):
            return "fp64: segment %d" % i
    return None


def check_grid(o, segs, dims) -> str | None:
    """Bit-volume against brute-force membership and the list's distinct
    voxels; OR-into-existing semantics."""
    dims = tuple(int(v) for v in dims)
    g = o.grid(segs, dims)
    occ = unpack_grid(g, dims)
    exp = brute_grid(segs, dims)
    if not np.array_equal(occ, exp):
        return "grid: differs from brute-force membership"
    nbits = dims[0] * dims[1] * dims[2]
    tail = np.unpackbits(g.view(np.uint8), bitorder="little")[nbits:]
    if tail.any():
        return "grid: bits set past the volume"
    lst = o.voxel_list(segs)
    distinct = np.unique(lst, axis=0).shape[0] if lst.shape[0] else 0
    if int(occ.sum()) != distinct:
        return "grid: popcount != distinct voxels"
    half = len(segs) // 2
    g1 = o.grid(segs[:half], dims)
    g2 = o.grid(segs[half:], dims, base=g1)
    if not np.array_equal(g2, g):
        return "grid: OR into an existing volume"
    return None
