"""Pins of the oracle's Euclidean-length variant (the paper's eq. (1):
N = int(|E - S|); samples S + k (E - S) / N, k = 0..N, each mapped to the
voxel containing it, round half up; consecutive duplicates removed).  CPU
only.  Each pin is checked against something other than the oracle itself:
exact rational arithmetic, math.isqrt, closed forms, invariants, and
deliberately broken builds of the oracle's source."""

import math
import subprocess
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle


def brute_force(seg):
    """The variant in exact rational arithmetic, written out directly."""
    s = [int(v) for v in seg[:3]]
    e = [int(v) for v in seg[3:]]
    d = [e[a] - s[a] for a in range(3)]
    n = math.isqrt(sum(x * x for x in d))
    out = []
    for k in range(n + 1):
        if n == 0:
            v = tuple(s)
        else:
            # the voxel containing the sample: nearest centre, ties upward
            v = tuple(math.floor(s[a] + Fraction(k * d[a], n) + Fraction(1, 2)) for a in range(3))
        if not out or out[-1] != v:
            out.append(v)
    return out


def all_pairs(lo, hi):
    pts = np.array([(x, y, z) for z in range(lo, hi) for y in range(lo, hi) for x in range(lo, hi)],
                   np.int32)
    a = np.repeat(pts, len(pts), axis=0)
    b = np.tile(pts, (len(pts), 1))
    return np.concatenate([a, b], 1)


def check_against_brute_force(o, segs):
    got = o.voxel_list_euclid(segs)
    counts = o.counts_euclid(segs)
    offs = o.offsets_euclid(segs)
    j = 0
    for i, seg in enumerate(segs):
        exp = brute_force(seg)
        if counts[i] != len(exp) or offs[i] != j:
            return "segment %s: count %d offset %d, expected %d at %d" % (seg.tolist(), counts[i], offs[i],
                                                                          len(exp), j)
        if [tuple(int(c) for c in v) for v in got[j:j + len(exp)]] != exp:
            return "segment %s: voxels differ" % (seg.tolist(),)
        j += len(exp)
    return None if offs[-1] == j else "total"


def check_invariants(o, segs):
    lists = o.voxel_list_euclid(segs).astype(np.int64)
    offs = o.offsets_euclid(segs)
    for i, seg in enumerate(segs.astype(np.int64)):
        v = lists[offs[i]:offs[i + 1]]
        d = seg[3:] - seg[:3]
        nc, ne = int(np.abs(d).max()), math.isqrt(int((d * d).sum()))
        if not (nc + 1 <= len(v) <= ne + 1):
            return "count bounds %s" % (seg.tolist(),)
        if tuple(v[0]) != tuple(seg[:3]) or tuple(v[-1]) != tuple(seg[3:]):
            return "end points %s" % (seg.tolist(),)
        steps = np.abs(np.diff(v, axis=0))
        if len(v) > 1 and (steps.max() > 1 or (steps.sum(1) == 0).any()):
            return "not 26-adjacent and distinct %s" % (seg.tolist(),)
    return None


def test_length_is_integer_square_root():
    o = oracle.default()
    rng = np.random.default_rng(41)
    segs = np.concatenate([rng.integers(-32768, 32768, (2000, 6)),
                           [[0, 0, 0, 3, 4, 0], [0, 0, 0, 1, 1, 1], [0, 0, 0, 2, 2, 1],
                            [5, 5, 5, 5, 5, 5], [-32768, -32768, -32768, 32767, 32767, 32767]]]).astype(np.int32)
    for seg in segs:
        d = seg[3:].astype(np.int64) - seg[:3]
        assert o.length_euclid(seg) == math.isqrt(int((d * d).sum()))


def test_worked_example():
    # (0,0,0) -> (3,4,0): |E - S| = 5, samples k*(0.6, 0.8, 0):
    # (0,0) (0.6,0.8) (1.2,1.6) (1.8,2.4) (2.4,3.2) (3,4) -> nearest centres
    # (0,0) (1,1) (1,2) (2,2) (2,3) (3,4), all distinct.
    seg = np.array([[0, 0, 0, 3, 4, 0]], np.int32)
    assert oracle.voxel_list_euclid(seg).tolist() == [[0, 0, 0], [1, 1, 0], [1, 2, 0], [2, 2, 0],
                                                       [2, 3, 0], [3, 4, 0]]
    # (0,0,0) -> (1,1,1): N = int(sqrt 3) = 1, samples at k = 0, 1 only.
    assert oracle.voxel_list_euclid(np.array([[0, 0, 0, 1, 1, 1]], np.int32)).tolist() == [[0, 0, 0], [1, 1, 1]]


def test_brute_force_small_cubes():
    o = oracle.default()
    assert check_against_brute_force(o, all_pairs(0, 3)) is None
    rng = np.random.default_rng(43)
    ex = all_pairs(-2, 3)
    assert check_against_brute_force(o, ex[rng.choice(len(ex), 4000, replace=False)]) is None


def test_brute_force_random_lengths():
    rng = np.random.default_rng(44)
    p0 = rng.integers(-300, 300, (300, 3))
    segs = np.concatenate([p0, p0 + rng.integers(-200, 201, (300, 3))], 1).astype(np.int32)
    assert check_against_brute_force(oracle.default(), segs) is None


def test_invariants_random():
    rng = np.random.default_rng(45)
    p0 = rng.integers(-1000, 1000, (500, 3))
    segs = np.concatenate([p0, p0 + rng.integers(-700, 701, (500, 3))], 1).astype(np.int32)
    assert check_invariants(oracle.default(), segs) is None


def test_axis_aligned_equals_chebyshev():
    """With one moving axis the Euclidean and Chebyshev lengths agree, and so
    do the voxels."""
    rng = np.random.default_rng(46)
    p0 = rng.integers(-500, 500, (200, 3))
    d = np.zeros((200, 3), np.int64)
    d[np.arange(200), rng.integers(0, 3, 200)] = rng.integers(-400, 401, 200)
    segs = np.concatenate([p0, p0 + d], 1).astype(np.int32)
    assert np.array_equal(oracle.voxel_list_euclid(segs), oracle.voxel_list(segs))
    assert np.array_equal(oracle.counts_euclid(segs), oracle.counts(segs))


def test_translation_covariance():
    rng = np.random.default_rng(47)
    p0 = rng.integers(-100, 100, (100, 3))
    segs = np.concatenate([p0, p0 + rng.integers(-90, 91, (100, 3))], 1).astype(np.int32)
    shift = np.array([7, -11, 3] * 2, np.int32)
    a = oracle.voxel_list_euclid(segs).astype(np.int64)
    b = oracle.voxel_list_euclid(segs + shift).astype(np.int64)
    assert np.array_equal(b - a, np.broadcast_to(shift[:3], a.shape))


def test_grid_is_the_set_of_list_voxels():
    rng = np.random.default_rng(48)
    dims = (37, 21, 9)
    p = [np.stack([rng.integers(0, dv, 400) for dv in dims], 1) for _ in range(2)]
    segs = np.concatenate(p, 1).astype(np.int32)
    grid = oracle.grid_euclid(segs, dims)
    bits = np.zeros(dims[::-1], bool)
    for x, y, z in oracle.voxel_list_euclid(segs).astype(np.int64):
        bits[z, y, x] = True
    exp = np.packbits(bits.reshape(-1), bitorder="little")
    exp = np.concatenate([exp, np.zeros((-len(exp)) % 4, np.uint8)]).view(np.uint32)
    assert np.array_equal(grid, exp)
    with pytest.raises(ValueError):
        oracle.grid_euclid(np.array([[0, 0, 0, 37, 0, 0]], np.int32), dims)


EUCLID_MUTANTS = {
    "no duplicate removal": ("            continue;\n", "            (void)0;\n"),
    "ceiling square root": ("    return lo;\n}", "    return hi;\n}"),
    "round half down": ("out[a] = p0 + floor_div(2 * k * d + N, 2 * N);\n    }\n}\n\n/* Visits",
                        "out[a] = p0 + floor_div(2 * k * d + N - 1, 2 * N);\n    }\n}\n\n/* Visits"),
    "Chebyshev length": ("        ss += (uint64_t)(d * d);", "        ss = (uint64_t)(d < 0 ? -d : d) * (d < 0 ? -d : d) > ss ? (uint64_t)(d * d) : ss;"),
    "duplicates compared on x only": ("if (k > 0 && v[0] == prev[0] && v[1] == prev[1] && v[2] == prev[2])",
                                      "if (k > 0 && v[0] == prev[0])"),
}


@pytest.mark.parametrize("name", sorted(EUCLID_MUTANTS))
def test_euclid_mutant_is_caught(name, tmp_path):
    old, new = EUCLID_MUTANTS[name]
    src = open(oracle.SOURCE).read()
    assert src.count(old) == 1, "mutation anchor not unique: %r" % old
    csrc = tmp_path / "mutant.c"
    csrc.write_text(src.replace(old, new))
    lib = str(tmp_path / "mutant.so")
    oracle.compile_source(str(csrc), lib)
    o = oracle.Oracle(lib)
    rng = np.random.default_rng(49)
    ex = all_pairs(-2, 3)
    ex = ex[rng.choice(len(ex), 2000, replace=False)]
    p0 = rng.integers(-100, 100, (100, 3))
    rnd = np.concatenate([p0, p0 + rng.integers(-90, 91, (100, 3))], 1).astype(np.int32)
    fails = []
    for check in (lambda: check_against_brute_force(o, ex), lambda: check_invariants(o, rnd),
                  lambda: check_against_brute_force(o, rnd[:40])):
        try:
            r = check()
        except Exception as e:  # a crash or a rejected case is a detection too
            r = "raised %r" % (e,)
        if r is not None:
            fails.append(r)
    assert fails, "mutant %r passed every pin" % name


def test_brute_force_beyond_32767():
    """Euclidean lengths above 32767 (where the GPU kernels divide in 64 bits):
    the whole list by exact rational arithmetic, for the int16 diagonal
    (N = 113511) and two long skew segments."""
    segs = np.array([[-32768, -32768, -32768, 32767, 32767, 32767],
                     [32767, -30000, 5, -32768, 29999, -7],
                     [-100, 20000, -32768, 150, -20000, 32767]], np.int32)
    assert all(oracle.default().length_euclid(s) > 32767 for s in segs)
    assert check_against_brute_force(oracle.default(), segs) is None
