"""The CPU oracle against definitions other than its own formula (CPU only)."""

import numpy as np
import pytest

from oracle import oracle
from paper_2009_09500_amd import workloads
from tests import pins


@pytest.fixture(scope="module")
def o():
    oracle.build(force=False)
    return oracle.default()


def test_exhaustive_0_4(o):
    """Every endpoint pair in [0,4)^3 (4096 segments) by exhaustive search."""
    segs = pins.exhaustive(0, 3)
    assert pins.check_nearest_centre(o, segs) is None


def test_exhaustive_negative(o):
    """Every endpoint pair in [-3,3]^3 (117 649 segments), negatives included."""
    segs = pins.exhaustive(-3, 3)
    assert pins.check_nearest_centre(o, segs) is None


def test_fraction_sample(o):
    segs = pins.exhaustive(-2, 2)
    rng = np.random.default_rng(5)
    pick = segs[rng.choice(len(segs), 600, replace=False)]
    assert pins.check_fraction(o, pick) is None
    assert pins.check_fraction(o, pins.random_segments(60, 7, -40, 40)) is None


def test_invariants_random(o):
    assert pins.check_invariants(o, pins.random_segments(400, 11)) is None


def test_invariants_workloads(o):
    segs = np.concatenate([
        workloads.small_uniform(n=200)["segs"],
        workloads.fixed_length(n=200)["segs"],
        workloads.arbitrary_length(n=300)["segs"],
    ])
    assert pins.check_invariants(o, segs) is None
    assert pins.check_distance(o, segs) is None


def test_distance_band(o):
    assert pins.check_distance(o, pins.random_segments(400, 13)) is None


def test_symmetries(o):
    assert pins.check_symmetries(o, pins.random_segments(300, 17)) is None
    assert pins.check_symmetries(o, pins.exhaustive(-1, 1)) is None


def test_mirror_differs_only_at_ties(o):
    assert pins.check_mirror_ties(o, pins.random_segments(300, 19)) is None


def test_closed_forms(o):
    assert pins.check_closed_forms(o) is None


def test_fp64_cross_check(o):
    segs = pins.random_segments(200, 23, -8000, 8000)
    assert pins.check_fp64(o, segs) is None


@pytest.mark.parametrize("dims", [(32, 8, 8), (37, 5, 3), (1, 1, 1), (64, 3, 2)])
def test_grid_brute_force(o, dims):
    rng = np.random.default_rng(sum(dims))
    dx, dy, dz = dims
    n = 40
    p0 = np.stack([rng.integers(0, dx, n), rng.integers(0, dy, n), rng.integers(0, dz, n)], 1)
    p1 = np.stack([rng.integers(0, dx, n), rng.integers(0, dy, n), rng.integers(0, dz, n)], 1)
    segs = np.concatenate([p0, p1], 1).astype(np.int32)
    assert pins.check_grid(o, segs, dims) is None


def test_grid_rejects_out_of_volume(o):
    with pytest.raises(ValueError):
        o.grid(np.array([[0, 0, 0, 8, 0, 0]], dtype=np.int32), (8, 8, 8))
    with pytest.raises(ValueError):
        o.grid(np.array([[0, -1, 0, 3, 0, 0]], dtype=np.int32), (8, 8, 8))


def test_list_rejects_int16_overflow(o):
    with pytest.raises(ValueError):
        o.voxel_list(np.array([[0, 0, 0, 40000, 0, 0]], dtype=np.int32))


def test_empty_and_degenerate(o):
    empty = np.zeros((0, 6), dtype=np.int32)
    assert o.offsets(empty).tolist() == [0]
    assert o.voxel_list(empty).shape == (0, 3)
    assert not o.grid(empty, (32, 2, 2)).any()
    pt = np.array([[5, -6, 7, 5, -6, 7]], dtype=np.int32)
    assert o.voxel_list(pt).tolist() == [[5, -6, 7]]
    assert o.counts(pt).tolist() == [1]
