"""Pins of the oracle's int32 lists (the same voxels as the int16 lists, for
segments whose coordinates leave the int16 range: the paper's single-segment
experiment reaches 10^6 voxels, Section 5).  CPU only."""

import numpy as np
import pytest

from oracle import oracle
from tests import pins


def test_list32_pins():
    assert pins.check_list32(oracle.default()) is None


def test_nearest_centre_at_matches_fraction_list():
    # the sampled pin's helper against the whole-segment Fraction search
    for seg in pins.random_segments(40, 71, -60, 60):
        exp = pins.fraction_list(seg)
        assert [pins.nearest_centre_at(seg, k) for k in range(len(exp))] == exp


def test_list32_equals_list16_in_range():
    segs = pins.random_segments(300, 72, -2000, 2000)
    assert np.array_equal(oracle.voxel_list32(segs), oracle.voxel_list(segs).astype(np.int32))


def test_list32_domain():
    ok = np.array([[0, 0, 0, 5, -7, 3], [2 ** 31 - 1, -(2 ** 31), 0, 2 ** 31 - 4, -(2 ** 31) + 2, 0]], np.int32)
    assert oracle.voxel_list32(ok).shape == (8 + 4, 3)
    with pytest.raises(ValueError):
        oracle.voxel_list32(np.array([[0, 0, 0, 2 ** 30, 0, 0]], np.int32))
    with pytest.raises(ValueError):
        oracle.voxel_list32(np.array([[0, 2 ** 29, 0, 0, -(2 ** 29), 0]], np.int32))
    assert oracle.voxel_list32(np.zeros((0, 6), np.int32)).shape == (0, 3)
