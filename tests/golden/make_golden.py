"""Writes worked_segments.txt from the CPU oracle only.

Usage: python tests/golden/make_golden.py
The segments are hand-picked small cases of eq. (3) with round-half-up
voxels: both tie directions, every octant sign, N = 0, the three dominant
axes.  The test suite re-derives each list by exact nearest-centre search,
so the file is pinned independently of the oracle that wrote it.
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import oracle  # noqa: E402

SEGMENTS = [
    (0, 0, 0, 5, 2, 1),
    (0, 0, 0, -5, -2, 1),
    (0, 0, 0, 2, 1, 0),
    (0, 0, 0, 2, -1, 0),
    (3, 3, 3, 3, 3, 3),
    (1, 2, 3, 1, 9, 3),
    (10, 0, 0, 0, 3, 7),
    (-4, 7, 2, 3, -1, -6),
    (0, 0, 0, 4, 4, 4),
    (5, 5, 0, 0, 2, 7),
    (0, 0, 0, 6, 3, 2),
    (2, 0, 1, 2, 5, 4),
]


def main():
    segs = np.array(SEGMENTS, dtype=np.int32)
    lst = oracle.voxel_list(segs)
    offs = oracle.offsets(segs)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "worked_segments.txt")
    with open(path, "w") as f:
        f.write("# Worked cases of the parametric method (arXiv 2009.09500, Section 3,\n")
        f.write("# eq. (2)-(3), algorithm of Fig. 3) with N = max|d_a|, k = 0..N and\n")
        f.write("# round-half-up voxels.  Written by tests/golden/make_golden.py from\n")
        f.write("# the CPU oracle; one line per segment: x0 y0 z0 x1 y1 z1 : voxels.\n")
        for i, s in enumerate(segs):
            v = lst[offs[i]:offs[i + 1]]
            f.write("%s : %s\n" % (" ".join(str(int(c)) for c in s),
                                   " ".join("%d,%d,%d" % tuple(int(c) for c in p) for p in v)))


if __name__ == "__main__":
    main()
