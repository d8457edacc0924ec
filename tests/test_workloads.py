"""Seeded generators reproduce the stated shapes and distributions (CPU)."""

import numpy as np

from paper_2009_09500_amd import workloads


def _N(segs):
    s = segs.astype(np.int64)
    return np.abs(s[:, 3:] - s[:, :3]).max(axis=1)


def test_deterministic():
    a = workloads.arbitrary_length(n=1000)["segs"]
    b = workloads.arbitrary_length(n=1000)["segs"]
    assert np.array_equal(a, b)


def test_small_uniform():
    c = workloads.small_uniform()
    s = c["segs"]
    assert s.shape == (1000, 6) and s.dtype == np.int32
    assert s.min() >= 0 and s.max() < 256
    assert _N(s).max() <= 255


def test_fixed_length_every_N_is_64():
    s = workloads.fixed_length(n=100_000)["segs"]
    assert np.all(_N(s) == 64)
    assert s.min() >= -64 and s.max() <= 1023
    assert (s < 0).any()


def test_arbitrary_length_inside_volume():
    c = workloads.arbitrary_length(n=200_000)
    s = c["segs"]
    assert s.min() >= 0 and s.max() <= 2047
    N = _N(s)
    assert N.max() <= 2047
    assert 0 < (N == 0).mean() < 0.01
    # log-uniform lengths: the median sits near sqrt(2048) before clipping
    assert 20 < np.median(N) < 60


def test_scenes():
    sc = workloads.scenes(n_scenes=16)
    assert len(sc) == 16
    for x in sc:
        V = x["dims"][0]
        assert V in (64, 128, 256, 512)
        assert 1000 <= x["segs"].shape[0] <= 200_000
        assert x["segs"].min() >= 0 and x["segs"].max() < V


def test_icosphere_topology():
    for m in (1, 2, 5, 19):
        pos, edges, F = workloads.geodesic_icosphere(m)
        V, E = pos.shape[0], edges.shape[0]
        assert V == 10 * m * m + 2 and E == 30 * m * m and F == 20 * m * m
        assert V - E + F == 2
        assert np.allclose(np.linalg.norm(pos, axis=1), 1.0)
        assert np.all(edges[:, 0] < edges[:, 1])


def test_wireframe_request():
    q = workloads.wireframe_request(0)
    s = q["segs"]
    assert s.min() >= 0 and s.max() <= 511
    assert 10_000 * 0.8 <= s.shape[0] <= 1_000_000 * 1.2
    assert s.shape[0] == 30 * q["frequency"] ** 2


def test_paper_shapes():
    L = workloads.paper_arbitrary_lengths()
    assert L.size == 1024 and int(L.sum()) == 10 ** 9 and L.min() >= 1
    segs = workloads.paper_segments(L)["segs"].astype(np.int64)
    d = np.abs(segs[:, 3:] - segs[:, :3])
    assert np.array_equal(d.max(axis=1) + 1, L)
    assert d.max() < 2 ** 30
    one = workloads.paper_segments([10 ** 6])["segs"].astype(np.int64)
    assert np.abs(one[0, 3:] - one[0, :3]).max() == 10 ** 6 - 1
