"""The brick path's exact integer helpers (brick walk, the walk cut into
parts, k-window clipping), built for the host from the library's own header,
against the oracle's voxel lists grouped by brick (CPU only)."""

import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle
from paper_2009_09500_amd import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "cpp", "brick_walk_check.cpp")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("bwc") / "brick_walk_check")
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17",
                           "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2009_09500_amd", "csrc"),
                           "-o", out, SRC])
    return out


def run(driver, segs, dims, lg, euclid=False):
    inp = "%d %d %d %d %d %d %d\n" % (tuple(dims) + tuple(lg) + (len(segs),))
    inp += "\n".join(" ".join(str(int(v)) for v in s) for s in segs) + "\n"
    r = subprocess.run([driver] + (["euclid"] if euclid else []), input=inp, capture_output=True, text=True,
                       check=True)
    out = []
    for line in r.stdout.splitlines():
        # The driver reports a walk whose parts or windows disagree.
        assert "MISMATCH" not in line, line
        body = line.split(":", 1)[1].strip()
        if body == "out":
            out.append(None)
            continue
        out.append([tuple(int(v) for v in p.split()) for p in body.split(";") if p.strip()])
    return out


def expected(segs, dims, lg):
    offs = oracle.offsets(segs)
    lst = oracle.voxel_list(segs).astype(np.int64)
    nb = [(dims[a] + (1 << lg[a]) - 1) >> lg[a] for a in range(3)]
    res = []
    for i in range(len(segs)):
        v = lst[offs[i]:offs[i + 1]]
        b = v >> np.array(lg)
        bid = (b[:, 2] * nb[1] + b[:, 1]) * nb[0] + b[:, 0]
        pieces = []
        start = 0
        for k in range(1, len(bid) + 1):
            if k == len(bid) or bid[k] != bid[start]:
                pieces.append((int(bid[start]), start, k - 1))
                start = k
        res.append(pieces)
    return res


def inside(dims, n, seed):
    rng = np.random.default_rng(seed)
    p = [np.stack([rng.integers(0, d, n) for d in dims], 1) for _ in range(2)]
    return np.concatenate(p, 1).astype(np.int32)


CASES = [
    ((256, 256, 256), (7, 7, 6)),
    ((2048, 2048, 2048), (7, 7, 6)),
    ((2048, 2048, 2048), (8, 6, 5)),
    ((512, 512, 512), (8, 6, 6)),
    ((8192, 64, 16384), (8, 6, 5)),
    ((96, 40, 20), (5, 3, 2)),
    ((64, 64, 64), (7, 7, 6)),
    ((512, 512, 512), (8, 6, 6)),
    ((160, 33, 7), (6, 4, 1)),
]


@pytest.mark.parametrize("dims,lg", CASES)
def test_walk_and_windows(driver, dims, lg):
    segs = inside(dims, 1500, sum(dims) + sum(lg))
    got = run(driver, segs, dims, lg)
    exp = expected(segs, dims, lg)
    for i, (g, e) in enumerate(zip(got, exp)):
        assert g == e, "segment %s: %s != %s" % (segs[i].tolist(), g, e)


def test_arbitrary_length_workload(driver):
    c = workloads.arbitrary_length(n=3000)
    got = run(driver, c["segs"], c["dims"], (7, 7, 6))
    exp = expected(c["segs"], c["dims"], (7, 7, 6))
    assert got == exp


def test_boundary_hugging_segments(driver):
    """Segments along brick faces and edges, and through brick corners."""
    dims, lg = (256, 128, 128), (6, 5, 5)
    segs = []
    for a in (0, 31, 32, 63, 64, 127):
        segs.append([a, 0, 0, a, 127, 127])
        segs.append([0, a % 128, 0, 255, a % 128, 127])
        segs.append([0, 0, a % 128, 255, 127, a % 128])
    segs += [[0, 0, 0, 127, 127, 127], [127, 127, 127, 0, 0, 0], [31, 31, 31, 32, 32, 32],
             [32, 32, 32, 31, 31, 31], [0, 31, 0, 255, 32, 1], [255, 0, 127, 0, 127, 0]]
    segs = np.array(segs, dtype=np.int32)
    assert run(driver, segs, dims, lg) == expected(segs, dims, lg)


def test_out_of_volume_flagged(driver):
    segs = np.array([[0, 0, 0, 64, 0, 0], [-1, 0, 0, 3, 3, 3], [1, 1, 1, 2, 2, 2]], np.int32)
    got = run(driver, segs, (64, 64, 64), (5, 5, 5))
    assert got[0] is None and got[1] is None and got[2] is not None


def expected_euclid(segs, dims, lg):
    """Pieces under the Euclidean N from the oracle's samples k = 0..N (each
    sample, duplicates included, is one step of the walk)."""
    o = oracle.native()
    nb = [(dims[a] + (1 << lg[a]) - 1) >> lg[a] for a in range(3)]
    res = []
    for s in segs:
        n = o.length_euclid(s)
        v = np.array([o.sample_euclid(s, k) for k in range(n + 1)], dtype=np.int64)
        b = v >> np.array(lg)
        bid = (b[:, 2] * nb[1] + b[:, 1]) * nb[0] + b[:, 0]
        pieces, start = [], 0
        for k in range(1, len(bid) + 1):
            if k == len(bid) or bid[k] != bid[start]:
                pieces.append((int(bid[start]), start, k - 1))
                start = k
        res.append(pieces)
    return res


@pytest.mark.parametrize("dims,lg", [((96, 40, 20), (5, 3, 2)), ((320, 200, 100), (6, 5, 4)),
                                     ((64, 64, 64), (5, 3, 3))])
def test_walk_euclid(driver, dims, lg):
    """The walk (whole and cut into parts) under the Euclidean N."""
    segs = inside(dims, 250, 7 * sum(dims) + sum(lg))
    assert run(driver, segs, dims, lg, euclid=True) == expected_euclid(segs, dims, lg)


def test_parts_long_walks(driver):
    """Segments crossing many small bricks: every walk is cut into 8 parts,
    some of them empty (fewer bricks along the cut axis than parts), and the
    parts are checked against the whole walk for both lengths."""
    dims, lg = (1024, 512, 256), (5, 4, 4)
    segs = inside(dims, 800, 99)
    segs[:40, 3:] = segs[:40, :3]                  # points
    segs[40:80, 4:] = segs[40:80, 1:3]             # along x
    segs[80:120, 3] = segs[80:120, 0] + 17 * ((segs[80:120, 0] < 512) * 2 - 1)  # dx = +-17
    got = run(driver, segs, dims, lg)
    assert got == expected(segs, dims, lg)
    run(driver, segs, dims, lg, euclid=True)       # parts == whole, windows == box windows


def test_work_items():
    """The fill's work items (a brick of more than T records cut into parts):
    bounded extra items and cut bricks, exact tiling of each brick's records
    (tests/cpp/items_check.cpp, the library's own header built for the host)."""
    import tempfile
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "items_check")
        subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17",
                               "-I", os.path.join(ROOT, "include"),
                               "-I", os.path.join(ROOT, "paper_2009_09500_amd", "csrc"),
                               "-o", exe, os.path.join(ROOT, "tests", "cpp", "items_check.cpp")])
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
        assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
