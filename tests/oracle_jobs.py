"""Oracle results for the full-size workloads, computed in the background.

The CPU oracle is single-threaded and needs about a minute for the 4M-segment
2048^3 volume.  For the GPU parity tests at full size this module runs the
unchanged oracle on disjoint shards of the segments in forked CPU worker
processes and ORs the shard volumes (a volume is the OR of its segments'
voxels, so the union of shards is the oracle's own result).  It publishes
SHA-256 digests of fixed-size blocks of each expected volume, which the GPU
test compares with the same digests of the GPU output.

`python -m tests.oracle_jobs OUTDIR JOB...` writes OUTDIR/JOB.json.  The
pytest session starts it before any test touches the GPU (see conftest.py).
"""

from __future__ import annotations

import hashlib
import json
import mmap
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

BLOCK_BYTES = 16 << 20


def block_digests(words: np.ndarray) -> list:
    """SHA-256 (hex, 16 chars) of consecutive BLOCK_BYTES blocks."""
    buf = np.ascontiguousarray(words).view(np.uint8)
    return [hashlib.sha256(buf[i:i + BLOCK_BYTES]).hexdigest()[:16]
            for i in range(0, buf.size, BLOCK_BYTES)]


def popcount(words: np.ndarray) -> int:
    return int(np.unpackbits(np.ascontiguousarray(words).view(np.uint8)).sum())


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def sharded_grid(segs: np.ndarray, dims, euclid: bool = False) -> np.ndarray:
    """The oracle volume of all segments, computed as the OR of the oracle
    volumes of P disjoint shards (P forked workers, no GPU involved); euclid:
    the Euclidean N of eq. (1)."""
    from oracle import oracle
    oracle.default()  # build/load before forking
    grid_fn = oracle.grid_euclid if euclid else oracle.grid
    nwords = (int(dims[0]) * int(dims[1]) * int(dims[2]) + 31) // 32
    P = min(_workers(), max(1, segs.shape[0] // 50000))
    if P == 1:
        return grid_fn(segs, dims)
    bounds = np.linspace(0, segs.shape[0], P + 1).astype(np.int64)
    maps = [mmap.mmap(-1, nwords * 4) for _ in range(P)]
    pids = []
    for p in range(P):
        pid = os.fork()
        if pid == 0:  # child: one shard, result into its shared map
            try:
                g = grid_fn(segs[bounds[p]:bounds[p + 1]], dims)
                np.frombuffer(maps[p], dtype=np.uint32)[:] = g
                os._exit(0)
            except BaseException:
                os._exit(1)
        pids.append(pid)
    for pid in pids:
        _, st = os.waitpid(pid, 0)
        if st != 0:
            raise RuntimeError("oracle shard worker failed")
    out = np.frombuffer(maps[0], dtype=np.uint32).copy()
    for p in range(1, P):
        out |= np.frombuffer(maps[p], dtype=np.uint32)
    for m in maps:
        m.close()
    return out


def job_arbitrary4m() -> dict:
    from paper_2009_09500_amd import workloads
    c = workloads.arbitrary_length()
    g = sharded_grid(c["segs"], c["dims"])
    return {"dims": list(c["dims"]), "words": int(g.size), "digests": block_digests(g),
            "popcount": popcount(g)}


def sharded_counts_euclid(segs: np.ndarray) -> np.ndarray:
    """The oracle's per-segment voxel counts with the Euclidean N, on
    disjoint shards in forked workers."""
    from oracle import oracle
    oracle.default()
    P = min(_workers(), max(1, segs.shape[0] // 50000))
    bounds = np.linspace(0, segs.shape[0], P + 1).astype(np.int64)
    m = mmap.mmap(-1, max(4 * segs.shape[0], 4))
    pids = []
    for p in range(P):
        pid = os.fork()
        if pid == 0:
            try:
                c = oracle.counts_euclid(segs[bounds[p]:bounds[p + 1]])
                np.frombuffer(m, dtype=np.int32)[bounds[p]:bounds[p + 1]] = c
                os._exit(0)
            except BaseException:
                os._exit(1)
        pids.append(pid)
    for pid in pids:
        _, st = os.waitpid(pid, 0)
        if st != 0:
            raise RuntimeError("oracle count worker failed")
    out = np.frombuffer(m, dtype=np.int32)[:segs.shape[0]].copy()
    m.close()
    return out


def job_arbitrary4m_euclid() -> dict:
    """The arbitrary-length workload with the Euclidean N of eq. (1): every
    16 MiB block of the cleared 2048^3 volume, its popcount, and a digest of
    all per-segment counts."""
    from paper_2009_09500_amd import workloads
    c = workloads.arbitrary_length()
    g = sharded_grid(c["segs"], c["dims"], euclid=True)
    counts = sharded_counts_euclid(c["segs"])
    return {"dims": list(c["dims"]), "words": int(g.size), "digests": block_digests(g),
            "popcount": popcount(g), "counts_sha256": hashlib.sha256(counts.tobytes()).hexdigest(),
            "counts_sum": int(counts.astype(np.int64).sum())}


def job_scenes() -> dict:
    """Per-scene oracle volumes of the 256-scene batch (scenes split across
    workers; each scene computed whole)."""
    from oracle import oracle
    from paper_2009_09500_amd import workloads
    sc = workloads.scenes()
    oracle.default()
    P = _workers()
    res = [None] * len(sc)
    r, w = os.pipe()
    pids = []
    for p in range(P):
        pid = os.fork()
        if pid == 0:
            os.close(r)
            try:
                out = {}
                for s in range(p, len(sc), P):
                    g = oracle.grid(sc[s]["segs"], sc[s]["dims"])
                    out[s] = block_digests(g)
                os.write(w, (json.dumps(out) + "\n").encode())
                os._exit(0)
            except BaseException:
                os._exit(1)
        pids.append(pid)
    os.close(w)
    data = b""
    with os.fdopen(r, "rb") as f:
        data = f.read()
    for pid in pids:
        _, st = os.waitpid(pid, 0)
        if st != 0:
            raise RuntimeError("oracle scene worker failed")
    for line in data.decode().splitlines():
        for k, v in json.loads(line).items():
            res[int(k)] = v
    return {"n_scenes": len(sc), "digests": res}


JOBS = {"arbitrary4m": job_arbitrary4m, "scenes": job_scenes, "arbitrary4m_euclid": job_arbitrary4m_euclid}


def result_path(outdir: str, name: str) -> str:
    return os.path.join(outdir, name + ".json")


def wait_result(outdir: str, name: str, timeout: float) -> dict:
    """Waits for a job's result (raises on timeout or job failure)."""
    t0 = time.time()
    path = result_path(outdir, name)
    err = path + ".err"
    while time.time() - t0 < timeout:
        if os.path.exists(path):
            return json.load(open(path))
        if os.path.exists(err):
            raise RuntimeError("oracle job %s failed: %s" % (name, open(err).read()))
        time.sleep(0.5)
    raise TimeoutError("oracle job %s not done after %.0f s" % (name, timeout))


def main(argv):
    outdir = argv[0]
    os.makedirs(outdir, exist_ok=True)
    for name in argv[1:]:
        t = time.time()
        try:
            res = JOBS[name]()
            res["seconds"] = time.time() - t
            tmp = result_path(outdir, name) + ".tmp"
            with open(tmp, "w") as f:
                json.dump(res, f)
            os.replace(tmp, result_path(outdir, name))
        except BaseException as e:  # report, keep going with the next job
            with open(result_path(outdir, name) + ".err", "w") as f:
                f.write(repr(e))


if __name__ == "__main__":
    main(sys.argv[1:])
