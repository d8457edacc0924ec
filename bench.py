"""Benchmark of the voxelization hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

A step is one call of the grid path on the arbitrary-length workload:
4 194 304 segments (seed 1003) voxelized into a cleared 2048^3 packed
bit-volume (1 GiB) plus per-segment counts, inputs resident in HBM.  The
timed region is exactly K steps between HIP events on the launch stream,
bracketed by device synchronisation.  Prints ONE JSON line.

Also reported (in "extra"): the fixed-length list workload (1 048 576
segments, 68 157 440 voxels), the same lists and a 100 000-segment 512^3
bit-volume with the paper's Euclidean length of eq. (1), the paper's three
experiment shapes as int32 lists (with and without the copy to the host),
the small
1000-segment workload and a single
segment alone (launch latency), each timed the same way; the 256-scene
workload as plain calls, one batched launch sequence and a graph replay;
and the serving loop on wireframe requests (saturation throughput, then a
Poisson sweep with p50/p99 request latency).

The CPU baseline is the oracle (oracle/, single-threaded C) timed on a
bounded sample of the same workload; it is a reported reference, not the
target.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
# The paper's timings on its fastest GPU ("GTX 1070i" as printed) in ms,
# copy to the host included (Section 5, Table 2: one segment of L voxels;
# Table 3: 1024 segments of L voxels; Table 4: 1024 arbitrary segments
# totalling 10^9 voxels).
PAPER_GTX1070_MS = {
    "single": {10 ** 3: 0.45, 10 ** 4: 0.51, 10 ** 5: 0.92, 10 ** 6: 3.65428571},
    "fixed": {20: 0.42, 2000: 4.13, 20000: 43.85, 200000: 427.62},
    "arbitrary": 4071.01,
}
METRIC = "voxels/sec + HBM GB/s (batched vs plain), p50/p99 scene latency"


def _events_time(stream, fn, steps):
    import torch
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        start.record(stream)
        for _ in range(steps):
            fn()
        end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end)


def _time_then_profile(binding, stream, fn, reps):
    """(ms per call, per-kernel records): the calls timed as they run for a
    caller (no per-kernel events in the stream), then the same number of
    calls again with the library's per-kernel HIP events for the breakdown.
    For the small workloads the events themselves cost a visible share of
    the call."""
    ms = _events_time(stream, fn, reps) / reps
    binding.vox_profile_reset()
    binding.vox_profile_enable(True)
    _events_time(stream, fn, reps)
    binding.vox_profile_enable(False)
    prof = binding.vox_profile_records()
    binding.vox_profile_reset()
    return ms, prof


# The sources the brick kernels are compiled from (their translation unit):
# committed counter summaries stay valid while these are unchanged.
BRICK_SOURCES = ["include/vox.h"] + ["paper_2009_09500_amd/csrc/" + f for f in
                                      ("vox_brick.hip", "vox_device.h", "vox_direct.h", "vox_exact.h",
                                       "vox_internal.h")]


def source_digest(files) -> str:
    h = hashlib.sha256()
    for f in sorted(files):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def counter_traffic(kernel: str, workload: str, sources):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or
    None when there is none or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", "pmc_%s_%s.txt" % (kernel, workload))
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("source_digest") != source_digest(sources):
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def counter_fields(path: str, sources):
    """{kernel: {column: value}} of a committed rocprofv3 counter summary
    (profiles/*.txt), or None when there is none or the kernel sources
    changed since it was taken."""
    if not os.path.exists(path):
        return None
    rows, header, digest = {}, None, None
    for line in open(path):
        if line.startswith("#"):
            continue
        if line.startswith("source_digest:"):
            digest = line.split(":", 1)[1].strip()
            continue
        parts = line.split()
        if not parts:
            continue
        if parts[0] == "kernel":
            header = parts[1:]
            continue
        if header and len(parts) >= len(header) + 1:
            name = " ".join(parts[:len(parts) - len(header)])
            try:
                rows[name] = dict(zip(header, (float(v) for v in parts[-len(header):])))
            except ValueError:
                pass
    if digest != source_digest(sources):
        return None
    return rows


CUS = 256
CLOCK_HZ = 2.4e9
VALU_PEAK = CUS * CLOCK_HZ        # wave64 VALU instructions per second (one per CU per clock)
# 32-bit VALU lane operations per second: 4 SIMDs of 16 lanes per CU, one
# operation per lane per clock (the fp32 vector peak of 157.3 TFLOP/s counts
# an FMA as two and packed fp32 as two more).
ALU_PEAK_TOPS = CUS * 64 * CLOCK_HZ / 1e12
# The fill's algorithmic ALU work per voxel: the stepping of eq. (3) with the
# minor error terms in packed halves (packed add, packed shift, packed
# multiply-add, dot product, dominant stride) and the LDS word and bit of the
# voxel (shift, mask, shift): 8 lane operations; the LDS OR is not ALU work.
FILL_OPS_PER_VOXEL = 8


def counter_bound(kernel: str, workload: str, sources, avg_ms: float, traffic):
    """What bounds a kernel, from its committed SQ counters: the time its VALU
    wave instructions need at the chip's issue rate (256 CUs x 2.4 GHz, one
    wave64 instruction per CU per clock) against the time its HBM bytes (the
    FETCH/WRITE counters) need at 8 TB/s."""
    rows = counter_fields(os.path.join(ROOT, "profiles", "sq_%s_%s.txt" % (kernel, workload)), sources)
    if not rows or traffic is None:
        return None
    row = next((v for k, v in rows.items() if "k_" + kernel in k), None)
    if row is None or "INSTS_VALU" not in row:
        return None
    valu_ms = row["INSTS_VALU"] / VALU_PEAK * 1e3
    hbm_ms = traffic / (HBM_PEAK_GBS * 1e9) * 1e3
    return {"bound": "alu" if valu_ms > hbm_ms else "hbm", "valu_wave_instructions": row["INSTS_VALU"],
            "valu_ms_at_peak_issue": valu_ms, "hbm_ms_at_peak": hbm_ms,
            "valu_issue_frac": valu_ms / avg_ms if avg_ms > 0 else None}


def _roofline_line(kernel, algo_bytes, achieved_gbs, avg_ms, traffic, bound, voxels):
    """The dominant kernel's roofline.  Its bound comes from the committed
    counters while they match the kernel sources ("hbm" otherwise): against
    HBM, its algorithmic bytes per launch / launch time vs 8 TB/s; against
    the ALU, its algorithmic lane operations per launch (FILL_OPS_PER_VOXEL a
    voxel) / launch time vs ALU_PEAK_TOPS.  Both are given; the top-level
    fields are those of the bound."""
    hbm = {"achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved_gbs / HBM_PEAK_GBS,
           "algorithmic_bytes_per_launch": algo_bytes}
    ops = voxels * FILL_OPS_PER_VOXEL if kernel == "brick_fill" else None
    alu = None
    if ops is not None and avg_ms > 0:
        a = ops / (avg_ms * 1e-3) / 1e12
        alu = {"achieved": a, "peak": ALU_PEAK_TOPS, "unit": "Tlane-op/s", "frac": a / ALU_PEAK_TOPS,
               "algorithmic_lane_ops_per_launch": ops, "lane_ops_per_voxel": FILL_OPS_PER_VOXEL}
    kind = bound["bound"] if bound else "hbm"
    top = alu if (kind == "alu" and alu is not None) else hbm
    return {"kernel": kernel, "bound": kind if top is alu else "hbm", "achieved": top["achieved"],
            "peak": top["peak"], "unit": top["unit"], "frac": top["frac"], "traffic": traffic,
            "avg_launch_ms": avg_ms, "hbm": hbm, "alu": alu, "bound_from_counters": bound}


def bench_grid(args, torch, binding, workloads, dev, stream):
    import tempfile
    from paper_2009_09500_amd import autotune
    c = workloads.arbitrary_length()
    segs_np = c["segs"]
    dims = c["dims"]
    n = segs_np.shape[0]
    segs = torch.from_numpy(segs_np).to(dev)
    # Launch shape: the autotuner times every candidate on this workload and
    # installs the fastest for this volume and segment count (--no-tune: the
    # library default, as in the profiler runs).
    if args.no_tune:
        tuned = {"choice": "library default (not tuned in this run)"}
    else:
        with tempfile.TemporaryDirectory() as d:
            best, times = autotune.tune_grid(segs, dims, reps=2,
                                             cache=autotune.TuneCache(os.path.join(d, "t.json")))
        tuned = {"choice": {"brick_lg": list(best[:3]), "fill_wgs_per_cu": best[3]},
                 "ms_per_candidate": {"%d,%d,%d,%d" % k: round(v, 4) for k, v in times.items()}}
    grid = torch.empty(binding.grid_words(dims), dtype=torch.int32, device=dev)
    counts = torch.empty(n, dtype=torch.int32, device=dev)
    # The compact workspace (16 piece records a segment, about 1 GiB here,
    # against 4.4 GiB for the worst case of every segment crossing the whole
    # volume); the call would fall back to the direct kernels if its records
    # did not fit.
    work_bytes = binding.vox_workspace_bytes(binding.VOX_OP_GRID, n, 1)
    work = binding.workspace(work_bytes, dev)
    voxels = int((np.abs(segs_np[:, 3:].astype(np.int64) - segs_np[:, :3]).max(1) + 1).sum())

    def step():
        binding.vox_segments_to_grid(segs, dims, grid, counts, binding.VOX_GRID_CLEAR, work,
                                     stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    assert binding.vox_read_status(work, stream=stream) == binding.VOX_OK
    # The K timed steps run as a caller runs them; the per-kernel durations
    # (and the roofline's launch time) come from HIP events around every
    # launch over a second run of K steps.
    ms_call, prof = _time_then_profile(binding, stream, step, args.steps)
    ms = ms_call * args.steps
    pieces, direct_all = binding.vox_read_batch_info(work, stream=stream)
    assert not direct_all, "the piece records did not fit the compact workspace"
    grid_bytes = grid.numel() * 4
    algo_bytes = 24 * n + 4 * n + grid_bytes
    return {
        "n": n, "dims": dims, "voxels": voxels, "ms_total": ms, "prof": prof,
        "algo_bytes": algo_bytes, "grid_bytes": grid_bytes, "segs_np": segs_np, "tuning": tuned,
        "workspace_bytes": work_bytes, "piece_records": pieces,
    }


def bench_list(args, torch, binding, workloads, dev, stream, euclid=False):
    c = workloads.fixed_length()
    segs = torch.from_numpy(c["segs"]).to(dev)
    n = segs.shape[0]
    offsets = torch.empty(n + 1, dtype=torch.int64, device=dev)
    work0 = binding.workspace(binding.vox_list_workspace_bytes(n, 0), dev)
    total = binding.vox_segments_to_list(segs, offsets, None, 0, work0, want_total=True,
                                         stream=stream, euclid=euclid)
    vox = torch.empty((total, 3), dtype=torch.int16, device=dev)
    work = binding.workspace(binding.vox_list_workspace_bytes(n, total), dev)

    def step():
        binding.vox_segments_to_list(segs, offsets, vox, total, work, stream=stream, euclid=euclid)

    for _ in range(args.warmup):
        step()
    steps = max(args.steps, 5)
    ms, prof = _time_then_profile(binding, stream, step, steps)
    algo = 24 * n + 8 * (n + 1) + 6 * total
    kv = prof.get("list_voxels_euclid" if euclid else "list_voxels", (0.0, 1))
    kv_ms = kv[0] / max(kv[1], 1)
    return {
        "workload": ("fixed-length 1048576 segments (Chebyshev length 64) -> int16 lists with the "
                     "Euclidean N of eq. (1), duplicates removed (seed 1002)" if euclid else
                     "fixed-length 1048576 segments x 65 voxels -> int16 lists (seed 1002)"),
        "voxels": total, "ms_per_call": round(ms, 4),
        "voxels_per_s": total / (ms * 1e-3),
        "hbm_gbs_algorithmic": algo / (ms * 1e-3) / 1e9,
        "algorithmic_bytes": algo,
        "kernels_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in prof.items()},
        "list_voxels_kernel_gbs": (6 * total) / (kv_ms * 1e-3) / 1e9 if kv_ms > 0 else None,
        # The voxel kernel against the HBM roofline: it writes 6 B a voxel and
        # reads each segment (24 B) and its offset (8 B).
        "roofline": _roofline("list_voxels_euclid" if euclid else "list_voxels",
                              6 * total + 24 * n + 8 * (n + 1), kv_ms),
    }


def _roofline(kernel, algo_bytes, avg_ms):
    if avg_ms <= 0:
        return None
    achieved = algo_bytes / (avg_ms * 1e-3) / 1e9
    return {"kernel": kernel, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": algo_bytes,
            "avg_launch_ms": avg_ms}


def bench_grid_euclid(args, torch, binding, workloads, dev, stream):
    """Bit-volume with the Euclidean N of eq. (1): 100 000 arbitrary-length
    segments in a cleared 512^3 volume (brick path)."""
    c = workloads.arbitrary_length(n=100_000, volume=512)
    segs = torch.from_numpy(c["segs"]).to(dev)
    n = segs.shape[0]
    dims = c["dims"]
    grid = torch.empty(binding.grid_words(dims), dtype=torch.int32, device=dev)
    counts = torch.empty(n, dtype=torch.int32, device=dev)
    work = binding.workspace(binding.vox_grid_workspace_bytes(n, dims), dev)
    flags = binding.VOX_GRID_CLEAR | binding.VOX_GRID_EUCLID

    def step():
        binding.vox_segments_to_grid(segs, dims, grid, counts, flags, work, stream=stream)

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    voxels = int(counts.sum().item())
    reps = max(args.steps, 10)
    ms, prof = _time_then_profile(binding, stream, step, reps)
    algo = 24 * n + 4 * n + grid.numel() * 4
    return {
        "workload": "arbitrary-length 100000 segments (seed 1003) -> cleared 512^3 bit-volume with the "
                    "Euclidean N of eq. (1)",
        "voxels": voxels, "ms_per_call": round(ms, 4), "voxels_per_s": voxels / (ms * 1e-3),
        "hbm_gbs_algorithmic": algo / (ms * 1e-3) / 1e9, "algorithmic_bytes": algo,
        "kernels_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in prof.items()},
    }


def bench_paper(args, torch, binding, workloads, dev, stream):
    """The paper's three experiment shapes (Section 5, Tables 2-4) as int32
    lists: one segment of 10^3..10^6 voxels; 1024 segments of 20..200 000
    voxels each; 1024 segments of arbitrary length totalling 10^9 voxels.
    Each is timed on the device (inputs resident, the whole list call) and
    again with the copy of the voxel rows into pinned host memory on the
    same stream, the regime the paper's timings include."""

    def run(segs_np, reps, copy_reps):
        segs = torch.from_numpy(segs_np).to(dev)
        n = segs.shape[0]
        offsets = torch.empty(n + 1, dtype=torch.int64, device=dev)
        w0 = binding.workspace(binding.vox_list_workspace_bytes(n, 0), dev)
        total = binding.vox_segments_to_list(segs, offsets, None, 0, w0, want_total=True, stream=stream,
                                             wide=True)
        vox = torch.empty((total, 3), dtype=torch.int32, device=dev)
        work = binding.workspace(binding.vox_list_workspace_bytes(n, total), dev)
        host = torch.empty((total, 3), dtype=torch.int32, pin_memory=True)

        def gen():
            binding.vox_segments_to_list(segs, offsets, vox, total, work, stream=stream, wide=True)

        def gen_copy():
            gen()
            host.copy_(vox, non_blocking=True)

        for _ in range(2):
            gen()
        ms = _events_time(stream, gen, reps) / reps
        gen_copy()
        ms_copy = _events_time(stream, gen_copy, copy_reps) / copy_reps
        algo = 24 * n + 8 * (n + 1) + 12 * total
        out = {"voxels": total, "ms_device": round(ms, 4), "voxels_per_s": total / (ms * 1e-3),
               "hbm_gbs_algorithmic": algo / (ms * 1e-3) / 1e9,
               "hbm_frac_algorithmic": algo / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
               "ms_with_d2h": round(ms_copy, 4), "voxels_per_s_with_d2h": total / (ms_copy * 1e-3),
               "d2h_gbs": 12 * total / (max(ms_copy - ms, 1e-6) * 1e-3) / 1e9}
        del segs, offsets, vox, work, host, w0
        torch.cuda.empty_cache()
        return out

    res = {"output": "int32 xyz rows (vox_segments_to_list32)", "single_segment": {}, "fixed_1024": {}}
    for L in (10 ** 3, 10 ** 4, 10 ** 5, 10 ** 6):
        res["single_segment"][str(L)] = run(workloads.paper_segments([L])["segs"], 20, 5)
        res["single_segment"][str(L)]["paper_ms_gtx1070"] = PAPER_GTX1070_MS["single"][L]
    for L in (20, 200, 2000, 20000, 200000):
        res["fixed_1024"][str(L)] = run(workloads.paper_segments([L] * 1024, seed=90 + L)["segs"], 10, 3)
        res["fixed_1024"][str(L)]["paper_ms_gtx1070"] = PAPER_GTX1070_MS["fixed"].get(L)
    L = workloads.paper_arbitrary_lengths()
    res["arbitrary_1024_total_1e9"] = run(workloads.paper_segments(L)["segs"], 5, 2)
    res["arbitrary_1024_total_1e9"]["paper_ms_gtx1070"] = PAPER_GTX1070_MS["arbitrary"]
    res["paper_context"] = ("paper_ms_gtx1070: the paper's times on its fastest GPU ('GTX 1070i' as printed "
                            "in Tables 2-4 of arXiv 2009.09500), which include the copy of the "
                            "voxels to the host; compare with ms_with_d2h (null: length not in the tables)")
    return res


def bench_small(args, torch, binding, workloads, dev, stream):
    out = {}
    for name, c in (("small_1000_segments_256^3", workloads.small_uniform()),
                    ("single_segment_256_voxels", workloads.single_diagonal())):
        segs = torch.from_numpy(c["segs"]).to(dev)
        n = segs.shape[0]
        dims = c["dims"]
        grid = torch.empty(binding.grid_words(dims), dtype=torch.int32, device=dev)
        work = binding.workspace(binding.vox_grid_workspace_bytes(n, dims), dev)
        offsets = torch.empty(n + 1, dtype=torch.int64, device=dev)
        w0 = binding.workspace(binding.vox_list_workspace_bytes(n, 0), dev)
        total = binding.vox_segments_to_list(segs, offsets, None, 0, w0, want_total=True,
                                             stream=stream)
        vox = torch.empty((total, 3), dtype=torch.int16, device=dev)
        wl = binding.workspace(binding.vox_list_workspace_bytes(n, total), dev)

        def g():
            binding.vox_segments_to_grid(segs, dims, grid, None, binding.VOX_GRID_CLEAR, work,
                                         stream=stream)

        def l():
            binding.vox_segments_to_list(segs, offsets, vox, total, wl, stream=stream)

        for _ in range(3):
            g()
            l()
        reps = 50
        out[name] = {
            "voxels": total,
            "grid_us_per_call": round(_events_time(stream, g, reps) / reps * 1e3, 2),
            "list_us_per_call": round(_events_time(stream, l, reps) / reps * 1e3, 2),
        }
    return out


def bench_batch(args, torch, binding, workloads, dev, stream):
    """The scene workload: 256 volumes, one plain call each vs one batched
    launch sequence vs a HIP-graph replay of it (all clearing)."""
    sc = workloads.scenes()
    clear = binding.VOX_GRID_CLEAR
    segs = [torch.from_numpy(x["segs"]).to(dev) for x in sc]
    grids = [torch.empty(binding.grid_words(x["dims"]), dtype=torch.int32, device=dev) for x in sc]
    n = sum(s.shape[0] for s in segs)
    voxels = sum(int((np.abs(x["segs"][:, 3:].astype(np.int64) - x["segs"][:, :3]).max(1) + 1).sum())
                 for x in sc)
    algo = 24 * n + sum(g.numel() * 4 for g in grids)
    work = binding.workspace(max(binding.vox_grid_workspace_bytes(s.shape[0], x["dims"])
                                 for s, x in zip(segs, sc)), dev)

    def plain():
        for s, x, g in zip(segs, sc, grids):
            binding.vox_segments_to_grid(s, x["dims"], g, None, clear, work, stream=stream)

    d_scenes = torch.from_numpy(binding.scene_table([(s, x["dims"], g, None, clear)
                                                     for s, x, g in zip(segs, sc, grids)])).to(dev)
    bwork = binding.workspace(binding.batch_workspace_bytes(n, len(sc)), dev)

    def batched():
        binding.vox_batch_scenes(d_scenes, len(sc), n, bwork, stream=stream)

    for _ in range(2):
        plain()
        batched()
    torch.cuda.synchronize()
    assert binding.vox_read_status(bwork, stream=stream) == binding.VOX_OK
    side = torch.cuda.Stream(device=dev)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        binding.vox_batch_scenes(d_scenes, len(sc), n, bwork, stream=side)
    torch.cuda.synchronize()
    reps = max(args.steps // 4, 3)
    t_plain = _events_time(stream, plain, reps) / reps
    t_batch = _events_time(stream, batched, reps) / reps
    t_graph = _events_time(stream, graph.replay, reps) / reps
    binding.vox_profile_reset()
    binding.vox_profile_enable(True)
    batched()
    torch.cuda.synchronize()
    binding.vox_profile_enable(False)
    prof = binding.vox_profile_records()
    binding.vox_profile_reset()

    def rate(ms):
        return {"ms": round(ms, 4), "voxels_per_s": voxels / (ms * 1e-3),
                "hbm_gbs_algorithmic": algo / (ms * 1e-3) / 1e9}
    return {
        "workload": "256 scenes (seed 1004), volumes 64^3..512^3, %d segments, cleared grids" % n,
        "segments": n, "voxels": voxels, "algorithmic_bytes": algo,
        "plain_256_calls": rate(t_plain), "batched": rate(t_batch), "graph_replay": rate(t_graph),
        "speedup_batched_vs_plain": t_plain / t_batch,
        "speedup_graph_vs_plain": t_plain / t_graph,
        "batched_kernels_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in prof.items()},
        "workspace_bytes": int(bwork.numel()),
        "piece_records": binding.vox_read_batch_info(bwork, stream=stream)[0],
    }


def _wireframe_pool(n_requests, workers=16):
    """Requests r = 0..n-1 of the serving stream (seeds 1005 + r), generated
    in worker processes."""
    import concurrent.futures as cf
    from paper_2009_09500_amd import workloads
    with cf.ProcessPoolExecutor(max_workers=min(workers, os.cpu_count() or 1)) as ex:
        return list(ex.map(workloads.wireframe_request, range(n_requests), chunksize=8))


def bench_serving(args, torch, binding, workloads, dev, n_requests=1000):
    """Wireframe requests into resident 512^3 grids: saturation throughput
    (all requests at t=0), then Poisson arrivals at fractions of it.  Request
    r of every run is the icosphere of seed 1005 + r."""
    from paper_2009_09500_amd import serving
    pool = _wireframe_pool(n_requests)
    pinned = [serving.GpuExecutor.pin(w["segs"]) for w in pool]
    dims = pool[0]["dims"]
    vox = [int((np.abs(w["segs"][:, 3:].astype(np.int64) - w["segs"][:, :3]).max(1) + 1).sum())
           for w in pool]
    max_batch_segments, max_batch_scenes, n_slots = 2_000_000, 32, 48
    ex = serving.GpuExecutor(dims, n_slots=n_slots, max_batch_segments=max_batch_segments,
                             max_batch_scenes=max_batch_scenes, device=dev)
    budget = ex.admission_budget()

    def requests(arrivals):
        return [serving.Request(i, pool[i]["segs"], dims, float(t), voxels=vox[i],
                                dev={"pinned": pinned[i]})
                for i, t in enumerate(arrivals)]

    def once(arrivals):
        sched = serving.Scheduler(n_slots=n_slots, budget_bytes=budget, max_batch_segments=max_batch_segments,
                                  max_batch_scenes=max_batch_scenes)
        out = serving.run(requests(arrivals), ex, sched)
        assert ex.status() == binding.VOX_OK and out["failed_requests"] == 0
        return out

    once(np.zeros(min(24, n_requests)))                         # warm-up
    sat = once(np.zeros(n_requests))
    sweep = []
    for f in (0.25, 0.5, 0.75, 1.0, 1.25):
        rate = f * sat["requests_per_s"]
        st = once(serving.poisson_arrivals(n_requests, rate, seed=int(f * 100)))
        st["offered_rate_per_s"] = rate
        st["fraction_of_saturation"] = f
        sweep.append({k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.items()})
    edges = [w["segs"].shape[0] for w in pool]
    return {
        "workload": "wireframe requests: geodesic icospheres (request r: seed 1005+r, r < %d; "
                    "%d..%d edges) into resident 512^3 grids" % (n_requests, min(edges), max(edges)),
        "requests_per_rate": n_requests,
        "admission_budget_bytes": budget,
        "upload": "segments as int16 over PCIe (coordinates < 512), widened to int32 on the device",
        "upload_bytes_total": int(sum(p.numel() * p.element_size() for p in pinned)),
        "batch_workspace_bytes": int(ex.work.numel()),
        "saturation": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in sat.items()},
        "poisson_sweep": sweep,
    }


def host_cpu() -> dict:
    """CPU model and core counts of this host."""
    model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "nproc": usable, "logical_cpus": os.cpu_count()}


class _one_core:
    """Pins this process to one of its cores for the duration."""

    def __enter__(self):
        self.prev = None
        try:
            self.prev = os.sched_getaffinity(0)
            core = sorted(self.prev)[-1]
            os.sched_setaffinity(0, {core})
            self.core = core
        except (AttributeError, OSError):
            self.core = None
        return self

    def __exit__(self, *exc):
        if self.prev is not None:
            os.sched_setaffinity(0, self.prev)


def cpu_baseline(segs_np, dims, seconds_target=15.0):
    """The oracle (gcc -O2 -march=native, single-threaded, pinned to one
    core) on the first segments of the workload (bounded sample)."""
    from oracle import oracle
    o = oracle.native()
    with _one_core() as pin:
        # Calibrate on a small prefix, then run the sample once.
        probe = segs_np[:20000]
        t = time.perf_counter()
        o.grid(probe, dims)
        dt = time.perf_counter() - t
        per_seg = max(dt / probe.shape[0], 1e-9)
        m = int(min(segs_np.shape[0], max(50000, seconds_target / per_seg)))
        sample = segs_np[:m]
        vox = int((np.abs(sample[:, 3:].astype(np.int64) - sample[:, :3]).max(1) + 1).sum())
        t = time.perf_counter()
        o.grid(sample, dims)
        dt = time.perf_counter() - t
    return {
        "value": vox / dt, "unit": "voxels/s", "cores": 1, "kind": "oracle",
        "sample": "first %d of %d segments (%d voxels) into the cleared %dx%dx%d volume, "
                  "clear included; %.1f s" % (m, segs_np.shape[0], vox, dims[0], dims[1],
                                                dims[2], dt),
        "build": "gcc -O2 -march=native, single-threaded",
        "pinned_core": pin.core,
        "host_cpu": host_cpu(),
    }


def cpu_baseline_other(workloads):
    """The oracle beside the other workloads of "extra", each on a bounded
    sample (about a second or two): voxels per second on one core."""
    from oracle import oracle
    o = oracle.native()

    def rate(fn, segs, voxels):
        t = time.perf_counter()
        fn(segs)
        dt = time.perf_counter() - t
        return {"voxels_per_s": voxels / dt, "seconds": round(dt, 3)}

    out = {}
    fixed_all = workloads.fixed_length()["segs"]
    offs = o.offsets(fixed_all)
    out["list"] = dict(rate(o.voxel_list, fixed_all, int(offs[-1])), sample="all 1048576 fixed-length segments")
    fixed = fixed_all[:100_000]
    offs = o.offsets_euclid(fixed)
    out["list_euclid"] = dict(rate(o.voxel_list_euclid, fixed, int(offs[-1])),
                              sample="first 100000 fixed-length segments, Euclidean N")
    c = workloads.arbitrary_length(n=100_000, volume=512)
    vox = int(np.sum(np.diff(o.offsets_euclid(c["segs"]))))
    out["grid_euclid"] = dict(rate(lambda s: o.grid_euclid(s, c["dims"]), c["segs"], vox),
                              sample="the 100000-segment 512^3 Euclidean grid workload, clear included")
    one = workloads.paper_segments([10 ** 6])["segs"]
    out["paper_single_segment_1e6"] = dict(rate(o.voxel_list32, one, 10 ** 6),
                                           sample="the 10^6-voxel segment as int32 rows")
    f = workloads.paper_segments([20000] * 1024, seed=90 + 20000)["segs"]
    out["paper_fixed_1024x20000"] = dict(rate(o.voxel_list32, f, 1024 * 20000),
                                         sample="1024 x 20000 voxels as int32 rows")
    return out


ONLY_WORKLOADS = ("list", "list_euclid", "grid_euclid", "paper_shapes", "small", "batch", "serving")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuning (profiler runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one 1 GiB device copy (counter calibration)")
    ap.add_argument("--only", default="",
                    help="comma-separated extra workloads to run alone, for profiler runs (list, list_euclid, "
                         "grid_euclid, paper_shapes, small, batch, serving): no main workload, no CPU "
                         "baseline; prints {\"only\": {name: result}}")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs on a single MI355X and has "
              "no multi-GPU path (sharding is described, not implemented); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    only = [x for x in args.only.split(",") if x]
    unknown = [x for x in only if x not in ONLY_WORKLOADS]
    if unknown:
        print("unknown workload(s) for --only: %s" % ", ".join(unknown), file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2009_09500_amd import binding, workloads

    binding.load()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)

    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    if args.only:
        runs = {
            "list": lambda: bench_list(args, torch, binding, workloads, dev, stream),
            "list_euclid": lambda: bench_list(args, torch, binding, workloads, dev, stream, euclid=True),
            "grid_euclid": lambda: bench_grid_euclid(args, torch, binding, workloads, dev, stream),
            "paper_shapes": lambda: bench_paper(args, torch, binding, workloads, dev, stream),
            "small": lambda: bench_small(args, torch, binding, workloads, dev, stream),
            "batch": lambda: bench_batch(args, torch, binding, workloads, dev, stream),
            "serving": lambda: bench_serving(args, torch, binding, workloads, dev),
        }
        names = [x for x in args.only.split(",") if x]
        print(json.dumps({"only": {x: runs[x]() for x in names}}))
        return

    r = bench_grid(args, torch, binding, workloads, dev, stream)
    ms_step = r["ms_total"] / args.steps
    value = r["voxels"] / (ms_step * 1e-3)
    prof = r["prof"]
    dom = max(prof.items(), key=lambda kv: kv[1][0]) if prof else ("", (0.0, 1))
    dom_name, (dom_ms, dom_launches) = dom
    dom_avg_ms = dom_ms / max(dom_launches, 1)
    sources = BRICK_SOURCES
    # Algorithmic bytes the dominant kernel must move per launch.
    # brick_fill writes the volume once (the clear is fused); grid_direct
    # reads the segments, writes the counts and sets the volume's words.
    dom_algo = {"brick_fill": r["grid_bytes"],
                "grid_direct": 24 * r["n"] + 4 * r["n"] + r["grid_bytes"]}.get(
        dom_name, r["algo_bytes"])
    achieved = dom_algo / (dom_avg_ms * 1e-3) / 1e9 if dom_avg_ms > 0 else 0.0
    traffic = counter_traffic(dom_name, "arbitrary4m", sources)
    bound = counter_bound(dom_name, "arbitrary4m", sources, dom_avg_ms, traffic)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": "arbitrary-length: 4194304 segments (seed 1003), start uniform in "
                        "[0,2048)^3, log-uniform length clipped to the volume -> cleared "
                        "2048^3 packed bit-volume + per-segment counts",
            "segments": r["n"], "voxels": r["voxels"], "volume": list(r["dims"]),
            "parallelism": "single GPU",
            "tuning": r["tuning"],
            "workspace_bytes": r["workspace_bytes"],
            "piece_records": r["piece_records"],
        },
        "hbm_gbs_algorithmic": r["algo_bytes"] / (ms_step * 1e-3) / 1e9,
        # The whole step (all kernels) on its algorithmic bytes.
        "hbm_frac_algorithmic": r["algo_bytes"] / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "algorithmic_bytes_per_step": r["algo_bytes"],
        "kernels_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in prof.items()},
        "roofline": _roofline_line(dom_name, dom_algo, achieved, dom_avg_ms, traffic, bound, r["voxels"]),
    }
    if not args.no_extra:
        line["extra"] = {
            "list": bench_list(args, torch, binding, workloads, dev, stream),
            "list_euclid": bench_list(args, torch, binding, workloads, dev, stream, euclid=True),
            "grid_euclid": bench_grid_euclid(args, torch, binding, workloads, dev, stream),
            "paper_shapes": bench_paper(args, torch, binding, workloads, dev, stream),
            "small": bench_small(args, torch, binding, workloads, dev, stream),
            "batch": bench_batch(args, torch, binding, workloads, dev, stream),
        }
        if not args.no_serving:
            line["extra"]["serving"] = bench_serving(args, torch, binding, workloads, dev)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(r["segs_np"], r["dims"])
        if not args.no_extra:
            with _one_core():
                line["cpu_baseline"]["other_workloads"] = cpu_baseline_other(workloads)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
