#!/usr/bin/env python3
"""Benchmark of the lightcuts-learning hot path on one GPU.

One step is one whole rendering pass over the static workload (65,536
clustered emissive triangles, the 2,073,600 primary hits of a 1920x1080
camera in a box room, 4,096 box occluders in a 64^3 grid, 64^3 hashed cells,
cut size 64, 1 spp): the fused sample + shadow + learn kernel over every
point, then the end-of-pass adaptation of every touched cell.  Inputs are
resident in HBM before timing starts; the timed steps are passes 0..K-1 of a
fresh cell table (after W untimed warm-up passes and a reset).

Prints ONE JSON line.  Extra fields:
  roofline      - the fused kernel against HBM bandwidth: algorithmic bytes
                  per launch (see algorithmic_bytes) over its mean duration,
                  timed with HIP events on the library's stream;
  cpu_baseline  - the CPU oracle (single-threaded C) on a bounded sample of
                  the same workload: every 10th point, for the same passes.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "light samples/s (sample+shadow+learn) and MSE vs oracle at equal GPU time"
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_frame_static.json")
KERNEL_SOURCES = ("paper_1911_10217_amd/csrc/frame.hip", "paper_1911_10217_amd/csrc/rlc_internal.h")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(samples: int, spp: int, M: int, cells: int, bins: int) -> dict:
    """Bytes the method must move per pass (the per-point tables it avoids are
    not counted):
      fused kernel: per point position + normal (24 B), per sample one 64 B
        emitter record, per point the radiance write (12 B); per touched
        cell its cut table (C, Q~, end: 12 M B); per touched (cell, cluster)
        bin its reward sum and count (12 B);
      adapt kernel: per touched cell 56 M B (read cnt, sum, Q, node; write
        node, end, Q, Q~, C; clear sum, cnt)."""
    points = samples // spp
    fused = 24 * points + 64 * samples + 12 * points + 12 * M * cells + 12 * bins
    adapt = 56 * M * cells
    return dict(fused=fused, adapt=adapt)


def _pmc_rows(path):
    import csv
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _per_kernel(rows, counter):
    """Mean counter value (KiB per dispatch, summed over the dispatch's
    entries) for the fused kernel and for the calibration copy kernel."""
    per_dispatch = {}
    for r in rows:
        if r.get("Counter_Name", r.get("counter_name")) != counter:
            continue
        name = r.get("Kernel_Name", r.get("kernel_name", ""))
        did = r.get("Dispatch_Id", r.get("dispatch_id"))
        val = float(r.get("Counter_Value", r.get("counter_value", 0.0)))
        key = (name, did)
        per_dispatch[key] = per_dispatch.get(key, 0.0) + val
    frame, copy = [], []
    for (name, _), v in per_dispatch.items():
        if "k_frame" in name:
            frame.append(v)
        elif "copy" in name.lower() or "elementwise" in name.lower():
            copy.append(v)
    return frame, copy


def write_traffic(fetch_csv, write_csv, copy_mib):
    ff, fc = _per_kernel(_pmc_rows(fetch_csv), "FETCH_SIZE")
    wf, wc = _per_kernel(_pmc_rows(write_csv), "WRITE_SIZE")
    if not ff or not wf or not fc or not wc:
        raise SystemExit("counters for the fused kernel or the copy kernel are missing")
    copy_kib = copy_mib * 1024.0
    fetch_scale = copy_kib / max(fc)
    write_scale = copy_kib / max(wc)
    fetch = sum(ff) / len(ff) * fetch_scale * 1024.0
    write = sum(wf) / len(wf) * write_scale * 1024.0
    out = {
        "kernel": "k_frame",
        "kernel_source_hash": kernel_source_hash(),
        "fetch_bytes_per_launch": round(fetch),
        "write_bytes_per_launch": round(write),
        "bytes_per_launch": round(fetch + write),
        "copy_calibration": {"mib": copy_mib, "fetch_kib_read": max(fc), "write_kib_read": max(wc),
                             "fetch_scale": fetch_scale, "write_scale": write_scale},
        "launches": [len(ff), len(wf)],
    }
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=32)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="static", choices=("static", "dynamic"),
                    help="static: the headline workload; dynamic: animated lights in walled compartments")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-stride", type=int, default=10, help="CPU baseline runs every n-th point")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 --pmc counter collections (FETCH_SIZE, WRITE_SIZE) of "
                         "a run with --copy-calib-mib into the fused kernel's HBM bytes per launch")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(*args.write_traffic, copy_mib=args.copy_calib_mib or 256)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the hot path runs on one device, and multi-GPU "
              "sharding is not part of this build (requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world),
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1911_10217_amd import rlc, scenes

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    print("[bench] generating the %s workload" % args.workload, file=sys.stderr, flush=True)
    s = scenes.make_static() if args.workload == "static" else scenes.make_dynamic()
    p = dict(s.params, occ_grid_res=64)
    spp = int(p["spp"])
    P = s.P
    samples_per_step = P * spp

    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    tri, emit, boxes, pos, nrm = t(s.tri), t(s.emit), t(s.boxes), t(s.pos), t(s.nrm)
    radiance = torch.empty((P, 3), dtype=torch.float32, device=dev)
    ctx = rlc.Context(p)
    ctx.rlc_build_light_tree(tri, emit)
    ctx.rlc_set_occluders(boxes)

    if args.copy_calib_mib:
        n = args.copy_calib_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # animated lights: every pass's emission is resident on the device and
    # set by rlc_set_emission inside the timed pass
    emissions = None
    if s.emission_at is not None:
        emissions = [t(s.emission_at(f)) for f in range(max(args.steps, args.warmup) + 1)]

    def one_pass(f):
        if emissions is not None:
            ctx.rlc_set_emission(emissions[f])
        ctx.rlc_frame(pos, nrm, spp, f, radiance)

    print("[bench] warm-up: %d passes" % args.warmup, file=sys.stderr, flush=True)
    for f in range(args.warmup):
        one_pass(f)
    ctx.rlc_sync()

    # ---- timed: passes 0..K-1 from a fresh cell table ----
    ctx.rlc_reset_cells()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for f in range(args.steps):
        one_pass(f)
    stop.record()
    torch.cuda.synchronize()
    ctx.rlc_sync()
    total_ms = start.elapsed_time(stop)
    ms_per_step = total_ms / args.steps
    value = samples_per_step * args.steps / (total_ms * 1e-3)
    print("[bench] %d passes in %.3f ms" % (args.steps, total_ms), file=sys.stderr, flush=True)

    # ---- per-kernel durations (HIP events around each launch) ----
    ctx.rlc_reset_cells()
    ctx.rlc_set_timing(True)
    for f in range(args.steps):
        one_pass(f)
    fused_ms, adapt_ms, nframes = ctx.rlc_get_timing()
    ctx.rlc_set_timing(False)
    fused_avg_ms = fused_ms / max(nframes, 1)
    adapt_avg_ms = adapt_ms / max(nframes, 1)

    # ---- touched cells and (cell, cluster) bins of one steady-state pass ----
    smp = ctx.rlc_sample(pos, nrm, spp, args.steps)
    _, _, reward = ctx.rlc_shade(pos, nrm, spp, smp, contrib=False)
    ctx.rlc_learn(smp, reward)
    dump = ctx.rlc_dump_cells()
    cnt = dump["cnt"]
    cells_t = int((cnt.sum(axis=1) > 0).sum())
    bins_t = int((cnt > 0).sum())
    M = ctx.rlc_meff()
    alg = algorithmic_bytes(samples_per_step, spp, M, cells_t, bins_t)
    achieved = alg["fused"] / (fused_avg_ms * 1e-3) / 1e9

    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_source_hash") == kernel_source_hash():
            traffic = tr.get("bytes_per_launch")

    roofline = {
        "bound": "hbm",
        "achieved": round(achieved, 2),
        "peak": PEAK_HBM_GBS,
        "unit": "GB/s",
        "frac": round(achieved / PEAK_HBM_GBS, 4),
        "traffic": traffic,
        "kernel": "k_frame (fused sample+shadow+learn)",
        "alg_bytes_per_launch": alg["fused"],
        "kernel_ms": round(fused_avg_ms, 4),
        "adapt_kernel_ms": round(adapt_avg_ms, 4),
        "adapt_alg_bytes_per_launch": alg["adapt"],
        "cells_touched": cells_t,
        "bins_touched": bins_t,
    }

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        sel = np.arange(0, P, args.cpu_stride, dtype=np.uint32)
        orc = oracle.Oracle(p, s.tri, s.emit, s.boxes)
        print("[bench] CPU oracle: %d points x %d passes" % (sel.size, args.steps), file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        for f in range(args.steps):
            if s.emission_at is not None:
                orc.set_emission(s.emission_at(f))
            orc.frame(s.pos[sel], s.nrm[sel], spp, f, pid=sel)
            orc.adapt()
        dt = time.perf_counter() - t0
        cpu = {"value": round(sel.size * spp * args.steps / dt, 1), "unit": "samples/s", "cores": 1,
               "kind": "oracle",
               "sample": "every %dth point (%d of %d) for the same %d passes, single-threaded C oracle, %.1f s"
                         % (args.cpu_stride, sel.size, P, args.steps, dt)}

    if args.workload == "static":
        workload = ("static: 65,536 emissive triangles in 256 clusters, 2,073,600 primary hits "
                    "(1920x1080, in 16x16 pixel tiles), 4,096 box occluders in a 64^3 grid, 64^3 hashed "
                    "cells, cut size 64, 1 spp, passes from a fresh cell table")
    else:
        workload = ("dynamic: 1,048,576 emissive triangles in 16 walled compartments, emission "
                    "Le (1 + sin(2 pi f t + phi)) per compartment set every pass, 1,048,576 points, "
                    "16,384 wall bricks in a 64^3 grid, 64^3 hashed cells, cut size 64, 1 spp, "
                    "temporal adaptation, passes from a fresh cell table")
    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": workload,
            "samples_per_step": samples_per_step,
            "parallelism": "1 GPU",
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
