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
  cpu_baseline  - the CPU oracle (plain single-threaded C) on bounded samples
                  of the same workload, whole cells at a time (all points of
                  every k-th touched cell, so each sampled cell sees the GPU
                  run's sample density), for the same passes: on one core,
                  and on a pool of worker processes over disjoint cell sets
                  (cells learn independently, so the results are the same);
  mse           - the image error the learning buys at equal GPU time: the
                  method against the same passes with learning switched off
                  (temporal = 0, every pass from the initial cut), both
                  against a 1,024-pass mean at independent frame numbers.
"""
from __future__ import annotations

import argparse
import csv
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
VALU_FILE = os.path.join(ROOT, "profiles", "valu_frame_static.json")
KERNEL_SOURCES = ("paper_1911_10217_amd/csrc/frame.hip", "paper_1911_10217_amd/csrc/rlc_internal.h",
                  "paper_1911_10217_amd/csrc/occ_trace.h", "paper_1911_10217_amd/csrc/occ.hip")


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


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_worker(job):
    """One process of the CPU baseline's pool: the oracle over the points of
    its cells for every pass; returns the seconds the passes took."""
    import oracle
    params, tri, emit, boxes, pos, nrm, pid, spp, passes = job
    orc = oracle.Oracle(params, tri, emit, boxes)
    t0 = time.perf_counter()
    for f in range(passes):
        orc.frame(pos, nrm, spp, f, pid=pid)
        orc.adapt()
    return time.perf_counter() - t0


def _cell_sample(np, keys, stride):
    """Points of every stride-th distinct cell key (in key order), and the
    cell of each selected point."""
    uniq, inv = np.unique(keys, return_inverse=True)
    take = np.zeros(uniq.size, bool)
    take[::stride] = True
    sel = np.nonzero(take[inv])[0].astype(np.uint32)
    return sel, inv[sel], int(take.sum())


def cpu_baseline(np, p, s, spp, passes, stride1, strideN, workers):
    """The oracle on whole sampled cells: one core, then a pool of worker
    processes (spawned, so they hold no GPU state) over disjoint cell sets
    balanced by point count."""
    import multiprocessing as mp

    import oracle
    keys = oracle.Oracle(p, s.tri[:1], s.emit[:1]).cell_keys(s.pos)
    sel, _, ncell = _cell_sample(np, keys, stride1)
    orc = oracle.Oracle(p, s.tri, s.emit, s.boxes)
    print("[bench] CPU oracle, 1 core: %d points in %d cells x %d passes" % (sel.size, ncell, passes),
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for f in range(passes):
        orc.frame(s.pos[sel], s.nrm[sel], spp, f, pid=sel)
        orc.adapt()
    dt1 = time.perf_counter() - t0
    one = {"value": round(sel.size * spp * passes / dt1, 1), "unit": "samples/s", "cores": 1,
           "sample": "all %d points of every %dth touched cell (%d cells), %d passes, %.1f s"
                     % (sel.size, stride1, ncell, passes, dt1)}
    selN, cellN, ncellN = _cell_sample(np, keys, strideN)
    # cells to workers, largest first onto the least-loaded worker
    cells, counts = np.unique(cellN, return_counts=True)
    load = np.zeros(workers, np.int64)
    owner = {}
    for c in cells[np.argsort(-counts, kind="stable")]:
        w = int(np.argmin(load))
        owner[int(c)] = w
        load[w] += int(counts[np.searchsorted(cells, c)])
    wid = np.array([owner[int(c)] for c in cellN])
    jobs = []
    for w in range(workers):
        ids = selN[wid == w]
        if ids.size:
            jobs.append((p, s.tri, s.emit, s.boxes, s.pos[ids], s.nrm[ids], ids, spp, passes))
    print("[bench] CPU oracle, %d processes: %d points in %d cells x %d passes"
          % (len(jobs), selN.size, ncellN, passes), file=sys.stderr, flush=True)
    ctx = mp.get_context("spawn")
    with ctx.Pool(len(jobs)) as pool:
        pool.map(abs, range(len(jobs)))  # start the workers before timing
        t0 = time.perf_counter()
        per = pool.map(_cpu_worker, jobs)
        dtN = time.perf_counter() - t0
    return {"value": round(selN.size * spp * passes / dtN, 1), "unit": "samples/s", "cores": len(jobs),
            "kind": "oracle",
            "sample": "all %d points of every %dth touched cell (%d cells), %d passes, %d worker processes "
                      "over disjoint cell sets, %.1f s wall (slowest worker %.1f s)"
                      % (selN.size, strideN, ncellN, passes, len(jobs), dtN, max(per)),
            "single_core": one, "host_cpus": os.cpu_count(), "cpu_model": cpu_model()}


def mse_equal_time(np, torch, ctx, make_ctx, p, pos, nrm, spp, passes, budget_ms, P):
    """Image error at equal GPU time, in FP64 on the GPU, against the mean of
    1,024 passes of the method at frame numbers 100000... (independent random
    numbers): the method's mean over `passes` passes from a fresh cell table
    (the workload's reward reading, and the cluster-total reading), and the
    mean of as many passes with learning switched off (temporal = 0, every
    pass from the initial cut) as fit in the method's GPU time.  Besides the
    MSE over all pixel values, the MSE without the 0.1% largest squared
    errors: a few pixels whose cell gives a visible light a tiny probability
    carry most of the all-pixel MSE."""
    dev = pos.device
    rad = torch.empty((P, 3), dtype=torch.float32, device=dev)

    def mean_of(c, frames):
        acc = torch.zeros((P, 3), dtype=torch.float64, device=dev)
        for f in frames:
            c.rlc_frame(pos, nrm, spp, f, rad)
            acc += rad
        return (acc / len(frames)).float()

    def timed_ms(c):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c.rlc_reset_cells()
        e0.record()
        for f in range(passes):
            c.rlc_frame(pos, nrm, spp, f, rad)
        e1.record()
        torch.cuda.synchronize()
        c.rlc_reset_cells()
        return e0.elapsed_time(e1)

    print("[bench] MSE: reference of 1,024 passes", file=sys.stderr, flush=True)
    ref_ctx = make_ctx(p)
    ref = mean_of(ref_ctx, range(100000, 101024))
    ref_ctx.close()

    def errors(img):
        se = ((img.double() - ref.double()) ** 2).reshape(-1)
        k = max(1, int(se.numel() * 0.001))
        top = torch.topk(se, k).values.sum()
        return {"mse": float(ctx.rlc_image_error(img, ref)[2]),
                "mse_without_top_0.1pct": float((se.sum() - top) / (se.numel() - k))}

    out = {"budget_ms": round(budget_ms, 3), "reference": "mean of 1,024 passes of the method at frames 100000..101023"}
    ctx.rlc_reset_cells()
    out["learned"] = dict(errors(mean_of(ctx, range(passes))), passes=passes, reward=int(p["reward_mode"]))
    other = 1 - int(p["reward_mode"])
    c1 = make_ctx(dict(p, reward_mode=other))
    n1 = max(1, int(budget_ms / (timed_ms(c1) / passes)))
    out["learned_other_reward"] = dict(errors(mean_of(c1, range(n1))), passes=n1, reward=other)
    c1.close()
    off = make_ctx(dict(p, temporal=0))
    n_off = max(1, int(budget_ms / (timed_ms(off) / passes)))
    out["no_learning"] = dict(errors(mean_of(off, range(n_off))), passes=n_off)
    off.close()
    out["ratio_no_learning_over_learned"] = round(out["no_learning"]["mse"] / out["learned"]["mse"], 3)
    return out


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

def _sum_counters(path, names):
    """Per-dispatch sums of the given counters over the fused kernel's
    dispatches: {counter: mean over dispatches}."""
    per = {}
    for r in _pmc_rows(path):
        name = r.get("Kernel_Name", r.get("kernel_name", ""))
        if "k_frame" not in name:
            continue
        cn = r.get("Counter_Name", r.get("counter_name"))
        if cn not in names:
            continue
        did = r.get("Dispatch_Id", r.get("dispatch_id"))
        per.setdefault(cn, {}).setdefault(did, 0.0)
        per[cn][did] += float(r.get("Counter_Value", r.get("counter_value", 0.0)))
    return {k: sum(v.values()) / len(v) for k, v in per.items()}


SIMDS = 1024           # 256 CUs x 4 SIMDs
CLOCK_HZ = 2.4e9       # peak engine clock
VALU_ISSUE_CYCLES = 4  # a wave64 VALU instruction on a 16-lane SIMD


def _mean_kernel_ns(stats_csv, name):
    with open(stats_csv) as f:
        for r in csv.DictReader(f):
            if name in r["Name"]:
                return float(r["AverageNs"])
    raise SystemExit("no %s in %s" % (name, stats_csv))


def write_valu(valu_csv, wait_csv, stats_csv):
    """VALU issue and waits of the fused kernel from two counter collections
    and the kernel trace of the same configuration (see
    profiles/k_frame_static_valu_counters.md): the lanes' share of VALU work,
    the SIMDs' VALU issue time over the kernel's mean duration, and their
    product, the useful-lane fraction of the chip's VALU issue capacity."""
    a = _sum_counters(valu_csv, {"SQ_ACTIVE_INST_VALU", "SQ_THREAD_CYCLES_VALU", "SQ_WAVES", "SQ_WAVE_CYCLES",
                                 "SQ_INSTS_VALU", "SQ_INSTS_SALU"})
    b = _sum_counters(wait_csv, {"SQ_WAIT_ANY", "SQ_WAVE_CYCLES"})
    waves = a["SQ_WAVES"]
    lane_util = a["SQ_THREAD_CYCLES_VALU"] / (64.0 * a["SQ_ACTIVE_INST_VALU"])
    # VALU instructions issued per SIMD, 4 cycles each, over the kernel's
    # mean duration at the peak clock
    kernel_ns = _mean_kernel_ns(stats_csv, "k_frame")
    simd_busy = a["SQ_ACTIVE_INST_VALU"] * VALU_ISSUE_CYCLES / SIMDS / (kernel_ns * 1e-9 * CLOCK_HZ)
    out = {"kernel": "k_frame", "kernel_source_hash": kernel_source_hash(),
           "valu_insts_per_wave": round(a["SQ_INSTS_VALU"] / waves, 1),
           "salu_insts_per_wave": round(a["SQ_INSTS_SALU"] / waves, 1),
           "lane_utilisation": round(lane_util, 4), "simd_valu_busy": round(simd_busy, 4),
           "useful_lane_valu_frac": round(lane_util * simd_busy, 4), "kernel_ns": round(kernel_ns, 1),
           "wait_any_frac": round(b["SQ_WAIT_ANY"] / b["SQ_WAVE_CYCLES"], 4)}
    with open(VALU_FILE, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


MLP_FLOP_PER_TUPLE = 2 * (144 * 64 + 3 * 64 * 64) + 2 * 3 * 64 * 64 + 2 * (144 * 64 + 3 * 64 * 64)
PEAK_BF16_TFLOPS = 2500.0
LEARNED_TRUTH = os.path.join(ROOT, "tests", "golden", "learned_truth.txt")


def run_learned(args, np, torch, rlc, scenes, dev):
    """The learned proposal against the plain method at equal GPU time.

    Workload: the tiny scene (1,024 emissive triangles, 4,096 points, 64 box
    occluders, 8^3 cells, cut size 16, 16 spp per pass).  Plain: passes of
    the method from a fresh cell table.  Learned: 8 passes of the method that
    log (point, fixed-cut node, weight) for every sample; training of the MLP
    (epochs x minibatch Adam over the 524,288 logged tuples) in a second
    context on a side stream, while passes of the method go on in the first
    (as many as a trial run shows end before the training does); the trained
    weights taken over without a host synchronisation, one forward pass for
    the per-point cdf, then passes that draw from the 50/50 mixture.  The
    same with training first and rendering after is reported beside it.  A
    GPU-time budget is the plain method's time for n passes; each form's
    image is the mean of the passes that end within it.  MSE against the
    FP64 oracle truth at every 16th point (a stored table written by the
    oracle).  All times are HIP events, training included."""
    s = scenes.make_tiny()
    p = dict(s.params)
    spp = int(p["spp"])
    P = s.P
    log_passes = 8
    budgets = [int(x) for x in args.budgets.split(",")]
    nmax = max(budgets)
    truth = np.loadtxt(LEARNED_TRUTH)
    ref_pid = truth[:, 0].astype(np.int64)
    ref = truth[:, 1:]

    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    pos, nrm = t(s.pos), t(s.nrm)
    ctx = rlc.Context(p)
    ctx.rlc_build_light_tree(t(s.tri), t(s.emit))
    ctx.rlc_set_occluders(t(s.boxes))
    rad = torch.empty((nmax, P, 3), dtype=torch.float32, device=dev)
    n_log = log_passes * P * spp
    lp = torch.empty(n_log, dtype=torch.int32, device=dev)
    ln = torch.empty(n_log, dtype=torch.int32, device=dev)
    lw = torch.empty(n_log, dtype=torch.float32, device=dev)
    cdf = torch.empty((P, 64), dtype=torch.float32, device=dev)

    def events(n):
        return [torch.cuda.Event(enable_timing=True) for _ in range(n)]

    # points inside the emitter band (y >= 0.9) can lie arbitrarily close to
    # a triangle: their estimates are heavy-tailed, so the MSE is also given
    # over the points below the band
    below = s.pos[ref_pid, 1] < 0.9

    def mse_curve(frames):
        img = rad[:frames, ref_pid].double().cpu().numpy()
        mean = np.cumsum(img, axis=0) / np.arange(1, frames + 1)[:, None, None]
        err = (mean - ref[None]) ** 2
        return err.mean(axis=(1, 2)), err[:, below].mean(axis=(1, 2))

    # warm-up of every kernel involved, then a fresh state
    print("[bench] learned: warm-up", file=sys.stderr, flush=True)
    for f in range(2):
        ctx.rlc_frame(pos, nrm, spp, f, rad[f])
    ctx.rlc_mlp_init(p["seed"])
    # the warm-up trains on as many tuples as the timed call, so that the
    # library's training buffers are sized before the timed region (the
    # tuples past the first logged pass are zero: weight 0)
    lp.zero_()
    ln.zero_()
    lw.zero_()
    ctx.rlc_set_sample_log(lp[:P * spp], ln[:P * spp], lw[:P * spp])
    ctx.rlc_frame(pos, nrm, spp, 0, rad[0])
    ctx.rlc_set_sample_log()
    ctx.rlc_mlp_train(pos, nrm, lp, ln, lw, 1, args.mlp_batch, args.mlp_lr)
    ctx.rlc_mlp_forward(pos, nrm, cdf=cdf)
    ctx.rlc_set_mixture(cdf, 0.5)
    ctx.rlc_frame(pos, nrm, spp, 1, rad[1])
    ctx.rlc_set_mixture()
    torch.cuda.synchronize()

    # ---- plain: nmax passes, an event after each ----
    ctx.rlc_reset_cells()
    ev = events(nmax + 1)
    torch.cuda.synchronize()
    ev[0].record()
    for f in range(nmax):
        ctx.rlc_frame(pos, nrm, spp, f, rad[f])
        ev[f + 1].record()
    torch.cuda.synchronize()
    plain_t = np.array([ev[0].elapsed_time(e) for e in ev[1:]])
    plain_mse, plain_mse_b = mse_curve(nmax)

    # ---- learned: log, train, forward, mixture passes ----
    # Training runs in a second context on a side stream (default priority),
    # fed by the logged tuples: the training kernels occupy half of the
    # compute units, so the method's passes go on beside them until the
    # network is trained; the rendering context then takes the weights
    # (rlc_mlp_copy_params joins the streams) and switches to the mixture.
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        trainer = rlc.Context(p)
        trainer.rlc_build_light_tree(t(s.tri), t(s.emit))
        trainer.rlc_set_occluders(t(s.boxes))
    torch.cuda.synchronize()
    k_mix = nmax

    def learned_run(k_ov, passes=k_mix):
        """k_ov None: train on the rendering context's stream, then render;
        otherwise k_ov passes of the method beside the training."""
        ctx.rlc_reset_cells()
        ctx.rlc_mlp_init(p["seed"])
        trainer.rlc_mlp_init(p["seed"])
        ev = events(passes + 1)
        ev_train, ev_fwd = events(2)
        torch.cuda.synchronize()
        ev[0].record()
        for f in range(log_passes):
            sl = slice(f * P * spp, (f + 1) * P * spp)
            ctx.rlc_set_sample_log(lp[sl], ln[sl], lw[sl])
            ctx.rlc_frame(pos, nrm, spp, f, rad[f])
            ev[f + 1].record()
        ctx.rlc_set_sample_log()
        done = log_passes
        if k_ov is None:
            ctx.rlc_mlp_train(pos, nrm, lp, ln, lw, args.mlp_epochs, args.mlp_batch, args.mlp_lr, sync=False)
            ev_train.record()
        else:
            side.wait_event(ev[log_passes])
            trainer.rlc_mlp_train(pos, nrm, lp, ln, lw, args.mlp_epochs, args.mlp_batch, args.mlp_lr, sync=False)
            ev_train.record(side)
            for f in range(log_passes, min(log_passes + k_ov, passes)):
                ctx.rlc_frame(pos, nrm, spp, f, rad[f])
                ev[f + 1].record()
                done = f + 1
            ctx.rlc_mlp_copy_params(trainer)
        if done < passes:
            ctx.rlc_mlp_forward(pos, nrm, cdf=cdf)
            ctx.rlc_set_mixture(cdf, 0.5)
            ev_fwd.record()
            for f in range(done, passes):
                ctx.rlc_frame(pos, nrm, spp, f, rad[f])
                ev[f + 1].record()
        torch.cuda.synchronize()
        ctx.rlc_set_mixture()
        ctx.rlc_sync()
        trainer.rlc_sync()
        ends = np.array([ev[0].elapsed_time(e) for e in ev[1:]])
        out = {"ends": ends, "done": done, "t_log": ev[0].elapsed_time(ev[log_passes]),
               "t_train": ev[log_passes].elapsed_time(ev_train), "t_train_end": ev[0].elapsed_time(ev_train)}
        if done < passes:
            fwd_end = ev[0].elapsed_time(ev_fwd)
            out["t_fwd"] = fwd_end - max(ends[done - 1], out["t_train_end"])
            out["mix_ms"] = ev_fwd.elapsed_time(ev[passes])
            out["n_mix"] = passes - done
        return out

    # how many passes of the method fit beside the training: a trial run
    # with more than enough of them, counted by their end times
    trial = learned_run(256, passes=log_passes + 256)
    k_ov = int(np.sum(trial["ends"][log_passes:] <= trial["t_train_end"]))
    serial = learned_run(None)
    serial_mse, serial_mse_b = mse_curve(k_mix)
    lrun = learned_run(k_ov)
    learned_mse, learned_mse_b = mse_curve(k_mix)
    mix_t = lrun["ends"]
    t_log, t_train, t_fwd = lrun["t_log"], lrun["t_train"], lrun["t_fwd"]
    trainer.close()
    # per-kernel durations of the training steps, in a separate run with HIP
    # events around each launch (the same training from the same weights)
    ctx.rlc_mlp_init(p["seed"])
    ctx.rlc_set_timing(True)
    loss = ctx.rlc_mlp_train(pos, nrm, lp, ln, lw, args.mlp_epochs, args.mlp_batch, args.mlp_lr)
    ctx.rlc_set_timing(False)
    fb_ms, upd_ms, steps = ctx.rlc_get_mlp_timing()

    def serial_ratio(n):
        budget = float(plain_t[n - 1])
        fit = int(np.searchsorted(serial["ends"], budget, side="right"))
        return round(float(serial_mse[fit - 1] / plain_mse[n - 1]), 4) if fit >= 1 else None

    rows = []
    for n in budgets:
        budget = float(plain_t[n - 1])
        fit = int(np.searchsorted(mix_t, budget, side="right"))
        # every pass that ends within the budget counts: logged, beside the
        # training, mixture
        m = learned_mse[fit - 1] if fit >= 1 else float("nan")
        mb = learned_mse_b[fit - 1] if fit >= 1 else float("nan")
        rows.append({"budget_passes_plain": n, "budget_ms": round(budget, 4),
                     "plain_mse": float(plain_mse[n - 1]),
                     "learned_passes": fit, "learned_mse": float(m),
                     "ratio_learned_to_plain": round(float(m / plain_mse[n - 1]), 4) if fit >= 1 else None,
                     "plain_mse_below_band": float(plain_mse_b[n - 1]), "learned_mse_below_band": float(mb),
                     "ratio_below_band": round(float(mb / plain_mse_b[n - 1]), 4) if fit >= 1 else None,
                     "ratio_learned_to_plain_train_then_render": serial_ratio(n)})
    equal_samples = {"passes": nmax, "plain_mse": float(plain_mse[nmax - 1]),
                     "learned_mse": float(learned_mse[nmax - 1]),
                     "ratio_learned_to_plain": round(float(learned_mse[nmax - 1] / plain_mse[nmax - 1]), 4),
                     "plain_mse_below_band": float(plain_mse_b[nmax - 1]),
                     "learned_mse_below_band": float(learned_mse_b[nmax - 1]),
                     "ratio_below_band": round(float(learned_mse_b[nmax - 1] / plain_mse_b[nmax - 1]), 4)}

    mix_ms = lrun.get("mix_ms", 0.0)
    n_mix = lrun.get("n_mix", 0)
    value = P * spp * n_mix / (mix_ms * 1e-3) if mix_ms > 0 else 0.0
    fb_avg = fb_ms / max(steps, 1)
    flop = MLP_FLOP_PER_TUPLE * min(args.mlp_batch, n_log)
    achieved = flop / (fb_avg * 1e-3) / 1e12 if fb_avg > 0 else 0.0
    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": n_mix,
        "warmup": 2,
        "ms_per_step": round(mix_ms / max(n_mix, 1), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+bf16",
        "data": "synthetic",
        "config": {
            "workload": ("learned: tiny scene (1,024 emissive triangles, 4,096 points, 64 box occluders, "
                         "8^3 cells, cut size 16, 16 spp); 8 logged passes, MLP 144-64-64-64-64 trained "
                         "%d epochs (batch %d, lr %g) in a second context on a side stream while %d passes "
                         "of the method go on, then 50/50 mixture passes"
                         % (args.mlp_epochs, args.mlp_batch, args.mlp_lr, k_ov)),
            "samples_per_step": P * spp,
            "parallelism": "1 GPU",
        },
        "mse": {
            "reference": "FP64 oracle truth (12x12 strata per light, exact shadows) at every 16th point",
            "points": int(ref_pid.size), "points_below_band": int(below.sum()),
            "equal_gpu_time": rows,
            "equal_samples": equal_samples,
            "plain_ms_per_pass": round(float(plain_t[-1] / nmax), 4),
            "learned_ms": {"log_passes": round(t_log, 4), "train": round(t_train, 4),
                           "passes_beside_training": k_ov,
                           "forward": round(t_fwd, 4), "mixture_per_pass": round(mix_ms / max(n_mix, 1), 4),
                           "train_then_render": {"train": round(serial["t_train"], 4),
                                                 "forward": round(serial.get("t_fwd", 0.0), 4)}},
            "train_steps": steps,
            "train_last_loss": loss,
        },
        "roofline": {
            "bound": "mfma",
            "achieved": round(achieved, 3),
            "peak": PEAK_BF16_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_BF16_TFLOPS, 6),
            "traffic": None,
            "kernel": "k_mlp_fwd_bwd (forward + backward of one minibatch, BF16 MFMA)",
            "alg_flop_per_launch": flop,
            "kernel_ms": round(fb_avg, 4),
            "adam_ms": round(upd_ms / max(steps, 1), 4),
        },
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def run_batched(args, np, torch, rlc, scenes, dev):
    """Uneven scenes rendered by per-scene launches against one persistent,
    graph-captured batched launch, at equal GPU time.

    Workload: 16 static-style scenes with log-uniform sizes (emitters 4K-1M,
    points 64K-2M, occluders 64-16K, cut sizes 16/32/64), 1 spp, 16 passes.
    Plain: per pass, rlc_frame on every scene in turn (two launches each).
    Batched: the autotuned schedule, one graph launch per pass.  A pass of
    the batch gives exactly the images of the per-scene passes (a parity
    test), so at equal GPU time the batched form simply completes more
    passes.  MSE against a 1,024-pass mean of the method on other frame
    numbers (independent random numbers), over every pixel of every scene."""
    F = args.steps if args.steps else 16
    print("[bench] batched: generating 16 scenes", file=sys.stderr, flush=True)
    sc = scenes.make_batch(frames=F)
    st = torch.cuda.Stream()
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    with torch.cuda.stream(st):
        side = []
        for s in sc:
            ctx = rlc.Context(s.params)
            ctx.rlc_build_light_tree(t(s.tri), t(s.emit))
            ctx.rlc_set_occluders(t(s.boxes))
            side.append((ctx, t(s.pos), t(s.nrm), torch.empty((s.P, 3), dtype=torch.float32, device=dev)))
        samples = sum(s.P for s in sc)

        def reset():
            for c, _, _, _ in side:
                c.rlc_reset_cells()

        def plain_pass(f):
            for c, pos, nrm, rad in side:
                c.rlc_frame(pos, nrm, 1, f, rad)

        # ---- plain: per-scene launches ----
        plain_pass(0)
        reset()
        st.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for f in range(F):
            plain_pass(f)
        e1.record(st)
        st.synchronize()
        t_plain = e0.elapsed_time(e1)

        # ---- batched: autotune, then one graph launch per pass ----
        batch = rlc.Batch([(c, pos, nrm, 1) for c, pos, nrm, _ in side], st)
        print("[bench] batched: autotuning", file=sys.stderr, flush=True)
        best, cands = batch.rlc_batch_autotune(passes=2)
        reset()
        st.synchronize()
        e0.record(st)
        for f in range(F):
            batch.rlc_batch_frame(f)
        e1.record(st)
        st.synchronize()
        t_batch = e0.elapsed_time(e1)
        f_eq = int(F * t_plain / t_batch)

        # ---- MSE at equal GPU time (untimed replays; passes are deterministic) ----
        print("[bench] batched: reference and MSE replays", file=sys.stderr, flush=True)
        n_ref = 1024
        reset()
        ref = [torch.zeros((s.P, 3), dtype=torch.float64, device=dev) for s in sc]
        for j in range(n_ref):
            rads = batch.rlc_batch_frame(100000 + j)
            for r, x in zip(ref, rads):
                r += x
        for r in ref:
            r /= n_ref
        reset()
        acc = [torch.zeros((s.P, 3), dtype=torch.float64, device=dev) for s in sc]
        mse = {}
        for f in range(max(F, f_eq)):
            rads = batch.rlc_batch_frame(f)
            for a, x in zip(acc, rads):
                a += x
            if f + 1 in (F, f_eq):
                err = sum(float(((a / (f + 1) - r) ** 2).sum()) for a, r in zip(acc, ref))
                mse[f + 1] = err / (3.0 * samples)
        st.synchronize()
        batch.close()
        for c, _, _, _ in side:
            c.close()

    ms_pass = t_batch / F
    value = samples * F / (t_batch * 1e-3)
    alg = sum(24 * s.P + 64 * s.P + 12 * s.P for s in sc)
    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": F,
        "warmup": 2,
        "ms_per_step": round(ms_pass, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": ("batched: 16 static-style scenes, emitters log-uniform 4K-1M, points 64K-2M, "
                         "occluders 64-16K, cut sizes 16/32/64, 1 spp, %d passes; %d points per pass"
                         % (F, samples)),
            "samples_per_step": samples,
            "parallelism": "1 GPU",
            "schedule": best,
        },
        "batched_vs_plain": {
            "plain_ms_per_pass": round(t_plain / F, 4),
            "batched_ms_per_pass": round(ms_pass, 4),
            "speedup": round(t_plain / t_batch, 3),
            "plain_samples_per_s": round(samples * F / (t_plain * 1e-3), 1),
            "equal_gpu_time": {"budget_ms": round(t_plain, 4), "plain_passes": F, "batched_passes": f_eq,
                               "plain_mse": mse[F], "batched_mse": mse[f_eq],
                               "ratio_batched_to_plain": round(mse[f_eq] / mse[F], 4)},
            "reference": "mean of 1,024 passes of the method at frame numbers 100000..101023",
            "autotune_candidates": len(cands),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(alg / (ms_pass * 1e-3) / 1e9, 2),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(alg / (ms_pass * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
            "traffic": None,
            "kernel": "one batched pass (graph: k_batch_frame + k_batch_adapt)",
            "alg_bytes_per_launch": alg,
            "alg_bytes_note": "points, emitter records and radiance only; cell-table terms omitted (lower bound)",
        },
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)



def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=32)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="static", choices=("static", "dynamic", "learned", "batched"),
                    help="static: the headline workload; dynamic: animated lights in walled compartments; "
                         "learned: the tiny scene, plain method against the MLP mixture at equal GPU time; "
                         "batched: 16 uneven scenes, per-scene launches against one batched graph launch")
    ap.add_argument("--mlp-epochs", type=int, default=1)
    # 32,768 tuples per step give 256 training blocks, one per compute unit;
    # the rate follows the square-root rule for Adam from 0.01 at 16,384
    ap.add_argument("--mlp-batch", type=int, default=32768)
    ap.add_argument("--mlp-lr", type=float, default=0.014)
    ap.add_argument("--budgets", default="32,128,512,2048",
                    help="learned: GPU-time budgets, as the plain method's time for this many passes")
    ap.add_argument("--split-steps", type=int, default=1,
                    help="static/dynamic: split-collapse steps per pass (1: the basic algorithm; n > 1: "
                         "repeated until a step changes nothing, at most n times)")
    ap.add_argument("--normal-bits", type=int, default=0,
                    help="static/dynamic: 5-D cells with 2^n bins per octahedral normal coordinate")
    ap.add_argument("--jitter", type=float, default=0.0,
                    help="static/dynamic: jittered cell lookups (in cells and normal bins, 0..1)")
    ap.add_argument("--sub-frames", type=int, default=1,
                    help="static/dynamic: a step is one frame of this many passes (rlc_frame_sub), each "
                         "with the workload's samples per point")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-stride", type=int, default=40,
                    help="the one-core CPU baseline runs every n-th touched cell")
    ap.add_argument("--cpu-stride-pool", type=int, default=5,
                    help="the pooled CPU baseline runs every n-th touched cell")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="worker processes of the pooled CPU baseline (0: the host's CPUs, at most 16)")
    ap.add_argument("--no-mse", action="store_true")
    ap.add_argument("--footprint-tile", type=float, default=0.0,
                    help="footprint-sized cells: a primary hit's cell edge is wanted at this many times its "
                         "pixel footprint (0: the fixed 64^3 grid)")
    ap.add_argument("--footprint-levels", type=int, default=6)
    ap.add_argument("--max-cells", type=int, default=-1,
                    help="rows of the cell tables (-1: the workload's own; 0: one per lookup slot; "
                         "5-D cells default to 0)")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--write-valu", nargs=3, metavar=("VALU_CSV", "WAIT_CSV", "KERNEL_STATS_CSV"),
                    help="turn the two VALU / wait counter collections of the fused kernel into "
                         "profiles/valu_frame_static.json")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 --pmc counter collections (FETCH_SIZE, WRITE_SIZE) of "
                         "a run with --copy-calib-mib into the fused kernel's HBM bytes per launch")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(*args.write_traffic, copy_mib=args.copy_calib_mib or 256)
        return
    if args.write_valu:
        write_valu(*args.write_valu)
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
    if args.workload == "learned":
        run_learned(args, np, torch, rlc, scenes, dev)
        return
    if args.workload == "batched":
        run_batched(args, np, torch, rlc, scenes, dev)
        return

    print("[bench] generating the %s workload" % args.workload, file=sys.stderr, flush=True)
    s = scenes.make_static() if args.workload == "static" else scenes.make_dynamic()
    p = dict(s.params, occ_grid_res=64, split_steps=args.split_steps, normal_bits=args.normal_bits,
             jitter=args.jitter)
    if args.max_cells >= 0:
        p["max_cells"] = args.max_cells
    elif args.normal_bits > 0:
        p["max_cells"] = 0  # normal bins multiply the cells: one row per lookup slot
    if args.footprint_tile > 0:
        if s.footprint is None:
            raise SystemExit("--footprint-tile needs a workload with camera footprints (static)")
        p.update(footprint_levels=args.footprint_levels, footprint_tile=args.footprint_tile)
    spp = int(p["spp"])
    P = s.P
    n_sub = max(1, args.sub_frames)
    # the configuration the committed counter profiles were taken on
    profiled = (args.workload == "static" and args.split_steps <= 1 and args.normal_bits == 0
                and args.jitter == 0.0 and n_sub == 1 and args.footprint_tile == 0 and args.max_cells < 0)
    samples_per_pass = P * spp
    samples_per_step = samples_per_pass * n_sub

    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    tri, emit, boxes, pos, nrm = t(s.tri), t(s.emit), t(s.boxes), t(s.pos), t(s.nrm)
    radiance = torch.empty((P, 3), dtype=torch.float32, device=dev)
    fp_dev = t(s.footprint) if args.footprint_tile > 0 else None

    def make_ctx(params):
        c = rlc.Context(params)
        c.rlc_build_light_tree(tri, emit)
        c.rlc_set_occluders(boxes)
        if fp_dev is not None:
            c.rlc_set_footprints(fp_dev)
        return c

    ctx = make_ctx(p)

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
        emissions = [t(s.emission_at(f)) for f in range(max(args.steps + 8, args.warmup) + 1)]

    def one_pass(f):
        if emissions is not None:
            ctx.rlc_set_emission(emissions[f])
        if n_sub > 1:
            ctx.rlc_frame_sub(pos, nrm, spp * n_sub, n_sub, f, radiance)
        else:
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
    fused_avg_ms = fused_ms / max(nframes, 1)
    adapt_avg_ms = adapt_ms / max(nframes, 1)
    # steady state: 8 more passes that continue the learned tables
    for f in range(args.steps, args.steps + 8):
        one_pass(f)
    steady_fused_ms, steady_adapt_ms, steady_n = ctx.rlc_get_timing()
    ctx.rlc_set_timing(False)

    # ---- touched cells and (cell, cluster) bins of one steady-state pass ----
    smp = ctx.rlc_sample(pos, nrm, spp, args.steps)
    _, _, reward = ctx.rlc_shade(pos, nrm, spp, smp, contrib=False)
    ctx.rlc_learn(smp, reward)
    dump = ctx.rlc_dump_cells()
    cnt = dump["cnt"]
    cells_t = int((cnt.sum(axis=1) > 0).sum())
    bins_t = int((cnt > 0).sum())
    M = ctx.rlc_meff()
    alg = algorithmic_bytes(samples_per_pass, spp, M, cells_t, bins_t)
    achieved = alg["fused"] / (fused_avg_ms * 1e-3) / 1e9

    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if profiled and tr.get("kernel_source_hash") == kernel_source_hash():
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
        "steady_kernel_ms": round(steady_fused_ms / max(steady_n, 1), 4),
        "steady_adapt_kernel_ms": round(steady_adapt_ms / max(steady_n, 1), 4),
    }
    if traffic:
        # the bytes HBM actually moved (counters) over the same mean duration
        roofline["measured_frac"] = round(traffic / (fused_avg_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)
    if os.path.exists(VALU_FILE):
        with open(VALU_FILE) as f:
            vf = json.load(f)
        if profiled and vf.get("kernel_source_hash") == kernel_source_hash():
            # the kernel's actual limit: VALU issue (counters of the same sources)
            roofline["valu"] = {k: vf[k] for k in ("lane_utilisation", "simd_valu_busy", "useful_lane_valu_frac",
                                                   "wait_any_frac", "valu_insts_per_wave")}

    # ---- MSE at equal GPU time: learning on against learning off ----
    mse = None
    if not args.no_mse and n_sub == 1 and emissions is None:
        mse = mse_equal_time(np, torch, ctx, make_ctx, p, pos, nrm, spp, args.steps, total_ms, P)

    cpu = None
    if not args.no_cpu_baseline:
        if emissions is None and n_sub == 1 and args.footprint_tile == 0:
            workers = args.cpu_workers or min(16, os.cpu_count() or 1)
            cpu = cpu_baseline(np, p, s, spp, args.steps, args.cpu_stride, args.cpu_stride_pool, workers)
        else:
            import oracle
            sel = np.arange(0, P, 20, dtype=np.uint32)
            orc = oracle.Oracle(p, s.tri, s.emit, s.boxes)
            if fp_dev is not None:
                orc.set_footprints(s.footprint)
            print("[bench] CPU oracle: %d points x %d passes" % (sel.size, args.steps), file=sys.stderr,
                  flush=True)
            t0 = time.perf_counter()
            for f in range(args.steps):
                if s.emission_at is not None:
                    orc.set_emission(s.emission_at(f))
                if n_sub > 1:
                    orc.frame_sub(s.pos[sel], s.nrm[sel], spp * n_sub, n_sub, f, pid=sel)
                else:
                    orc.frame(s.pos[sel], s.nrm[sel], spp, f, pid=sel)
                    orc.adapt()
            dt = time.perf_counter() - t0
            cpu = {"value": round(sel.size * spp * n_sub * args.steps / dt, 1), "unit": "samples/s", "cores": 1,
                   "kind": "oracle",
                   "sample": "every 20th point (%d of %d) for the same %d passes, single-threaded C oracle, %.1f s"
                             % (sel.size, P, args.steps, dt),
                   "host_cpus": os.cpu_count(), "cpu_model": cpu_model()}

    if args.workload == "static":
        workload = ("static: 65,536 emissive triangles in 256 clusters, 2,073,600 primary hits "
                    "(1920x1080, in 16x16 pixel tiles), 4,096 box occluders in a 64^3 grid, 64^3 hashed "
                    "cells, cut size 64, 1 spp, passes from a fresh cell table")
    else:
        workload = ("dynamic: 1,048,576 emissive triangles in 16 walled compartments, emission "
                    "Le (1 + sin(2 pi f t + phi)) per compartment set every pass, 1,048,576 points, "
                    "16,384 wall bricks in a 64^3 grid, 64^3 hashed cells, cut size 64, 1 spp, "
                    "temporal adaptation, passes from a fresh cell table")
    if args.split_steps > 1:
        workload += "; split-collapse repeated until a step changes nothing (at most %d steps)" % args.split_steps
    if n_sub > 1:
        workload += "; a step is one frame of %d sub-frame passes, the cuts adapted after each" % n_sub
    if args.footprint_tile > 0:
        workload += ("; footprint-sized cells: %d levels, a point's cell edge at least %g times its pixel "
                     "footprint" % (args.footprint_levels, args.footprint_tile))
    if args.normal_bits or args.jitter > 0:
        workload += "; 5-D cells: %d x %d normal bins, jitter %g" % (1 << args.normal_bits, 1 << args.normal_bits,
                                                                   args.jitter)
    rows = int(p.get("max_cells", 0))
    workload += ("; cell tables with rows for %s cells" % format(rows, ",") if rows
                 else "; cell tables with one row per lookup slot")
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
    if mse is not None:
        line["mse"] = mse
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
