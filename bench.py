#!/usr/bin/env python3
"""Benchmark: brushed spherical-shell ray casting on one MI355X.

Workload (the precision-study configuration): 512^3 x 5 fields (temperature,
temperature anomaly, conductivity, expansivity, |velocity|; seeded synthetic
stand-ins for the paper's mantle snapshots), octree LOD 512/256/128,
1920x1080 image, step 0.5 voxel, 5-axis upper-tail brush keeping ~10 % of the
shell, transfer function on the temperature anomaly, early termination at 0.99.

One step = one interactive brush update followed by one frame: the brush
cycles through four nearby 5-axis brushes, so every step recomputes the brick
skip bits (brush changes rebuild nothing else) and ray-marches the frame with
the level chosen automatically (level 0 at this size).  The volume stays
resident; nothing crosses PCIe inside the timed region.

value = nominal samples/s with FP16 fields (samples the method visits, including
discarded ones, up to early termination; counted once per brush outside the
timed region).  FP32 and 8-bit-brick storage are measured the same way and
reported alongside.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HBM_PEAK = 8.0e12          # bytes/s, MI355X
ALU_PEAK = 256 * 64 * 2.4e9  # non-packed fp32 lane-ops/s: 256 CUs x 64 lanes/clk x 2.4 GHz
IMAGE_BYTES_PER_PIXEL = 16


N_NEEDED_DEFAULT = 5  # fields read per sample in the headline workload (5 brushed, TF field among them)
# FP32 lane operations of the method's own work: per evaluated (not skipped) sample ~15 for its position
# and voxel index, per interpolated field value ~22 (weights, eight corners, brush test), per sample that
# passes the brush ~35 (table lookup, opacity correction with log2 / exp2, front-to-back update)
OPS_PER_EVALUATED, OPS_PER_FETCH, OPS_PER_PASSED = 15, 22, 35
PROFILES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles")
TRAFFIC_RECORD = os.path.join(PROFILES, "raymarch_f16_512x5_1080p_traffic.json")
SERVING_TRAFFIC_RECORD = os.path.join(PROFILES, "serving_f16_saturated_traffic.json")


def traffic_record(path):
    """A committed rocprofv3 counter record (HBM traffic, VALU figures), or None when the kernel
    sources changed since the counters were taken."""
    import hashlib
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    root = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for f in rec["source_files"]:
        h.update(open(os.path.join(root, f), "rb").read())
    return rec if h.hexdigest() == rec["source_sha256"] else None


def measured_traffic(path=TRAFFIC_RECORD):
    """HBM bytes per launch (per replay for the serving record) from the committed FETCH_SIZE /
    WRITE_SIZE record, or None when the kernel sources changed since the counters were taken."""
    rec = traffic_record(path)
    return None if rec is None else rec["traffic_bytes_per_launch"]


HEADLINE_SOURCES = ["paper_2207_12011_amd/csrc/raymarch.hip", "paper_2207_12011_amd/csrc/raymarch_impl.h",
                    "paper_2207_12011_amd/csrc/internal.h", "paper_2207_12011_amd/csrc/preprocess.hip"]
SERVING_SOURCES = ["paper_2207_12011_amd/csrc/raymarch_impl.h", "paper_2207_12011_amd/csrc/raymarch_batch.hip",
                   "paper_2207_12011_amd/csrc/server.hip", "paper_2207_12011_amd/csrc/internal.h",
                   "paper_2207_12011_amd/csrc/preprocess.hip"]


def counter_record(kind, root, frames, out_path, trace_frames=50):
    """Summarise rocprofv3 output under `root` (every *_counter_collection.csv of the --pmc passes,
    and a *_kernel_trace.csv if present) into the counter record read by the roofline.

    kind "headline": the last `frames` launches of the headline ray march (bench.py
    --profile-frames runs), averaged per launch; kind "serving": every batched ray-march and skip
    launch of a bench.py --profile-serving run, summed.  FETCH_SIZE and WRITE_SIZE are scaled by
    what they read for the 1 GiB device copy at the end of the same run."""
    import csv
    import glob
    import hashlib
    root_dir = os.path.dirname(os.path.abspath(__file__))
    rows = []
    for f in sorted(glob.glob(os.path.join(root, "**", "*_counter_collection.csv"), recursive=True)):
        rows += [(f, r) for r in csv.DictReader(open(f))]
    if not rows:
        raise SystemExit(f"no *_counter_collection.csv under {root}")

    def is_kernel(name):
        if kind == "headline":
            return "raymarch_kernel" in name
        return "raymarch_batch_kernel" in name or "skip_kernel" in name

    # counter -> {(pass file, launch): value}; a counter collected in several passes is averaged over
    # them (headline) rather than added up
    counters = {}
    copy = {}
    by_file = {}
    for f, r in rows:
        by_file.setdefault(f, []).append(r)
    for f, rs in by_file.items():
        launches = {}
        for r in rs:
            launches.setdefault(int(r["Dispatch_Id"]), []).append(r)
        order = sorted(launches)
        picked = [d for d in order if is_kernel(launches[d][0]["Kernel_Name"])]
        if kind == "headline":
            picked = picked[-frames:]
        copies = [d for d in order if "copyBuffer" in launches[d][0]["Kernel_Name"]]
        for d in picked:
            per = {}
            for r in launches[d]:
                per[r["Counter_Name"]] = per.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
            for c, v in per.items():
                counters.setdefault(c, {})[(f, d)] = v
        if copies:
            per = {}
            for r in launches[copies[-1]]:
                per[r["Counter_Name"]] = per.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
            for c, v in per.items():
                copy.setdefault(c, []).append(v)
    def combine(vals):
        per_file = {}
        for (f, _), v in vals.items():
            per_file.setdefault(f, []).append(v)
        if kind == "headline":   # mean per launch
            return sum(vals.values()) / len(vals)
        return sum(sum(v) for v in per_file.values()) / len(per_file)   # whole replay, mean over passes
    agg = {c: combine(v) for c, v in counters.items()}
    copy = {c: sum(v) / len(v) for c, v in copy.items()}
    gib_kib = float(1 << 20)
    fetch_scale = gib_kib / copy["FETCH_SIZE"]
    write_scale = gib_kib / copy["WRITE_SIZE"]
    traffic = (agg["FETCH_SIZE"] * fetch_scale + agg["WRITE_SIZE"] * write_scale) * 1024.0
    files = HEADLINE_SOURCES if kind == "headline" else SERVING_SOURCES
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(root_dir, f), "rb").read())
    rec = {"kernel": ("raymarch_kernel<f16 neighbourhood records, 5 brushed fields, no counts, 32-bit record offsets>"
                      if kind == "headline" else
                      "raymarch_batch_kernel (every field count) and skip_kernel of the saturated serving replay"),
           "workload": ("512^3 x 5 fields f16, 1920x1080, step 0.5, ~10% 5-axis brush (the benchmark's headline frame)"
                        if kind == "headline" else
                        "serving trace: 256^3 and 512^3 x 5 f16 volumes, 512 requests 256^2..2048^2, all submitted "
                        "at once"),
           "source_sha256": h.hexdigest(), "source_files": files,
           "copy_1gib_fetch_size_kib": copy["FETCH_SIZE"], "copy_1gib_write_size_kib": copy["WRITE_SIZE"],
           "fetch_scale": fetch_scale, "write_scale": write_scale, "traffic_bytes_per_launch": traffic}
    if kind == "headline":
        rec["fetch_size_kib_per_dispatch"] = agg["FETCH_SIZE"]
        rec["write_size_kib_per_dispatch"] = agg["WRITE_SIZE"]
    else:
        rec["fetch_size_kib_total"] = agg["FETCH_SIZE"]
        rec["write_size_kib_total"] = agg["WRITE_SIZE"]
        rec["note"] = ("traffic_bytes_per_launch is the whole replay (every batched and skip launch of it); "
                       "FETCH_SIZE and WRITE_SIZE from separate rocprofv3 --pmc runs of bench.py --profile-serving, "
                       "scaled by what they read for the 1 GiB copy at the end of the same runs")
    traces = sorted(glob.glob(os.path.join(root, "**", "*_kernel_trace.csv"), recursive=True))
    if kind == "headline" and traces:
        ts = [r for r in csv.DictReader(open(traces[-1])) if is_kernel(r["Kernel_Name"])]
        ts = sorted(ts, key=lambda r: int(r["Start_Timestamp"]))[-trace_frames:]
        rec["trace_avg_ms"] = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in ts) / len(ts) / 1e6
        rec["trace_note"] = f"mean of the last {len(ts)} launches of the kernel trace run (one stream)"
    if kind == "headline" and "SQ_INSTS_VALU" in agg and "GRBM_GUI_ACTIVE" in agg:
        simds, xcds = 1024, 8
        cycles = agg["GRBM_GUI_ACTIVE"] / xcds
        valu = {"busy_frac": agg["SQ_INSTS_VALU"] * 4 / (simds * cycles)}
        if "SQ_THREAD_CYCLES_VALU" in agg and "SQ_ACTIVE_INST_VALU" in agg:
            valu["lane_active_frac"] = agg["SQ_THREAD_CYCLES_VALU"] / (64 * agg["SQ_ACTIVE_INST_VALU"])
            valu["executed_lane_ops"] = agg["SQ_THREAD_CYCLES_VALU"]
            valu["lane_op_frac"] = valu["busy_frac"] * valu["lane_active_frac"]
        if "SQ_WAVE_CYCLES" in agg:
            valu["waves_per_simd"] = agg["SQ_WAVE_CYCLES"] * 4 / (simds * cycles)
        rec["valu"] = valu
        rec["counters_per_launch"] = agg
        if "TCC_HIT_sum" in agg:
            rec["l2_hit_frac"] = agg["TCC_HIT_sum"] / (agg["TCC_HIT_sum"] + agg["TCC_MISS_sum"])
        if "TCP_TCC_READ_REQ_sum" in agg:
            rec["l1_hit_frac"] = 1 - agg["TCP_TCC_READ_REQ_sum"] / agg["TCP_TOTAL_CACHE_ACCESSES_sum"]
    json.dump(rec, open(out_path, "w"), indent=1)
    print(json.dumps(rec, indent=1))


def ordinal(k: int) -> str:
    return f"{k}{'th' if 10 <= k % 100 <= 20 else {1: 'st', 2: 'nd', 3: 'rd'}.get(k % 10, 'th')}"


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q))


def profile(args, wl, raypc, torch):
    """A short, fixed sequence for hardware-counter runs."""
    ctx = raypc.create(0)
    raypc.set_transfer_function(ctx, 0, wl.tf.field, wl.tf.vmin, wl.tf.vmax, wl.tf.rgba, wl.tf.ref_step)
    raypc.set_options(ctx, wl.ert)
    storage = args.storages.split(",")[0]
    vid = raypc.load_fields(ctx, torch.from_numpy(wl.fields).cuda(), storage, 3, wl.r_inner, wl.r_outer)
    raypc.set_brush(ctx, vid, wl.brush.active, wl.brush.lo, wl.brush.hi)
    out = torch.empty((wl.height, wl.width, 4), dtype=torch.float32, device="cuda")
    cam = wl.camera.as_array()
    # the default launch shape (4x4-pixel wave tiles in 32x32-pixel super-tiles, the one the benchmark's
    # autotuner keeps on this device), fixed so that every counter pass profiles the same launches
    # (timing a tuner under counter collection would pick among nearly equal shapes by noise); a few
    # warm-up frames, then the profiled frames are the last launches
    raypc.set_launch_shape(ctx, 2, 2)
    for _ in range(5):
        raypc.render(ctx, vid, cam, wl.width, wl.height, -1, wl.step, out=out)
    print("[bench] profile mode: launch shape: 4x4 px wave tiles, super_log2 2 (fixed)", file=sys.stderr)
    torch.cuda.synchronize()
    for _ in range(args.profile_frames):
        raypc.render(ctx, vid, cam, wl.width, wl.height, -1, wl.step, out=out)
    if args.profile_warps > 0:
        # the image warp of the bench: the depth render, then warps to the pose moved sideways by 0.1
        rgba, depth = raypc.render_depth(ctx, vid, cam, wl.width, wl.height, -1, wl.step)
        c1 = cam.copy()
        c1[0] += np.float32(0.1)
        for _ in range(args.profile_warps):
            raypc.warp(ctx, rgba, depth, cam, c1)
    torch.cuda.synchronize()
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    raypc.destroy(ctx)
    print(f"[bench] profile mode: {args.profile_frames} frames ({storage}), {args.profile_warps} warps + 1 GiB copy",
          file=sys.stderr)


def brush_axis_sweep(raypc, torch, ctx, vid, wl, lod, stream, frames=30):
    """Frame time against the number k of brushed variables (the paper notes the brush cost grows
    linearly with the restricted variables), k = 0..F on the headline view: (a) k fields with
    all-inclusive bounds, which adds the fetch and test of k fields to every evaluated sample and
    discards nothing; (b) the first k axes of the headline brush.  Least-squares line and R^2 each."""
    nf = wl.n_fields
    out = torch.empty((wl.height, wl.width, 4), dtype=torch.float32, device="cuda")
    cam = wl.camera.as_array()

    def frame_ms():
        raypc.render(ctx, vid, cam, wl.width, wl.height, lod, wl.step, out=out, stream=stream)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(frames)]
        for a, e in ev:
            a.record(stream)
            raypc.render(ctx, vid, cam, wl.width, wl.height, lod, wl.step, out=out, stream=stream)
            e.record(stream)
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(e) for a, e in ev]))

    res = {}
    for mode in ("inclusive", "brush_prefix"):
        ks, ms = list(range(nf + 1)), []
        for k in ks:
            act = np.zeros(nf, np.uint8)
            act[:k] = 1
            if mode == "inclusive":
                lo, hi = np.full(nf, -np.inf, np.float32), np.full(nf, np.inf, np.float32)
            else:
                lo, hi = wl.brush.lo, wl.brush.hi
            raypc.set_brush(ctx, vid, act, lo, hi)
            ms.append(frame_ms())
        slope, icpt = np.polyfit(ks, ms, 1)
        fit = slope * np.asarray(ks) + icpt
        ss_res = float(((np.asarray(ms) - fit) ** 2).sum())
        ss_tot = float(((np.asarray(ms) - np.mean(ms)) ** 2).sum())
        res[mode] = {"k": ks, "ms": ms, "slope_ms_per_field": float(slope), "intercept_ms": float(icpt),
                     "r2": 1.0 - ss_res / ss_tot if ss_tot > 0 else 1.0}
        print(f"[bench] brush-axis sweep ({mode}): {res[mode]}", file=sys.stderr, flush=True)
    # coordinate axes with the headline brush: a half-space cut and a radius (altitude) band
    raypc.set_brush(ctx, vid, wl.brush.active, wl.brush.lo, wl.brush.hi)
    cuts = {"none": ([0, 0, 0, 0], [0] * 4, [0] * 4),
            "x >= 0": ([1, 0, 0, 0], [0.0, 0, 0, 0], [1.0, 0, 0, 0]),
            "0.7 <= r <= 0.85": ([0, 0, 0, 1], [0, 0, 0, 0.7], [0, 0, 0, 0.85])}
    res["coordinate_cuts_ms"] = {}
    for name, c in cuts.items():
        raypc.set_coordinate_brush(ctx, vid, *c)
        res["coordinate_cuts_ms"][name] = frame_ms()
    raypc.set_coordinate_brush(ctx, vid, *cuts["none"])
    print(f"[bench] coordinate cuts (ms): {res['coordinate_cuts_ms']}", file=sys.stderr, flush=True)
    return res


def jittered_timing(raypc, torch, ctx, vid, wl, lod, stream, n_passes=8, seed=0x5EED2207):
    """Jittered progressive passes on the headline view and brush: median time of one pass (with the
    running-mean update) against the plain frame, and the mean-abs error of the running mean after
    1, 2, 4 and 8 passes against the render at step / 8."""
    cam = wl.camera.as_array()
    W_, H_ = wl.width, wl.height
    out = torch.empty((H_, W_, 4), dtype=torch.float32, device="cuda")
    fine = torch.empty((H_, W_, 4), dtype=torch.float32, device="cuda")
    mean = torch.empty((H_, W_, 4), dtype=torch.float32, device="cuda")
    raypc.render(ctx, vid, cam, W_, H_, lod, wl.step / n_passes, out=fine, stream=stream)
    errs, times = {}, []
    for rnd in range(3):
        for k in range(n_passes):
            a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            raypc.render_jittered(ctx, vid, cam, W_, H_, lod, wl.step, k, n_passes, seed, mean=mean, stream=stream)
            e.record(stream)
            torch.cuda.synchronize()
            if rnd > 0:
                times.append(a.elapsed_time(e))
            if rnd == 0 and (k + 1) in (1, 2, 4, 8):
                errs[k + 1] = float((mean - fine).abs().mean().item())
    res = {"passes": n_passes, "ms_per_pass": float(np.median(times)),
           "mean_abs_err_vs_step_over_8": errs}
    print(f"[bench] jittered passes: {res}", file=sys.stderr, flush=True)
    return res


WARP_BYTES_PER_PIXEL = 68  # key fill 8, depth 4, atomic 8, key read 8, RGBA gather 16, outputs 16 + 4 + 4


def warp_timing(raypc, torch, ctx, vid, wl, lod, stream, calls=50):
    """Image warping of the headline frame: the depth render against the plain frame, and the warp
    of the rendered frame to a pose moved sideways by 0.1 and 0.2 (median of `calls` warps), with
    the mean-abs error of the stale and of the warped frame against the frame rendered at the new
    pose."""
    cam = wl.camera.as_array()
    W_, H_ = wl.width, wl.height
    rgba = torch.empty((H_, W_, 4), dtype=torch.float32, device="cuda")
    depth = torch.empty((H_, W_), dtype=torch.float32, device="cuda")
    truth = torch.empty((H_, W_, 4), dtype=torch.float32, device="cuda")
    out = torch.empty((H_, W_, 4), dtype=torch.float32, device="cuda")
    out_d = torch.empty((H_, W_), dtype=torch.float32, device="cuda")
    out_s = torch.empty((H_, W_), dtype=torch.int32, device="cuda")

    def median_ms(fn, n):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        for a, e in ev:
            a.record(stream)
            fn()
            e.record(stream)
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(e) for a, e in ev]))

    depth_ms = median_ms(lambda: raypc.render_depth(ctx, vid, cam, W_, H_, lod, wl.step, out=rgba, depth=depth,
                                                    stream=stream), 20)
    plain_ms = median_ms(lambda: raypc.render(ctx, vid, cam, W_, H_, lod, wl.step, out=truth, stream=stream), 20)
    raypc.render_depth(ctx, vid, cam, W_, H_, lod, wl.step, out=rgba, depth=depth, stream=stream)
    moves = {}
    for dx in (0.1, 0.2):
        c1 = cam.copy()
        c1[0] += np.float32(dx)
        ms = median_ms(lambda: raypc.warp(ctx, rgba, depth, cam, c1, out=out, out_depth=out_d, out_source=out_s,
                                          stream=stream), calls)
        raypc.render(ctx, vid, c1, W_, H_, lod, wl.step, out=truth, stream=stream)
        torch.cuda.synchronize()
        moves[f"eye x + {dx}"] = {
            "warp_ms": ms, "gb_per_s": W_ * H_ * WARP_BYTES_PER_PIXEL / (ms * 1e-3) / 1e9,
            "covered": float((out_s >= 0).float().mean().item()),
            "mean_abs_err_stale": float((rgba - truth).abs().mean().item()),
            "mean_abs_err_warped": float((out - truth).abs().mean().item())}
    res = {"pixels": W_ * H_, "render_depth_ms": depth_ms, "render_ms": plain_ms,
           "alg_bytes_per_pixel": WARP_BYTES_PER_PIXEL, "moves": moves}
    print(f"[bench] image warp: {res}", file=sys.stderr, flush=True)
    return res


def pc_lines_timing(raypc, torch, W, ctx, vid, wl, stream, n_lines=100_000, n_bins=64, calls=50):
    """The parallel-coordinates lines of the paper's preprocessing (up to 100 000 random shell cells):
    values, brush flags and 64-bin histograms of all / passing lines per axis, for the headline
    brush; median time of one call."""
    cells = torch.from_numpy(W.pc_line_cells(wl.n, n_lines).astype(np.int32)).cuda()
    nf = wl.n_fields
    axis_lo = wl.fields.reshape(nf, -1).min(axis=1)
    axis_hi = wl.fields.reshape(nf, -1).max(axis=1)
    raypc.pc_lines(ctx, vid, 0, cells, axis_lo, axis_hi, n_bins, stream=stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(calls)]
    for a, e in ev:
        a.record(stream)
        _, passes, _ = raypc.pc_lines(ctx, vid, 0, cells, axis_lo, axis_hi, n_bins, stream=stream)
        e.record(stream)
    torch.cuda.synchronize()
    us = 1e3 * float(np.median([a.elapsed_time(e) for a, e in ev]))
    res = {"lines": int(cells.numel()), "bins": n_bins, "fields": nf, "us": us,
           "lines_per_s": cells.numel() / (us * 1e-6), "passing": int(passes.sum().item())}
    print(f"[bench] parallel-coordinates lines: {res}", file=sys.stderr, flush=True)
    return res


def serving(args, raypc, torch, W, wl512, fields512_dev, profile_only=False):
    """Serving configuration: 256^3 and 512^3 x 5 FP16 volumes resident; a seeded trace of
    requests (sizes 256^2 .. 2048^2, orbit cameras, 1-5-axis quantile brushes, level by the
    selection rule, step 0.5) replayed with Poisson arrivals at several rates through the
    continuous-batching server; latency = completion - submission (host monotonic clock).
    The plain FP32 single-request path renders the same requests one at a time (no load)."""
    wl256 = W.make_workload(1)
    rng = np.random.default_rng(3)
    tables = [W.quantile_table(wl256.fields, W.shell_mask(W.radius(256)), rng),
              W.quantile_table(wl512.fields, W.shell_mask(W.radius(512)), rng)]
    trace = W.serving_trace(tables, n=args.serving_requests)
    ctx = raypc.create(0)
    tf = wl512.tf
    raypc.set_transfer_function(ctx, 0, tf.field, tf.vmin, tf.vmax, tf.rgba, tf.ref_step)
    raypc.set_options(ctx, wl512.ert)
    f256 = torch.from_numpy(wl256.fields).cuda()
    vols16 = [raypc.load_fields(ctx, f256, "f16", 3), raypc.load_fields(ctx, fields512_dev, "f16", 3)]
    outs = [torch.empty((q.height, q.width, 4), dtype=torch.float32, device="cuda") for q in trace]
    reqs = [raypc.make_request(vols16[q.volume], q.camera, q.width, q.height, o, -1, 0.5, q.active, q.lo, q.hi, 0)
            for q, o in zip(trace, outs)]
    pixels = sum(q.width * q.height for q in trace)
    # the method's own work and algorithmic bytes of every request (outside the timed region): touched
    # bricks x fields read x 2 bytes + the image; evaluated samples, field fetches, passing samples
    alg_bytes, alg_ops, nominal = 0, 0, 0
    for q, o in zip(trace, [] if profile_only else outs):
        vid = vols16[q.volume]
        raypc.set_brush(ctx, vid, q.active, q.lo, q.hi)
        lv = raypc.select_lod(ctx, vid, q.camera, q.width, q.height)
        nb = (raypc.volume_info(ctx, vid)["n"] >> lv) // 8
        touched = torch.zeros(((nb ** 3 + 31) // 32,), dtype=torch.int32, device="cuda")
        _, nom, comp = raypc.render_debug(ctx, vid, q.camera, q.width, q.height, -1, 0.5, touched=touched)
        _, ev_, fe_ = raypc.render_work(ctx, vid, q.camera, q.width, q.height, -1, 0.5)
        torch.cuda.synchronize()
        n_needed = len(set(np.flatnonzero(q.active).tolist()) | {tf.field})
        tb = int(np.unpackbits(touched.cpu().numpy().view(np.uint8)).sum())
        alg_bytes += tb * 512 * n_needed * 2 + q.width * q.height * IMAGE_BYTES_PER_PIXEL
        alg_ops += (OPS_PER_EVALUATED * int(ev_.to(torch.int64).sum().item()) +
                    OPS_PER_FETCH * int(fe_.to(torch.int64).sum().item()) +
                    OPS_PER_PASSED * int(comp.to(torch.int64).sum().item()))
        nominal += int(nom.to(torch.int64).sum().item())
    result = {"requests": len(trace), "pixels": pixels, "volumes": ["256^3 x 5 f16", "512^3 x 5 f16"],
              "alg_bytes": alg_bytes, "alg_ops": alg_ops, "nominal_samples": nominal,
              "sizes": [list(s) for s in W.SERVING_SIZES], "server": {"max_inflight": 64, "tiles_per_step": 32768,
                                                                     "steps_in_flight": 2, "mem_budget_bytes": 8 << 30},
              "by_qps": {}}
    # warm the batched kernel (not in profiling mode, whose counters cover the replay alone)
    if not profile_only:
        raypc.server_start(ctx, 8 << 30, 64, 32768, 2)
        for r in reqs[:8]:
            raypc.wait(ctx, raypc.submit(ctx, r), 120000)
        raypc.server_stop(ctx)
    for qps_s in ("inf",) if profile_only else args.serving_qps.split(","):
        qps = float(qps_s)
        raypc.server_start(ctx, 8 << 30, 64, 32768, 2)
        tickets = []
        t0 = time.perf_counter()
        due = 0.0
        for q, r in zip(trace, reqs):
            if math.isfinite(qps):
                due += q.gap / qps
                while time.perf_counter() - t0 < due:
                    pass
            tickets.append(raypc.submit(ctx, r))
        for t in tickets:
            raypc.wait(ctx, t, 120000)
        times = np.array([raypc.request_times(ctx, t) for t in tickets])
        stats = raypc.server_get_stats(ctx)
        raypc.server_stop(ctx)
        lat = times[:, 3] - times[:, 0]
        span = (times[:, 3].max() - times[:, 0].min()) / 1e3
        result["by_qps"][qps_s] = {"p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
                                   "max_ms": float(lat.max()), "requests_per_s": len(trace) / span,
                                   "pixels_per_s": pixels / span, "samples_per_s": nominal / span,
                                   "steps": stats["steps"], "peak_bytes_in_use": stats["peak_bytes_in_use"]}
        if not math.isfinite(qps):
            # the saturated replay: the serving path's own roofline (wall time of the whole replay)
            traffic = measured_traffic(SERVING_TRAFFIC_RECORD)
            result["roofline"] = {
                "span_s": span,
                "alu": {"bound": "alu", "achieved": alg_ops / span / 1e12, "peak": ALU_PEAK / 1e12,
                        "unit": "Tlane-op/s", "frac": alg_ops / span / ALU_PEAK},
                "hbm_algorithmic": {"achieved": alg_bytes / span / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                                    "frac": alg_bytes / span / HBM_PEAK},
                "hbm_measured": None if traffic is None else
                {"achieved": traffic / span / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                 "frac": traffic / span / HBM_PEAK, "traffic_bytes": traffic}}
        print(f"[bench] serving qps={qps_s}: {result['by_qps'][qps_s]}", file=sys.stderr, flush=True)
    for v in vols16:
        raypc.unload(ctx, v)
    if profile_only:
        raypc.destroy(ctx)
        return result
    # plain FP32 single-request path on the same GPU
    vols32 = [raypc.load_fields(ctx, f256, "f32", 3), raypc.load_fields(ctx, fields512_dev, "f32", 3)]
    lat32 = []
    for i, (q, o) in enumerate(zip(trace, outs)):
        vid = vols32[q.volume]
        raypc.set_brush(ctx, vid, q.active, q.lo, q.hi)
        torch.cuda.synchronize()
        a = time.perf_counter()
        raypc.render(ctx, vid, q.camera, q.width, q.height, -1, 0.5, out=o)
        torch.cuda.synchronize()
        lat32.append(1e3 * (time.perf_counter() - a))
    result["fp32_single_request"] = {"p50_ms": percentile(lat32, 50), "p99_ms": percentile(lat32, 99),
                                     "max_ms": max(lat32), "requests_per_s": len(lat32) / (sum(lat32) / 1e3)}
    print(f"[bench] fp32 single-request path: {result['fp32_single_request']}", file=sys.stderr, flush=True)
    raypc.destroy(ctx)
    return result


def progressive(args, raypc, torch, W):
    """Large progressive configuration: a 1024^3 x 5 volume, a 3840x2160 view (the default camera),
    three passes at step 1.0 / 0.5 / 0.25 voxel after every brush change, for 10 brush requests
    narrowing linearly in quantile space from all-inclusive to the ~10 % 5-axis brush.  Per request:
    brush change -> first pass and -> final pass latency (host clock, from the set_brush call to
    the pass's completion event; the volume stays resident, only the brush crosses to the device).
    The requests run twice; the second round is reported.  Prints its own JSON line."""
    t_gen = time.perf_counter()
    wl = W.make_workload(4, n=args.prog_n, width=args.prog_width, height=args.prog_height,
                         progress=lambda msg: print(f"[bench] generated {msg} ({time.perf_counter() - t_gen:.0f}s)",
                                                    file=sys.stderr, flush=True))
    mask = W.shell_mask(W.radius(wl.n))
    brushes = W.narrowing_brushes(wl.fields, mask, np.random.default_rng(W.SEED_BASE + 4), wl.brush)
    del mask
    print(f"[bench] progressive workload {wl.name} generated in {time.perf_counter() - t_gen:.1f}s",
          file=sys.stderr, flush=True)
    ctx = raypc.create(0)
    raypc.set_transfer_function(ctx, 0, wl.tf.field, wl.tf.vmin, wl.tf.vmax, wl.tf.rgba, wl.tf.ref_step)
    raypc.set_options(ctx, wl.ert)
    fields_dev = torch.from_numpy(wl.fields).cuda()
    stream = torch.cuda.current_stream()
    cam = wl.camera.as_array()
    W_, H_ = wl.width, wl.height
    steps = [wl.step * 4, wl.step * 2, wl.step]
    outs = [torch.empty((H_, W_, 4), dtype=torch.float32, device="cuda") for _ in steps]
    results = {}
    for storage in args.prog_storages.split(","):
        t_load = time.perf_counter()
        vid = raypc.load_fields(ctx, fields_dev, storage, 3, wl.r_inner, wl.r_outer)
        load_s = time.perf_counter() - t_load
        lod = raypc.select_lod(ctx, vid, cam, W_, H_)
        # nominal samples per pass for the final brush (counting variant, outside the timed region)
        raypc.set_brush(ctx, vid, brushes[-1].active, brushes[-1].lo, brushes[-1].hi)
        pass_samples = []
        for st in steps:
            _, nom, _ = raypc.render_debug(ctx, vid, cam, W_, H_, lod, st)
            torch.cuda.synchronize()
            pass_samples.append(int(nom.to(torch.int64).sum().item()))
        first, final, passes = [], [], []
        for rnd in range(2):
            first, final, passes = [], [], []
            for b in brushes:
                torch.cuda.synchronize()
                ev0 = torch.cuda.Event(enable_timing=True)
                evs = [torch.cuda.Event(enable_timing=True) for _ in steps]
                t0 = time.perf_counter()
                raypc.set_brush(ctx, vid, b.active, b.lo, b.hi)
                ev0.record(stream)
                for st, o, e in zip(steps, outs, evs):
                    raypc.render(ctx, vid, cam, W_, H_, lod, st, out=o, stream=stream)
                    e.record(stream)
                evs[0].synchronize()
                first.append(1e3 * (time.perf_counter() - t0))
                evs[-1].synchronize()
                final.append(1e3 * (time.perf_counter() - t0))
                passes.append([ev0.elapsed_time(evs[0])] + [evs[i - 1].elapsed_time(evs[i]) for i in range(1, len(evs))])
        last = passes[-1]
        results[storage] = {
            "brush_to_first_pass_ms": first, "brush_to_final_pass_ms": final, "pass_ms": passes,
            "final_brush_nominal_samples_per_pass": pass_samples,
            "final_brush_samples_per_s_per_pass": [n / (t * 1e-3) for n, t in zip(pass_samples, last)],
            "lod": lod, "load_s": load_s, "volume_bytes": raypc.volume_info(ctx, vid)["bytes"]}
        print(f"[bench] progressive {storage}: first {np.round(first, 2).tolist()} final {np.round(final, 2).tolist()} "
              f"samples/pass {pass_samples} load {load_s:.1f}s", file=sys.stderr, flush=True)
        raypc.unload(ctx, vid)
    raypc.destroy(ctx)
    line = {"metric": "large progressive: brush change -> first / final pass latency (ms)",
            "unit": "ms", "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
            "config": {"workload": wl.name + f", passes at step {steps} voxel, 10 narrowing brushes",
                       "volume": wl.n, "fields": wl.n_fields, "width": W_, "height": H_},
            "per_storage": results}
    print(json.dumps(line), flush=True)


def cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_run(args, wl, head, cam, b, frame_samples_gpu):
    """The FP64 oracle as it stands, timed on the host: the render call only, median of 3 runs after
    one warm-up, with the threads this process may use (OMP_NUM_THREADS, else the CPU affinity),
    plus a one-thread figure on every 8th row and column."""
    import oracle
    from oracle import preprocess as pp
    W_, H_ = wl.width, wl.height
    level = np.stack([pp.stored_values(wl.fields[f], head) for f in range(wl.n_fields)])
    ys, xs = np.meshgrid(np.arange(0, H_, args.cpu_stride), np.arange(0, W_, args.cpu_stride), indexing="ij")
    pix = (ys * W_ + xs).ravel()
    affinity = len(os.sched_getaffinity(0))
    threads = int(os.environ.get("OMP_NUM_THREADS") or affinity)
    kw = dict(active=b.active, lo=b.lo, hi=b.hi, tf_field=wl.tf.field, vmin=wl.tf.vmin, vmax=wl.tf.vmax,
              tf_rgba=wl.tf.rgba, ref_step=wl.tf.ref_step, ert=wl.ert, r_inner=wl.r_inner, r_outer=wl.r_outer)

    def timed(p, th, runs):
        ts, ref = [], None
        for k in range(runs + 1):
            t0 = time.perf_counter()
            ref = oracle.render(level, cam, W_, H_, wl.step, pixels=p, threads=th, **kw)
            if k > 0:
                ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), ts, int(ref.nominal.astype(np.int64).sum())

    dt, ts, ns = timed(pix, threads, 3)
    ys1, xs1 = np.meshgrid(np.arange(0, H_, 8), np.arange(0, W_, 8), indexing="ij")
    pix1 = (ys1 * W_ + xs1).ravel()
    dt1, ts1, ns1 = timed(pix1, 1, 1)
    frame_samples = ns if args.cpu_stride == 1 else frame_samples_gpu
    res = {"value": ns / dt, "unit": "samples/s", "cores": threads, "kind": "oracle",
           "frames_per_s": ns / dt / frame_samples,
           "sample": (f"the whole {W_}x{H_} frame" if args.cpu_stride == 1 else
                      f"every {ordinal(args.cpu_stride)} row and column of the {W_}x{H_} frame") +
                     f" ({pix.size} px, {ns} nominal samples, median of 3 runs after a warm-up: "
                     f"{', '.join(f'{t:.2f}' for t in ts)} s on {threads} threads), brush 0, "
                     f"{head}-stored {wl.n}^3 x {wl.n_fields} level 0, FP64",
           "host": {"cpu_model": cpu_model(), "nproc": os.cpu_count(), "affinity_cpus": affinity,
                    "omp_num_threads": os.environ.get("OMP_NUM_THREADS")},
           "single_thread": {"value": ns1 / dt1, "unit": "samples/s", "frames_per_s": ns1 / dt1 / frame_samples,
                             "sample": f"every 8th row and column ({pix1.size} px, {ns1} nominal samples, "
                                       f"{dt1:.1f} s on 1 thread after a warm-up)"}}
    print(f"[bench] cpu baseline: {res}", file=sys.stderr, flush=True)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--in-flight", type=int, default=2,
                    help="frames in flight in the timed loop (streams used in turn); 1 = serial")
    ap.add_argument("--in-flight-sweep", default="",
                    help="also time the headline storage's loop with each of these frames-in-flight counts")
    ap.add_argument("--storages", default="f16,f32,u8,f16c,u8c",
                    help="first one is the headline value; a trailing c keeps only the compact layout")
    ap.add_argument("--cpu-stride", type=int, default=1, help="oracle sample: every k-th row and column")
    ap.add_argument("--orbit-frames", type=int, default=200, help="single-request latency frames (seeded orbit cameras)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--width", type=int, default=1920)
    ap.add_argument("--height", type=int, default=1080)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the brush-axis sweep")
    ap.add_argument("--progressive", action="store_true",
                    help="run only the large progressive configuration (1024^3 x 5, 3840x2160) and print its JSON line")
    ap.add_argument("--prog-n", type=int, default=1024)
    ap.add_argument("--prog-width", type=int, default=3840)
    ap.add_argument("--prog-height", type=int, default=2160)
    ap.add_argument("--prog-storages", default="f16,f16c,u8,u8c")
    ap.add_argument("--serving-requests", type=int, default=512)
    ap.add_argument("--serving-qps", default="25,50,100,200,400,inf",
                    help="Poisson arrival rates (requests/s); inf submits the whole trace at once")
    ap.add_argument("--profile-frames", type=int, default=0,
                    help="profiling mode: load the headline storage, render this many frames with the first "
                         "brush, then copy 1 GiB device-to-device (a known-size kernel for counter scaling); "
                         "prints no JSON")
    ap.add_argument("--profile-warps", type=int, default=0,
                    help="profiling mode: also render the frame with depth and warp it this many times to the "
                         "pose moved sideways by 0.1")
    ap.add_argument("--profile-serving", action="store_true",
                    help="profiling mode: replay the serving trace once, all requests at once, then copy 1 GiB "
                         "device-to-device; prints no JSON")
    ap.add_argument("--counter-record", choices=["headline", "serving"], default=None,
                    help="no GPU: summarise the rocprofv3 CSVs under --counter-dir into the counter record "
                         "--counter-out (the headline's last --counter-frames launches, or the serving replay)")
    ap.add_argument("--counter-dir", default="")
    ap.add_argument("--counter-out", default="")
    ap.add_argument("--counter-frames", type=int, default=2)
    ap.add_argument("--counter-trace-frames", type=int, default=50)
    args = ap.parse_args()
    if args.counter_record:
        counter_record(args.counter_record, args.counter_dir, args.counter_frames, args.counter_out,
                       args.counter_trace_frames)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU (got --gpus {args.gpus}): the renderer shards by request across "
              "GPUs with no communication, so per-GPU numbers are the 1-GPU numbers.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2207_12011_amd import autotune, raypc
    from paper_2207_12011_amd import workloads as W

    if args.progressive:
        progressive(args, raypc, torch, W)
        return
    t_gen = time.perf_counter()
    wl = W.make_workload(2, n=args.n, width=args.width, height=args.height)
    if args.profile_frames > 0:
        profile(args, wl, raypc, torch)
        return
    if args.profile_serving:
        # the saturated serving replay alone, then a known-size copy for counter scaling
        serving(args, raypc, torch, W, wl, torch.from_numpy(wl.fields).cuda(), profile_only=True)
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] profile mode: saturated serving replay + 1 GiB copy", file=sys.stderr)
        return
    mask = W.shell_mask(W.radius(wl.n))
    rng = np.random.default_rng(7)
    brushes = [wl.brush] + [W.upper_tail_brush(wl.fields, mask, rng, target=t) for t in (0.08, 0.12, 0.09)]
    del mask
    print(f"[bench] workload generated in {time.perf_counter() - t_gen:.1f}s", file=sys.stderr, flush=True)

    cam = wl.camera.as_array()
    W_, H_ = wl.width, wl.height
    ctx = raypc.create(0)
    # the device's measured ceilings (a 1 GiB copy, an FMA loop) beside the vendor's figures
    peaks = raypc.measure_peaks(ctx)
    peaks.update({"copy_frac_of_hbm_peak": peaks["copy_bytes_per_s"] / HBM_PEAK,
                  "fma_frac_of_vendor_rate": peaks["fma_lane_ops_per_s"] / ALU_PEAK,
                  "vendor": {"hbm_bytes_per_s": HBM_PEAK, "fp32_lane_ops_per_s": ALU_PEAK}})
    print(f"[bench] measured peaks: {peaks}", file=sys.stderr, flush=True)
    fields_dev = torch.from_numpy(wl.fields).cuda()
    raypc.set_transfer_function(ctx, 0, wl.tf.field, wl.tf.vmin, wl.tf.vmax, wl.tf.rgba, wl.tf.ref_step)
    raypc.set_options(ctx, wl.ert)
    stream = torch.cuda.current_stream()
    # the streams frames in flight use in turn, created once and one after the other (the runtime maps
    # streams onto a few hardware queues in turn, so these land on different queues and can overlap)
    n_streams = max([args.in_flight] + [int(x) for x in args.in_flight_sweep.split(",") if x])
    flight_streams = [torch.cuda.Stream() for _ in range(n_streams)]
    out = torch.empty((H_, W_, 4), dtype=torch.float32, device="cuda")
    results = {}
    sweep_result = None
    pc_result = None
    jit_result = None
    warp_result = None
    storages = args.storages.split(",")
    bpv = {"f32": 4, "f16": 2, "u8": 1, "f32c": 4, "f16c": 2, "u8c": 1}

    for si, storage in enumerate(storages):
        vid = raypc.load_fields(ctx, fields_dev, storage, 3, wl.r_inner, wl.r_outer)
        lod = raypc.select_lod(ctx, vid, cam, W_, H_)
        # launch shape picked by the autotuner on the headline brush (outside the timed region)
        raypc.set_brush(ctx, vid, brushes[0].active, brushes[0].lo, brushes[0].hi)
        shape = autotune.tune_render(raypc, ctx, vid, cam, W_, H_, lod, wl.step, repeats=10)
        nb = (wl.n >> lod) // 8
        # per-brush nominal sample counts and touched bricks (outside the timed region)
        samples, touched_bricks = [], []
        for b in brushes:
            raypc.set_brush(ctx, vid, b.active, b.lo, b.hi)
            touched = torch.zeros(((nb ** 3 + 31) // 32,), dtype=torch.int32, device="cuda")
            _, nom, comp = raypc.render_debug(ctx, vid, cam, W_, H_, lod, wl.step, touched=touched)
            torch.cuda.synchronize()
            samples.append(int(nom.to(torch.int64).sum().item()))
            tb = touched.cpu().numpy().view(np.uint32)
            touched_bricks.append(int(np.unpackbits(tb.view(np.uint8)).sum()))
            if b is brushes[0]:
                # the method's own work on the headline brush: samples not skipped, field values
                # interpolated for them, samples that passed the brush
                _, ev_, fe_ = raypc.render_work(ctx, vid, cam, W_, H_, lod, wl.step)
                torch.cuda.synchronize()
                work = {"evaluated_samples": int(ev_.to(torch.int64).sum().item()),
                        "field_fetches": int(fe_.to(torch.int64).sum().item()),
                        "passed_samples": int(comp.to(torch.int64).sum().item())}
        n_needed = len(set(np.flatnonzero(brushes[0].active).tolist()) | {wl.tf.field})

        # timed: K steps (brush change + frame).  Frames go to `args.in_flight` streams in turn (each
        # with its own output image), so a frame's first blocks start while the previous frame's last
        # blocks drain; the skip flags of each brush are a new version, so frames in flight never share
        # them.  in_flight 1 is the serial loop.
        def timed_loop(n_flight, steps, warm):
            sts = flight_streams[:n_flight]
            images = [out] + [torch.empty_like(out) for _ in range(n_flight - 1)]
            for s_ in range(warm):
                b_ = brushes[s_ % len(brushes)]
                raypc.set_brush(ctx, vid, b_.active, b_.lo, b_.hi)
                raypc.render(ctx, vid, cam, W_, H_, -1, wl.step, out=images[s_ % n_flight], stream=sts[s_ % n_flight])
            torch.cuda.synchronize()
            ev_ = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
            tot = 0
            t0_ = time.perf_counter()
            for s_ in range(steps):
                k_ = s_ % len(brushes)
                b_ = brushes[k_]
                st_ = sts[s_ % n_flight]
                raypc.set_brush(ctx, vid, b_.active, b_.lo, b_.hi)
                ev_[s_][0].record(st_)
                raypc.render(ctx, vid, cam, W_, H_, -1, wl.step, out=images[s_ % n_flight], stream=st_)
                ev_[s_][1].record(st_)
                tot += samples[k_]
            torch.cuda.synchronize()
            return time.perf_counter() - t0_, tot, [a_.elapsed_time(e_) for a_, e_ in ev_]

        serial_wall, serial_samples, serial_lat = timed_loop(1, args.steps, args.warmup)
        wall, total_samples, lat = timed_loop(args.in_flight, args.steps, args.warmup)
        in_flight_sweep = None
        if si == 0 and args.in_flight_sweep:
            in_flight_sweep = {}
            for nf_ in (int(x) for x in args.in_flight_sweep.split(",")):
                w_, t_, l_ = timed_loop(nf_, args.steps, args.warmup)
                in_flight_sweep[str(nf_)] = {"ms_per_step": 1e3 * w_ / args.steps, "samples_per_s": t_ / w_,
                                             "latency_p50_ms": percentile(l_, 50), "latency_p99_ms": percentile(l_, 99)}
            print(f"[bench] frames in flight: {in_flight_sweep}", file=sys.stderr, flush=True)

        # kernel-only: fixed brush (skip bits cached), back-to-back launches on the same stream
        b = brushes[0]
        raypc.set_brush(ctx, vid, b.active, b.lo, b.hi)
        raypc.render(ctx, vid, cam, W_, H_, lod, wl.step, out=out, stream=stream)
        torch.cuda.synchronize()
        kev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(50)]
        for a, e in kev:
            a.record(stream)
            raypc.render(ctx, vid, cam, W_, H_, lod, wl.step, out=out, stream=stream)
            e.record(stream)
        torch.cuda.synchronize()
        kms = float(np.mean([a.elapsed_time(e) for a, e in kev]))

        # single-request latency over seeded orbit cameras (headline brush, LOD by the rule, HIP events)
        orng = np.random.default_rng(220712011 + 7)
        ocams = [W.orbit_camera(orng.uniform(0.0, 2 * math.pi), math.radians(orng.uniform(-60.0, 60.0))).as_array()
                 for _ in range(args.orbit_frames)]
        raypc.set_brush(ctx, vid, b.active, b.lo, b.hi)
        for c in ocams[:5]:
            raypc.render(ctx, vid, c, W_, H_, -1, wl.step, out=out, stream=stream)
        oev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in ocams]
        for c, (a_, e_) in zip(ocams, oev):
            a_.record(stream)
            raypc.render(ctx, vid, c, W_, H_, -1, wl.step, out=out, stream=stream)
            e_.record(stream)
        torch.cuda.synchronize()
        olat = [a_.elapsed_time(e_) for a_, e_ in oev]

        alg_bytes = touched_bricks[0] * 512 * n_needed * bpv[storage] + W_ * H_ * IMAGE_BYTES_PER_PIXEL
        if storage.startswith("u8"):
            alg_bytes += touched_bricks[0] * 8 * n_needed
        alg_ops = (OPS_PER_EVALUATED * work["evaluated_samples"] + OPS_PER_FETCH * work["field_fetches"] +
                   OPS_PER_PASSED * work["passed_samples"])
        work["ops_model"] = (f"{OPS_PER_EVALUATED} per evaluated sample + {OPS_PER_FETCH} per field fetch + "
                             f"{OPS_PER_PASSED} per passing sample")
        work["dense_equivalent_ops"] = samples[0] * (50 + 22 * n_needed)
        results[storage] = {
            "samples_per_s": total_samples / wall,
            "frames_per_s": args.steps / wall,
            "ms_per_step": 1e3 * wall / args.steps,
            "frames_in_flight": args.in_flight,
            "frames_in_flight_sweep": in_flight_sweep,
            "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99), "max": max(lat)},
            "serial": {"frames_in_flight": 1, "samples_per_s": serial_samples / serial_wall,
                       "frames_per_s": args.steps / serial_wall, "ms_per_step": 1e3 * serial_wall / args.steps,
                       "latency_ms": {"p50": percentile(serial_lat, 50), "p99": percentile(serial_lat, 99),
                                      "max": max(serial_lat)}},
            "nominal_samples_per_frame": samples,
            "touched_bricks": touched_bricks[0],
            "bricks_per_level": nb ** 3,
            "lod": lod,
            "kernel_ms": kms,
            "alg_bytes_per_launch": alg_bytes,
            "alg_ops_per_launch": alg_ops,
            "work": work,
            "volume_bytes": raypc.volume_info(ctx, vid)["bytes"],
            "orbit_latency_ms": {"frames": len(olat), "p50": percentile(olat, 50), "p99": percentile(olat, 99),
                                 "max": max(olat), "cameras": "seeded orbit: azimuth U[0, 360), elevation U[-60, 60] deg, "
                                                              "distance 3, up +z, 60 deg"},
            "launch_shape": {"wave_tile_px": shape["wave_tile_px"], "super_tile_px": shape["super_tile_px"],
                             "ms_by_wave_tile_and_super_log2":
                             {f"{1 << t}x{16 >> t}": {str(k): ms for k, ms in enumerate(row)}
                              for t, row in enumerate(shape["ms"])}},
        }
        print(f"[bench] {storage}: {results[storage]}", file=sys.stderr, flush=True)
        if si == 0 and not args.no_sweep:
            sweep_result = brush_axis_sweep(raypc, torch, ctx, vid, wl, lod, stream)
        if si == 0:
            pc_result = pc_lines_timing(raypc, torch, W, ctx, vid, wl, stream)
            jit_result = jittered_timing(raypc, torch, ctx, vid, wl, lod, stream)
            warp_result = warp_timing(raypc, torch, ctx, vid, wl, lod, stream)
        raypc.unload(ctx, vid)

    head = storages[0]
    r = results[head]
    ksec = r["kernel_ms"] * 1e-3
    achieved_bw = r["alg_bytes_per_launch"] / ksec
    achieved_ops = r["alg_ops_per_launch"] / ksec
    rec = traffic_record(TRAFFIC_RECORD) if head == "f16" and (wl.n, W_, H_) == (512, 1920, 1080) else None
    traffic = None if rec is None else rec["traffic_bytes_per_launch"]
    dense = r["work"]["dense_equivalent_ops"] / ksec
    piped = r["alg_ops_per_launch"] / (r["ms_per_step"] * 1e-3)
    roofline = {"bound": "alu", "kernel": f"raymarch_kernel ({head})", "achieved": achieved_ops / 1e12,
                "peak": ALU_PEAK / 1e12, "unit": "Tlane-op/s", "frac": achieved_ops / ALU_PEAK,
                "traffic": traffic, "kernel_ms": r["kernel_ms"],
                "work": r["work"],
                "frac_of_measured_fma_rate": achieved_ops / peaks["fma_lane_ops_per_s"],
                "pipelined": {"achieved": piped / 1e12, "frac": piped / ALU_PEAK,
                              "frames_in_flight": r["frames_in_flight"],
                              "note": "the method's work per step over the timed loop's time per step (frames "
                                      "overlapping on streams used in turn); 'achieved' above is one launch alone"},
                "dense_equivalent": {"achieved": dense / 1e12, "frac": dense / ALU_PEAK,
                                     "note": "every nominal sample charged 50 + 22 x 5 lane-ops, skipped ones "
                                             "included: not the work done"},
                "valu_counters": None if rec is None else rec.get("valu"),
                "hbm_algorithmic": {"achieved": achieved_bw / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                                    "frac": achieved_bw / HBM_PEAK,
                                    "frac_of_measured_copy": achieved_bw / peaks["copy_bytes_per_s"]},
                "hbm_measured": None if traffic is None else
                {"achieved": traffic / ksec / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                 "frac": traffic / ksec / HBM_PEAK}}

    serving_result = None
    if not args.no_serving and (wl.n, W_, H_) == (512, 1920, 1080):
        serving_result = serving(args, raypc, torch, W, wl, fields_dev)

    cpu_baseline = None
    if not args.no_cpu_baseline:
        cpu_baseline = cpu_baseline_run(args, wl, head, cam, brushes[0], results[head]["nominal_samples_per_frame"][0])

    line = {
        "metric": "brushed ray-march samples/s (FP16 fields; frames/s, p50/p99 latency and FP32/u8 alongside)",
        "value": r["samples_per_s"],
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"precision study: {wl.n}^3 x {wl.n_fields} fields stored {head}, LOD 3 levels, "
                               f"{W_}x{H_}, step {wl.step} voxel, 5-axis ~10% brush changed every step, ERT 0.99",
                   "volume": wl.n, "fields": wl.n_fields, "width": W_, "height": H_, "step": wl.step,
                   "storage": head, "lod": r["lod"], "frames_in_flight": args.in_flight},
        "frames_per_s": r["frames_per_s"],
        "latency_ms": r["latency_ms"],
        "per_storage": results,
        "roofline": roofline,
        "serving": serving_result,
        "brush_axis_sweep": sweep_result,
        "pc_lines": pc_result,
        "jittered_passes": jit_result,
        "image_warp": warp_result,
        "cpu_baseline": cpu_baseline,
        "peaks": peaks,
    }
    raypc.destroy(ctx)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
