#!/usr/bin/env python
"""Benchmark of the fusion path on the 8x1280x720 rig: serving vs plain, one MI355X.

Workload: 4 independent rigs of 8 cameras at 1280x720 (cluttered scene: 200 primitives,
dense near field and sparse far field, 3 % depth outliers, Beta(5, 2) confidence, RGB).
Inputs are synthetic, seeded, and resident in device memory before any timed region.

A step is one pass of the whole fusion path over one batch of input: one frame from each of
the 4 rigs (4 x 7,372,800 pixels).  Timed runs:
  * saturation throughput: steps x 4 frames submitted at once to the continuous-batching
    server (4 lanes, batches of up to 2 frames: the fastest of a sweep over lanes x batch)
    -> `value` (input px/s);
  * the same frames through the plain loop (one ff_fuse at a time, each waiting for the
    previous to finish);
  * Poisson arrivals at 30 Hz per rig times each --rates multiplier: p50/p99 latency of
    both paths on the same trace;
Before them, every input frame goes once through ff_fuse (its M, S, R give the algorithmic
bytes) and one frame is traced kernel by kernel (HIP events) to name the dominant kernel.
After them, a timed region of the same steps in the serving batch size, batched calls one
after another on the caller's stream, times that kernel alone with events around it
(roofline), and the CPU oracle runs on a bounded sample (cpu_baseline); the same frames go
through the server in the timed configuration and are checked against the oracle's output.
Beside the headline: the two workloads whose inputs exceed the last-level cache (the
30-frame 16-camera sequence in batched calls; rigs of 2/6/12/32 cameras served at saturation
and as a 30 Hz Poisson stream for --c5-seconds, p50/p99 against the plain loop), each with
its fraction of the HBM roofline; a 1/2/4/8-camera sweep at 1280x720; and the oracle on the
two small configurations in full and on one 16-camera frame, each checked against the GPU.
--copy-calibration MiB first runs a plain elementwise copy (read N, write N bytes) so that
hardware byte counters of the same profiled run can be scaled.
Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "input depth px/s & p50/p99 frame latency, 8x1280x720 rig; serving vs plain"
HBM_PEAK_GBS = 8000.0
N_RIGS = 4


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# algorithmic bytes per launch of each kernel, from the frame sizes (P pixels, M gated
# points, S cells, R representatives, K view budget, key bytes kb)
def kernel_bytes(name, P, M, S, R, K, kb):
    if name in ("backproject_aabb", "coarse_hist"):
        return 8 * P                                   # read depth + confidence
    if name == "keys":
        return 8 * P + (kb + 4) * M                    # read D, C; write key + pixel id
    if name.startswith("radix_up"):
        return kb * M                                  # read keys
    if name.startswith("radix_down"):
        return 2 * (kb + 4) * M                        # read and write keys + ids
    if name == "head_count":
        return kb * M                                  # read sorted keys
    if name == "head_write":
        return kb * M + 4 * S + 4 * S                  # read keys; write starts; frame ids
    if name == "cells_top3_consistency_fuse":
        return (4 * S + 8 * M + (8 + 4 * (K - 1)) * R + 3 * R
                + (12 + 4 + 3 + 4 + 12 + 8) * S)       # gathers + all per-cell outputs
    return 0


# Hardware byte counters of the dominant kernel, from two rocprofv3 --pmc passes (FETCH_SIZE,
# then WRITE_SIZE) over the launches that the roofline region times: batched calls of two
# 8x1280x720 frames.  Each pass is scaled by what the same counter reads for a plain copy
# kernel of known size (1 GiB read, 1 GiB written: FETCH_SIZE reads 0.5 GiB, WRITE_SIZE
# 1 GiB).  Valid only for the kernel sources they were taken on (their digest) and for
# launches of that many frames; otherwise the traffic is reported as null.
COUNTERS = {
    "kernel": "cells_top3_consistency_fuse",
    "source_digest": "c42fb2f44b61f40e",
    "frames_per_launch": 2,
    "fetch_kib_per_launch": 203482.3,
    "write_kib_per_launch": 106585.9,
    "fetch_scale": 2.0,
    "write_scale": 1.0,
    # SQ_INSTS_VALU of the same launches (rocprofv3 --pmc): VALU wave-instructions issued
    "valu_wave_instr_per_launch": 118.27e6,
}
# VALU issue peak: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 VALU instruction per SIMD every
# 4 cycles (16 lanes wide; packed FP32 disabled)
VALU_PEAK_G_PER_S = 256 * 4 * 2.4 / 4


def kernel_source_digest():
    """Digest of the device sources' code (comments and whitespace removed)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in ("common.hpp", "phases.hpp", "fuseflow.hip"):
        with open(os.path.join(ROOT, "paper_2602_01035_amd", "csrc", name)) as f:
            src = f.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def frame_alg_bytes(P, M, S, R, K):
    """Whole-frame algorithmic bytes of the method (three traversals of D and C, one key
    write, one grouping scatter, segmentation/ranking, consistency gathers, output)."""
    return 24 * P + 52 * M + (8 + 4 * (K - 1)) * R + 16 * S


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def serving_parity(ff, torch, np, O, frames, devs, oracle_out, P, params, args):
    """The oracle's frames through the continuous-batching server in the timed configuration:
    count, keys, member counts and representatives bit for bit, fused coordinates and
    weights within 1e-5 (relative; floors 1 m and 1e-6), colours within 1."""
    srv = ff.Server(hbm_budget_bytes=8 << 30, lanes=args.lanes, max_batch_frames=args.batch)
    outs = [ff.Output(P, rgb=True) for _ in devs]
    for i, d in enumerate(devs):
        srv.submit(i, d, outs[i], params)
    srv.drain()
    srv.close()
    ok, worst_xyz, worst_w = True, 0.0, 0.0
    for o, g in zip(oracle_out, (x.result() for x in outs)):
        good, ex, ew = compare_to_oracle(np, g, o)
        ok = ok and good
        worst_xyz, worst_w = max(worst_xyz, ex), max(worst_w, ew)
    return {"frames": len(devs), "ok": bool(ok), "max_rel_xyz_err": worst_xyz,
            "max_rel_weight_err": worst_w}


MALL_BYTES = 256 << 20
WARM_SECONDS = 0.5      # untimed work before each larger-workload measurement
C4_FRAMES = 30          # length of the 16-camera dynamic sequence


def render_inputs(name, frame, rig=0):
    """The inputs of one synthetic frame (cameras, depth, confidence, colour) in a form that
    crosses a process pool cheaply (no ground-truth layers)."""
    import types
    from synth import make_config
    f = make_config(name, frame=frame, rig=rig)
    return types.SimpleNamespace(cams=f.cams, depth=f.depth, conf=f.conf, rgb=f.rgb)


def compare_to_oracle(np, g, o):
    """count, keys, member counts and representatives bit for bit; fused coordinates and
    weights within 1e-5 (relative; floors 1 m and 1e-6); colours within 1."""
    same = (g["status"] == 0 and g["count"] == len(o["keys"]) and
            all(np.array_equal(g[k], o[k]) for k in ("keys", "n_members", "reps")))
    scale = np.maximum(np.abs(o["xyz"]).max(axis=1), 1.0) if len(o["keys"]) else 1.0
    ex = float((np.abs(g["xyz"].astype(np.float64) - o["xyz"]).max(axis=1) / scale).max()) \
        if len(o["keys"]) else 0.0
    ew = float((np.abs(g["weight"].astype(np.float64) - o["weight"]) /
                np.maximum(o["weight"], 1e-6)).max()) if len(o["keys"]) else 0.0
    rgb_ok = (g.get("rgb") is None or o.get("rgb") is None or not len(o["keys"]) or
              int(np.abs(g["rgb"].astype(int) - o["rgb"].astype(int)).max()) <= 1)
    return same and ex <= 1e-5 and ew <= 1e-5 and rgb_ok, ex, ew


def frame_sizes(ff, dev, params, stream):
    """P, M, S, R of one frame (one ff_fuse call of its own), for the algorithmic bytes."""
    P = sum(int(c.width) * int(c.height) for c in dev["cams"])
    ctx = ff.Context(max_pixels=P, max_cameras=len(dev["cams"]))
    o = ff.Output(P)
    ctx.fuse(dev["cams"], dev["depth"], dev["conf"], None, params=params, out=o, stream=stream)
    info = o.result()["info"]
    ctx.close()
    return dict(P=P, M=int(info[0]), S=int(info[1]), R=int(info[2]))


def run_regimes(ff, torch, params, stream, args, c4_host):
    """Throughput of the two larger workloads, whose inputs per call or step exceed the
    256 MB last-level cache (one headline frame's 81 MB of inputs fits it); each is the
    median of three timed runs after half a second of untimed work:
      * 16 cameras at mixed resolutions (6 x 640x480, 6 x 1280x720, 4 x 1920x1080): the
        30 frames of the moving-sphere sequence, two frames per batched call
        (ff_fuse_batch, replayed from a hipGraph), with the tile and digit sizes the
        autotuner picks for that batch shape;
      * rigs of 2, 6, 12 and 32 cameras (resolutions drawn from 640x480, 1280x720,
        1920x1080) through the continuous-batching server at saturation and through the
        plain loop, then the Poisson stream of those rigs at 30 Hz."""
    import numpy as np
    from synth import make_config
    res = {}
    t0 = time.time()
    seq = [ff.to_device(f) for f in c4_host]
    nseq = len(seq)
    P16 = sum(int(c.width) * int(c.height) for c in seq[0]["cams"])
    in_bytes = sum(t.numel() * t.element_size() for d in seq[:2]
                   for t in d["depth"] + d["conf"] + d["rgb"])
    ctx = ff.Context(max_pixels=2 * P16, max_cameras=32, max_frames=2)
    outs = [ff.Output(P16, rgb=True) for _ in range(2)]
    tuned = ctx.autotune(seq[:2], params=params, outs=outs, stream=stream)
    pairs = [seq[i:i + 2] for i in range(0, nseq - 1, 2)]
    # the GPU idled while the frames were rendered: keep it saturated for a while (clocks
    # ramp up over tens of milliseconds) before timing, then take the median of three runs
    t_end = time.perf_counter() + WARM_SECONDS
    while time.perf_counter() < t_end:
        for pr in pairs[:8]:
            ctx.fuse_batch(pr, params=params, outs=outs, stream=stream)
        torch.cuda.synchronize()
    reps = max(1, args.steps // (2 * len(pairs)))     # passes over the sequence per run

    def timed():
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            for pr in pairs:
                ctx.fuse_batch(pr, params=params, outs=outs, stream=stream)
        torch.cuda.synchronize()
        return time.perf_counter() - t

    runs = sorted(timed() for _ in range(3))
    dt = runs[1]
    ctx.close()
    K = params.k_views
    zs = [frame_sizes(ff, d, params, stream) for d in seq[:2 * len(pairs)]]
    B_pass = sum(frame_alg_bytes(z["P"], z["M"], z["S"], z["R"], K) for z in zs)
    nfr = reps * 2 * len(pairs)
    res["mixed16_batched"] = {
        "sequence_frames": 2 * len(pairs), "passes_per_run": reps,
        "alg_bytes_per_frame": B_pass / len(zs),
        "frac_hbm": round(reps * B_pass / dt / (HBM_PEAK_GBS * 1e9), 4),
        "px_s": nfr * P16 / dt, "ms_per_frame": dt / nfr * 1e3,
        "fused_points_per_s": reps * sum(z["S"] for z in zs) / dt,
        "pixels_per_frame": P16, "frames_per_call": 2, "tuning": tuned,
        "runs_ms_per_frame": [round(r / nfr * 1e3, 4) for r in runs],
        "input_mb_per_call": round(in_bytes / 1e6, 1),
        "regime": "HBM: inputs exceed the 256 MB last-level cache" if in_bytes > MALL_BYTES
                  else "inputs fit the 256 MB last-level cache"}
    del seq, pairs
    torch.cuda.empty_cache()

    rigs = [ff.to_device(make_config("c5", rig=r)) for r in range(4)]
    Pr = [sum(int(c.width) * int(c.height) for c in d["cams"]) for d in rigs]
    zr = [frame_sizes(ff, d, params, stream) for d in rigs]
    service = []
    for d, p in zip(rigs, Pr):
        # one rig's frame alone through ff_fuse, calls back to back (graph replay)
        sctx = ff.Context(max_pixels=p, max_cameras=len(d["cams"]))
        so = ff.Output(p, rgb=True)
        for _ in range(3):
            sctx.fuse(d["cams"], d["depth"], d["conf"], d["rgb"], params=params, out=so,
                      stream=stream)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(10):
            sctx.fuse(d["cams"], d["depth"], d["conf"], d["rgb"], params=params, out=so,
                      stream=stream)
        torch.cuda.synchronize()
        service.append(round((time.perf_counter() - t) / 10 * 1e3, 4))
        sctx.close()
    B_step = sum(frame_alg_bytes(z["P"], z["M"], z["S"], z["R"], K) for z in zr)
    in_bytes = sum(t.numel() * t.element_size() for d in rigs
                   for t in d["depth"] + d["conf"] + d["rgb"])
    routs = [[ff.Output(p, rgb=True) for _ in range(2)] for p in Pr]
    row = {"cameras": [len(d["cams"]) for d in rigs], "pixels_per_frame": Pr,
           "ms_per_frame_alone": service,
           "input_mb_per_step": round(in_bytes / 1e6, 1),
           "regime": "HBM: inputs exceed the 256 MB last-level cache" if in_bytes > MALL_BYTES
                     else "inputs fit the 256 MB last-level cache"}

    def run(srv, steps):
        srv.reset_stats()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for s in range(steps):
            for i, d in enumerate(rigs):
                srv.submit(i, d, routs[i][s % 2], params)
        srv.drain()
        torch.cuda.synchronize()
        return time.perf_counter() - t

    steps = max(4, args.steps // 2)
    for name, kw in (("serving", dict(lanes=args.lanes, max_batch_frames=args.batch)),
                     ("plain", dict(plain=True))):
        srv = ff.Server(hbm_budget_bytes=64 << 30, max_pending=1 << 20, **kw)
        nb = 1 if kw.get("plain") else min(2, args.batch)
        srv.reserve(nb * max(Pr), nb * max(len(d["cams"]) for d in rigs), nb)
        t_end = time.perf_counter() + WARM_SECONDS
        while time.perf_counter() < t_end:
            run(srv, 2)
        runs = []
        for _ in range(3):
            runs.append((run(srv, steps), srv.stats()["mean_batch_frames"]))
        dt, mbf = sorted(runs)[1]
        row[name] = {"px_s": steps * sum(Pr) / dt, "steps": steps, "mean_batch_frames": mbf,
                     "frac_hbm": round(steps * B_step / dt / (HBM_PEAK_GBS * 1e9), 4),
                     "runs_px_s": [steps * sum(Pr) / r for r, _ in runs]}
        srv.close()
    row["speedup_serving_vs_plain"] = row["serving"]["px_s"] / row["plain"]["px_s"]
    row["alg_bytes_per_step"] = B_step
    # the serving stream itself: Poisson arrivals at 30 Hz per rig (seeds 7000 + rig) for
    # args.c5_seconds, the same trace through the server and through the plain loop (each
    # rig's one rendered frame stands for all of its time steps)
    if args.c5_seconds > 0:
        from synth.scenes import poisson_arrivals
        trace = sorted((float(a), r) for r in range(4)
                       for a in poisson_arrivals(30.0, args.c5_seconds, 7000 + r))
        tr = {"rate_hz_per_rig": 30.0, "seconds": args.c5_seconds, "frames": len(trace),
              "offered_px_s": sum(Pr[r] for _, r in trace) / args.c5_seconds}
        for name, kw in (("serving", dict(lanes=args.lanes, max_batch_frames=args.batch)),
                         ("plain", dict(plain=True))):
            # every lane sized up front for its largest batch: two frames of the largest
            # rig (the plain loop: one); 64 GB of the 288 GB
            srv = ff.Server(hbm_budget_bytes=64 << 30, max_pending=1 << 20, **kw)
            nb = 1 if kw.get("plain") else min(2, args.batch)
            srv.reserve(nb * max(Pr), nb * max(len(d["cams"]) for d in rigs), nb)
            count = [0] * 4
            # untimed: the first two seconds of the same trace (workspaces sized, graphs
            # captured for each lane and shape met), then the whole trace timed
            for span in (min(2.0, args.c5_seconds), None):
                srv.reset_stats()
                lead = srv.now() + 0.2
                for a, r in trace:
                    if span is not None and a >= span:
                        break
                    srv.submit(r, rigs[r], routs[r][count[r] % 2], params, arrival_s=lead + a)
                    count[r] += 1
                srv.drain()
            st = srv.stats()
            rig_ids, lat = srv.latencies()
            per_rig = {}
            for r in range(4):
                v = np.sort(lat[rig_ids == r])
                if len(v):
                    per_rig[f"{len(rigs[r]['cams'])}_cams"] = dict(
                        frames=len(v), p50_ms=round(float(v[int(np.ceil(0.5 * len(v))) - 1]), 4),
                        p99_ms=round(float(v[int(np.ceil(0.99 * len(v))) - 1]), 4))
            tr[name] = dict(p50_ms=round(st["p50_ms"], 4), p99_ms=round(st["p99_ms"], 4),
                            mean_ms=round(st["mean_ms"], 4), max_ms=round(st["max_ms"], 4),
                            frames=int(st["frames"]),
                            mean_batch_frames=round(st["mean_batch_frames"], 3),
                            hbm_peak_bytes=int(st["hbm_peak_bytes"]), per_rig=per_rig)
            srv.close()
        row["poisson_30hz"] = tr
        log(f"rigs 2/6/12/32 at 30 Hz: serving p50 {tr['serving']['p50_ms']:.2f} / p99 "
            f"{tr['serving']['p99_ms']:.2f} ms; plain p50 {tr['plain']['p50_ms']:.2f} / p99 "
            f"{tr['plain']['p99_ms']:.2f} ms")
    res["rigs_2_6_12_32_served"] = row
    log(f"larger workloads in {time.time() - t0:.1f} s: 16 mixed cameras "
        f"{res['mixed16_batched']['px_s'] / 1e9:.2f} Gpx/s; rigs 2/6/12/32 serving "
        f"{row['serving']['px_s'] / 1e9:.2f} Gpx/s, plain {row['plain']['px_s'] / 1e9:.2f}")
    return res


def camera_sweep(ff, torch, dev, params, stream, args):
    """Cost against camera count: the first 1, 2, 4 and 8 cameras of a headline frame
    (1280x720 each) through ff_fuse, calls back to back on one stream (median of three
    timed runs), plus the summed kernel time of one call from the per-kernel trace, and the
    least-squares line of time per frame against the camera count."""
    import numpy as np
    rows = {}
    calls = max(10, args.steps // 2)
    for n in (1, 2, 4, 8):
        sub = {k: v[:n] for k, v in dev.items()}
        P = sum(int(c.width) * int(c.height) for c in sub["cams"])
        ctx = ff.Context(max_pixels=P, max_cameras=n)
        out = ff.Output(P, rgb=True)

        def call():
            ctx.fuse(sub["cams"], sub["depth"], sub["conf"], sub["rgb"], params=params,
                     out=out, stream=stream)

        for _ in range(5):
            call()
        torch.cuda.synchronize()
        runs = []
        for _ in range(3):
            t = time.perf_counter()
            for _ in range(calls):
                call()
            torch.cuda.synchronize()
            runs.append((time.perf_counter() - t) / calls)
        ctx.trace(True)
        for _ in range(5):
            call()
        tr = ctx.trace_read()
        ctx.trace(False)
        info = out.result()["info"]
        ctx.close()
        dt = sorted(runs)[1]
        rows[n] = {"pixels": P, "ms_per_frame": round(dt * 1e3, 4), "px_s": P / dt,
                   "kernel_ms_per_frame": round(sum(v["total_ms"] for v in tr["kernels"].values())
                                                / max(1, tr["calls"]), 4),
                   "M": int(info[0]), "S": int(info[1])}
    ns = np.array(sorted(rows), dtype=np.float64)
    ts = np.array([rows[int(n)]["ms_per_frame"] for n in ns])
    slope, icpt = np.polyfit(ns, ts, 1)
    fit = slope * ns + icpt
    log("cameras 1/2/4/8: " + ", ".join(f"{rows[int(n)]['ms_per_frame']:.3f}" for n in ns)
        + f" ms per frame; {slope:.4f} ms per camera + {icpt:.4f} ms")
    return {"frames": {str(n): v for n, v in rows.items()}, "calls_per_run": calls,
            "fit_ms_per_camera": round(float(slope), 5), "fit_intercept_ms": round(float(icpt), 5),
            "fit_max_rel_residual": round(float(np.max(np.abs(ts - fit) / ts)), 4)}


def oracle_configs(ff, np, O, params, stream, c4_frame):
    """The oracle on the two small configurations in full (2 x 320x240; 4 x 640x480) and
    on one 16-camera frame (15.7 Mpx), each checked against ff_fuse on the same frame."""
    from synth import make_config
    res = {}
    for name, host in (("c1_2x320x240", make_config("c1")), ("c2_4x640x480", make_config("c2")),
                       ("c4_16_mixed_frame0", c4_frame)):
        P = sum(int(c.width) * int(c.height) for c in host.cams)
        c0, w0 = time.process_time(), time.perf_counter()
        o = O.fuse_frame(host)
        wall = time.perf_counter() - w0
        cpu_t = time.process_time() - c0
        dev = ff.to_device(host)
        ctx = ff.Context(max_pixels=P, max_cameras=len(host.cams))
        out = ff.Output(P, rgb=True)
        ctx.fuse(dev["cams"], dev["depth"], dev["conf"], dev["rgb"], params=params, out=out,
                 stream=stream)
        good, ex, ew = compare_to_oracle(np, out.result(), o)
        ctx.close()
        res[name] = {"pixels": P, "seconds": round(wall, 3), "px_s": P / wall,
                     "cores": max(1, round(cpu_t / wall)), "cells": len(o["keys"]),
                     "parity_ok": bool(good), "max_rel_xyz_err": ex, "max_rel_weight_err": ew}
        log(f"oracle {name}: {wall:.2f} s, parity {'ok' if good else 'FAILED'}")
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--frames-per-rig", type=int, default=2)
    ap.add_argument("--rates", default="1,8,12", help="Poisson rate multipliers of 30 Hz/rig")
    ap.add_argument("--trace-seconds", type=float, default=2.0)
    ap.add_argument("--lanes", type=int, default=4)
    ap.add_argument("--batch", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-latency", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MiB",
                    help="run a plain copy kernel of this size first (counter scaling)")
    ap.add_argument("--c5-seconds", type=float, default=10.0,
                    help="length of the 30 Hz Poisson stream of the 2/6/12/32-camera rigs")
    ap.add_argument("--no-regimes", action="store_true",
                    help="skip the two larger workloads (16 mixed cameras; 2/6/12/32 rigs)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (frames "
              "are independent and would shard across GPUs by frame or rig, with no "
              "communication)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    # counting devices does not initialise the GPU; the render workers below are started
    # before anything does (a process that has initialised the GPU starts no programs)
    if torch.cuda.device_count() == 0:
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(2)

    # the 16-camera sequence renders in worker processes (they import only NumPy and the
    # scene generator) while this one renders the headline frames
    c4_jobs, pool = [], None
    if not args.no_regimes or not args.no_cpu_baseline:
        import concurrent.futures as cf
        import multiprocessing as mp
        pool = cf.ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1),
                                      mp_context=mp.get_context("spawn"))
        n4 = C4_FRAMES if not args.no_regimes else 1
        # each submit starts a worker until there are max_workers: all exist after this
        c4_jobs = [pool.submit(render_inputs, "c4", i) for i in range(n4)]
    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(2)
    import paper_2602_01035_amd as ff
    from synth import make_config
    from synth.scenes import poisson_arrivals

    if args.copy_calibration > 0:
        n = args.copy_calibration << 18                      # float32 elements
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.neg(a, out=b)                              # reads 4n bytes, writes 4n
        torch.cuda.synchronize()
        log(f"copy calibration: 3 x {4 * n} bytes read + written")
        del a, b

    # ------------------------------------------------------------------ inputs
    t0 = time.time()
    frames = {}            # (rig, f) -> host frame
    devs = {}
    for rig in range(N_RIGS):
        for f in range(args.frames_per_rig):
            fr = make_config("c3", frame=f, rig=rig)
            frames[(rig, f)] = fr
            devs[(rig, f)] = ff.to_device(fr)
    P = frames[(0, 0)].pixels
    log(f"rendered {len(frames)} frames of {P} px in {time.time() - t0:.1f} s")
    torch.cuda.synchronize()

    n_out = 16
    params = ff.Params()
    K = params.k_views

    # ------------------------------------------------------------------ frame sizes + kernels
    # every input frame once through ff_fuse: M, S, R per frame (for algorithmic bytes) and
    # a per-kernel breakdown (HIP events on the call's stream) that names the dominant kernel
    ctx = ff.Context(max_pixels=P, max_cameras=8)
    stream = torch.cuda.current_stream()
    sizes = {}
    for key, d in devs.items():
        o = ff.Output(P, rgb=True)
        ctx.fuse(d["cams"], d["depth"], d["conf"], d["rgb"], out=o, stream=stream)
        info = o.result()["info"]
        sizes[key] = dict(P=P, M=int(info[0]), S=int(info[1]), R=int(info[2]),
                          kb=4 if int(info[3]) <= 32 else 8)
    d0 = devs[(0, 0)]
    out0 = ff.Output(P, rgb=True)
    # quality of the fused cloud: Eq. 12 against the frame's own depth maps
    ctx.fuse(d0["cams"], d0["depth"], d0["conf"], d0["rgb"], out=out0, stream=stream)
    emc0 = ctx.emc(d0["cams"], d0["depth"], out0, stream=stream)
    ctx.trace(True)
    n_tr = 10
    for _ in range(n_tr):
        ctx.fuse(d0["cams"], d0["depth"], d0["conf"], d0["rgb"], out=out0, stream=stream)
    tr = ctx.trace_read()
    ctx.trace(False)
    ctx.close()
    z = sizes[(0, 0)]
    kernels = {}
    for name, v in tr["kernels"].items():
        b = kernel_bytes(name, P, z["M"], z["S"], z["R"], K, z["kb"])
        kernels[name] = dict(slot=v["slot"], mean_ms=round(v["mean_ms"], 5),
                             ms_per_frame=round(v["total_ms"] / max(1, tr["calls"]), 5),
                             alg_bytes=b,
                             gbs=round(b / (v["mean_ms"] * 1e-3) / 1e9, 1) if b else None)
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_frame"])
    dom_slot = kernels[dom]["slot"]
    frame_ms_kernels = sum(v["ms_per_frame"] for v in kernels.values())
    log(f"dominant kernel {dom} ({kernels[dom]['mean_ms'] * 1e3:.1f} us of "
        f"{frame_ms_kernels * 1e3:.1f} us per frame)")

    outs = {rig: [ff.Output(P, rgb=True) for _ in range(n_out)] for rig in range(N_RIGS)}

    def step_frames(step):
        f = step % args.frames_per_rig
        return [(rig, f) for rig in range(N_RIGS)]

    # every lane's workspace made up front for its largest batch (no workspace is created
    # or grown inside a timed region)
    srv = ff.Server(hbm_budget_bytes=8 << 30, lanes=args.lanes, max_batch_frames=args.batch,
                    max_pending=1 << 20)
    srv.reserve(args.batch * P, args.batch * 8, args.batch)
    plain = ff.Server(hbm_budget_bytes=8 << 30, plain=True, max_pending=1 << 20)
    plain.reserve(P, 8, 1)

    def saturate(server, steps):
        """steps x 4 frames submitted back to back; returns (seconds, frames, alg bytes of
        the dominant kernel over those frames)."""
        server.reset_stats()
        torch.cuda.synchronize()
        t = time.perf_counter()
        k, nbytes = 0, 0
        for s in range(steps):
            for rig, f in step_frames(s):
                server.submit(rig, devs[(rig, f)], outs[rig][s % n_out], params)
                z = sizes[(rig, f)]
                nbytes += kernel_bytes(dom, z["P"], z["M"], z["S"], z["R"], K, z["kb"])
                k += 1
        server.drain()
        torch.cuda.synchronize()
        return time.perf_counter() - t, k, nbytes

    # ------------------------------------------------------------------ warmup + throughput
    saturate(srv, args.warmup)
    saturate(plain, args.warmup)
    dt_srv, n_srv, _ = saturate(srv, args.steps)
    st_srv = srv.stats()
    dt_pl, n_pl, _ = saturate(plain, args.steps)
    st_pl = plain.stats()
    px_srv = n_srv * P / dt_srv
    px_pl = n_pl * P / dt_pl
    log(f"serving {px_srv / 1e9:.2f} Gpx/s ({dt_srv / args.steps * 1e3:.3f} ms/step, "
        f"{st_srv['mean_batch_frames']:.2f} frames/batch); plain {px_pl / 1e9:.2f} Gpx/s")

    M_mean = float(np.mean([z["M"] for z in sizes.values()]))
    S_mean = float(np.mean([z["S"] for z in sizes.values()]))
    R_mean = float(np.mean([z["R"] for z in sizes.values()]))
    S_timed = sum(sizes[(rig, f)]["S"] for s in range(args.steps) for rig, f in step_frames(s))
    fused_per_s = S_timed / dt_srv

    # ------------------------------------------------------------------ latency traces
    latency = []
    if not args.no_latency:
        for mult in [float(x) for x in args.rates.split(",") if x]:
            row = {"rate_hz_per_rig": 30.0 * mult, "offered_px_s": 30.0 * mult * N_RIGS * P}
            for name, server, cap in (("serving", srv, px_srv), ("plain", plain, px_pl)):
                if row["offered_px_s"] > 0.95 * cap:
                    # above this path's saturated throughput the queue grows without bound
                    row[name] = {"overloaded": True}
                    continue
                server.reset_stats()
                lead = server.now() + 0.3
                trace = []
                for rig in range(N_RIGS):
                    for i, a in enumerate(poisson_arrivals(30.0 * mult, args.trace_seconds,
                                                           7000 + rig)):
                        trace.append((a, rig, i))
                trace.sort()
                for a, rig, i in trace:
                    server.submit(rig, devs[(rig, i % args.frames_per_rig)],
                                  outs[rig][i % n_out], params, arrival_s=lead + a)
                server.drain()
                s = server.stats()
                row[name] = dict(p50_ms=round(s["p50_ms"], 4), p99_ms=round(s["p99_ms"], 4),
                                 mean_ms=round(s["mean_ms"], 4), frames=int(s["frames"]),
                                 px_s=s["px_per_s"],
                                 mean_batch_frames=round(s["mean_batch_frames"], 3))
            log(f"rate x{mult:g}: serving {row['serving']}; plain {row['plain']}")
            latency.append(row)
    srv.close()
    plain.close()

    # ------------------------------------------------------------------ roofline
    # The dominant kernel in its own timed region: the same frames in the serving batch size,
    # batched calls one after another on the caller's stream (no other lane shares the GPU:
    # under concurrent lanes a kernel's event-timed duration also counts the time it waits
    # for compute units held by other lanes).  HIP events around that kernel in every call
    # (the probe, on the stream it is launched on); achieved = algorithmic bytes of the frames
    # it processed / its summed duration.
    rctx = ff.Context(max_pixels=P * args.batch, max_cameras=8 * args.batch,
                      max_frames=args.batch)
    routs = [ff.Output(P, rgb=True) for _ in range(args.batch)]

    def roof_calls(steps):
        nbytes = 0
        seq = [k for s in range(steps) for k in step_frames(s)]
        for i in range(0, len(seq), args.batch):
            grp = seq[i:i + args.batch]
            rctx.fuse_batch([devs[k] for k in grp], params=params, outs=routs[:len(grp)],
                            stream=stream)
            for k in grp:
                zk = sizes[k]
                nbytes += kernel_bytes(dom, zk["P"], zk["M"], zk["S"], zk["R"], K, zk["kb"])
        return nbytes

    roof_calls(args.warmup)
    torch.cuda.synchronize()
    rctx.probe(dom_slot)
    dom_bytes = roof_calls(args.steps)
    probe = rctx.probe_read()
    rctx.probe(-1)
    rctx.close()
    mean_launch_ms = probe["total_ms"] / max(1, probe["launches"])
    achieved = dom_bytes / (probe["total_ms"] * 1e-3) / 1e9
    fpl = probe["frames"] / max(1, probe["launches"])
    traffic = None
    if (COUNTERS["kernel"] == dom and COUNTERS["source_digest"] == kernel_source_digest()
            and abs(fpl - COUNTERS["frames_per_launch"]) < 1e-9):
        traffic = round(1024 * (COUNTERS["fetch_kib_per_launch"] * COUNTERS["fetch_scale"] +
                                COUNTERS["write_kib_per_launch"] * COUNTERS["write_scale"]))
    valu = None
    if traffic is not None:
        g = COUNTERS["valu_wave_instr_per_launch"] / (mean_launch_ms * 1e-3) / 1e9
        valu = {"achieved": round(g, 1), "peak": VALU_PEAK_G_PER_S,
                "unit": "G VALU wave-instructions/s", "frac": round(g / VALU_PEAK_G_PER_S, 4)}
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "alg_bytes_per_launch": dom_bytes / max(1, probe["launches"]),
                "mean_launch_ms": round(mean_launch_ms, 5), "launches": probe["launches"],
                "frames_per_launch": fpl, "valu_issue": valu}
    B_frame = frame_alg_bytes(P, z["M"], z["S"], z["R"], K)
    B_timed = sum(frame_alg_bytes(P, sizes[k]["M"], sizes[k]["S"], sizes[k]["R"], K)
                  for s in range(args.steps) for k in step_frames(s))
    frame_roofline = {
        "alg_bytes_per_frame": B_frame,
        "serving_ms_per_frame": dt_srv / n_srv * 1e3,
        "frac_serving": round(B_timed / dt_srv / (HBM_PEAK_GBS * 1e9), 4),
        "plain_ms_per_frame": dt_pl / n_pl * 1e3,
        "frac_plain": round(B_timed / dt_pl / (HBM_PEAK_GBS * 1e9), 4),
        "kernel_ms_per_frame": round(frame_ms_kernels, 4),
    }

    # ------------------------------------------------------------------ copy bandwidth
    # a plain device copy over 4 GiB (far beyond the 256 MB last-level cache): the HBM rate
    # a streaming kernel actually reaches, against which the frame fraction is also given
    ncopy = 1 << 30                                          # float32 elements = 4 GiB
    ca = torch.empty(ncopy, device="cuda")
    cb = torch.empty_like(ca)
    ca.fill_(1.0)
    cb.copy_(ca)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        cb.copy_(ca)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * 4 * ncopy / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del ca, cb
    torch.cuda.empty_cache()
    frame_roofline["copy_gbs"] = round(copy_gbs, 1)
    frame_roofline["frac_serving_vs_copy"] = round(B_timed / dt_srv / (copy_gbs * 1e9), 4)
    log(f"copy {copy_gbs:.0f} GB/s")

    # ------------------------------------------------------------------ larger workloads
    c4_host = [f.result() for f in c4_jobs]
    if pool is not None:
        pool.shutdown()
    regimes = None if args.no_regimes else run_regimes(ff, torch, params, stream, args, c4_host)

    # ------------------------------------------------------------------ camera sweep
    sweep = camera_sweep(ff, torch, devs[(0, 0)], params, stream, args)

    # ------------------------------------------------------------------ CPU oracle
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import core as O
        sample = [(0, f) for f in range(min(2, args.frames_per_rig))]
        c0, w0 = time.process_time(), time.perf_counter()
        oracle_out = [O.fuse_frame(frames[key]) for key in sample]
        wall = time.perf_counter() - w0
        cpu_t = time.process_time() - c0
        cpu = {"value": len(sample) * P / wall, "unit": "px/s",
               "cores": max(1, round(cpu_t / wall)), "kind": "oracle",
               "sample": f"{len(sample)} frame(s) of rig 0 (8 x 1280x720 = {P} px each) "
                         f"through the NumPy oracle, {wall:.1f} s wall, "
                         f"{os.cpu_count()} host CPUs visible ({cpu_model()})"}
        log(f"oracle {wall / len(sample):.1f} s per frame")
        # the same frames through the timed serving configuration, against the oracle
        cpu["parity"] = serving_parity(ff, torch, np, O, [frames[k] for k in sample],
                                       [devs[k] for k in sample], oracle_out, P, params, args)
        log(f"parity of the served frames against the oracle: {cpu['parity']}")
        cpu["other_configs"] = oracle_configs(ff, np, O, params, stream, c4_host[0])

    line = {
        "metric": METRIC, "value": px_srv, "unit": "px/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt_srv / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "4 rigs x 8 cameras x 1280x720 (cluttered 200-primitive scene, "
                               "3% outliers, Beta(5,2) confidence, RGB); a step = one frame "
                               "per rig through the continuous-batching server",
                   "frames_per_step": N_RIGS, "pixels_per_frame": P, "lanes": args.lanes,
                   "max_batch_frames": args.batch, "params": "tau 0.6, K 4, sigma 0.02, "
                   "coarse 64, max level 6, target 16"},
        # saturation: every frame is submitted at once, so completion times measure the queue;
        # frame latency under arrivals is in "latency"
        "serving": {"px_s": px_srv, "ms_per_frame": dt_srv / n_srv * 1e3,
                    "mean_batch_frames": st_srv["mean_batch_frames"],
                    "saturation_p50_ms": st_srv["p50_ms"], "saturation_p99_ms": st_srv["p99_ms"]},
        "plain": {"px_s": px_pl, "ms_per_frame": dt_pl / n_pl * 1e3,
                  "saturation_p50_ms": st_pl["p50_ms"], "saturation_p99_ms": st_pl["p99_ms"]},
        "speedup_serving_vs_plain": px_srv / px_pl,
        "fused_points_per_s": fused_per_s,
        "frame_sizes": {"P": P, "M": M_mean, "S": S_mean, "R": R_mean},
        "emc_mm_rig0": round(emc0["emc_m"] * 1e3, 3),
        "latency": latency,
        "kernels": kernels,
        "roofline": roofline,
        "frame_roofline": frame_roofline,
        "regimes": regimes,
        "camera_sweep": sweep,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
