#!/usr/bin/env python
"""Benchmark of the fusion path on the 8x1280x720 rig: serving vs plain, one MI355X.

Workload: 4 independent rigs of 8 cameras at 1280x720 (cluttered scene: 200 primitives,
dense near field and sparse far field, 3 % depth outliers, Beta(5, 2) confidence, RGB).
Inputs are synthetic, seeded, and resident in device memory before any timed region.

A step is one pass of the whole fusion path over one batch of input: one frame from each of
the 4 rigs (4 x 7,372,800 pixels).  Timed runs:
  * saturation throughput: steps x 4 frames submitted at once to the continuous-batching
    server (2 lanes, batches of up to 4 frames) -> `value` (input px/s);
  * the same frames through the plain loop (one ff_fuse at a time, each waiting for the
    previous to finish);
  * Poisson arrivals at 30 Hz per rig times each --rates multiplier: p50/p99 latency of
    both paths on the same trace;
  * per-kernel times from HIP events on the plain path (roofline of the dominant kernel);
  * the CPU oracle on one frame (cpu_baseline).
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


def frame_alg_bytes(P, M, S, R, K):
    """Whole-frame algorithmic bytes of the method (three traversals of D and C, one key
    write, one grouping scatter, segmentation/ranking, consistency gathers, output)."""
    return 24 * P + 52 * M + (8 + 4 * (K - 1)) * R + 16 * S


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=25)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames-per-rig", type=int, default=2)
    ap.add_argument("--rates", default="1,8,24", help="Poisson rate multipliers of 30 Hz/rig")
    ap.add_argument("--trace-seconds", type=float, default=2.0)
    ap.add_argument("--lanes", type=int, default=2)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-latency", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(frames would shard across GPUs with no communication; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(2)
    import paper_2602_01035_amd as ff
    from synth import make_config
    from synth.scenes import poisson_arrivals

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
    outs = {rig: [ff.Output(P, rgb=True) for _ in range(n_out)] for rig in range(N_RIGS)}
    params = ff.Params()
    K = params.k_views

    def step_frames(step):
        return [(rig, devs[(rig, step % args.frames_per_rig)]) for rig in range(N_RIGS)]

    srv = ff.Server(hbm_budget_bytes=8 << 30, lanes=args.lanes, max_batch_frames=args.batch,
                    max_pending=1 << 20)
    plain = ff.Server(hbm_budget_bytes=8 << 30, plain=True, max_pending=1 << 20)

    def saturate(server, steps):
        """steps x 4 frames submitted back to back; returns (seconds, frames)."""
        server.reset_stats()
        torch.cuda.synchronize()
        t = time.perf_counter()
        k = 0
        for s in range(steps):
            for rig, d in step_frames(s):
                server.submit(rig, d, outs[rig][k % n_out], params)
                k += 1
        server.drain()
        torch.cuda.synchronize()
        return time.perf_counter() - t, k

    # ------------------------------------------------------------------ warmup + throughput
    saturate(srv, args.warmup)
    saturate(plain, args.warmup)
    dt_srv, n_srv = saturate(srv, args.steps)
    st_srv = srv.stats()
    dt_pl, n_pl = saturate(plain, args.steps)
    st_pl = plain.stats()
    px_srv = n_srv * P / dt_srv
    px_pl = n_pl * P / dt_pl
    log(f"serving {px_srv / 1e9:.2f} Gpx/s ({dt_srv / args.steps * 1e3:.3f} ms/step, "
        f"{st_srv['mean_batch_frames']:.2f} frames/batch); plain {px_pl / 1e9:.2f} Gpx/s")

    # fused points of one step (cells per frame), read back after the run
    S_frames, info = [], []
    for rig in range(N_RIGS):
        r = outs[rig][0].result()
        S_frames.append(r["count"])
        info.append(r["info"])
    M_mean = float(np.mean([i[0] for i in info]))
    S_mean = float(np.mean([i[1] for i in info]))
    R_mean = float(np.mean([i[2] for i in info]))
    key_bits = int(info[0][3])
    fused_per_s = S_mean * n_srv / dt_srv

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

    # ------------------------------------------------------------------ per-kernel times
    ctx = ff.Context(max_pixels=P, max_cameras=8)
    stream = torch.cuda.current_stream()
    d0 = devs[(0, 0)]
    out0 = ff.Output(P, rgb=True)
    for _ in range(2):
        ctx.fuse(d0["cams"], d0["depth"], d0["conf"], d0["rgb"], out=out0)
    ctx.trace(True)
    n_tr = 10
    for _ in range(n_tr):
        ctx.fuse(d0["cams"], d0["depth"], d0["conf"], d0["rgb"], out=out0, stream=stream)
    tr = ctx.trace_read()
    ctx.trace(False)
    r0 = out0.result()
    M0, S0, R0, kb0 = int(r0["info"][0]), int(r0["info"][1]), int(r0["info"][2]), int(r0["info"][3])
    kb = 4 if kb0 <= 32 else 8
    kernels = {}
    for name, v in tr["kernels"].items():
        b = kernel_bytes(name, P, M0, S0, R0, K, kb)
        per_call_ms = v["total_ms"] / max(1, tr["calls"])
        kernels[name] = dict(mean_ms=round(v["mean_ms"], 5), ms_per_frame=round(per_call_ms, 5),
                             alg_bytes=b, gbs=round(b / (v["mean_ms"] * 1e-3) / 1e9, 1) if b else None)
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_frame"])
    frame_ms_kernels = sum(v["ms_per_frame"] for v in kernels.values())
    dk = kernels[dom]
    roofline = {"bound": "hbm", "kernel": dom, "achieved": dk["gbs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(dk["gbs"] / HBM_PEAK_GBS, 4) if dk["gbs"] else None,
                "traffic": None, "alg_bytes_per_launch": dk["alg_bytes"],
                "mean_launch_ms": dk["mean_ms"]}
    B_frame = frame_alg_bytes(P, M0, S0, R0, K)
    frame_roofline = {
        "alg_bytes_per_frame": B_frame,
        "serving_ms_per_frame": dt_srv / n_srv * 1e3,
        "frac_serving": round(B_frame * n_srv / dt_srv / (HBM_PEAK_GBS * 1e9), 4),
        "plain_ms_per_frame": dt_pl / n_pl * 1e3,
        "frac_plain": round(B_frame * n_pl / dt_pl / (HBM_PEAK_GBS * 1e9), 4),
        "kernel_ms_per_frame": round(frame_ms_kernels, 4),
    }

    # ------------------------------------------------------------------ CPU oracle
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import core as O
        fr = frames[(0, 0)]
        c0, w0 = time.process_time(), time.perf_counter()
        O.fuse_frame(fr)
        wall = time.perf_counter() - w0
        cpu_t = time.process_time() - c0
        cpu = {"value": P / wall, "unit": "px/s", "cores": max(1, round(cpu_t / wall)),
               "kind": "oracle",
               "sample": f"1 frame of rig 0 (8 x 1280x720 = {P} px) through the NumPy oracle, "
                         f"{wall:.1f} s wall, {os.cpu_count()} host CPUs visible"}
        log(f"oracle {wall:.1f} s per frame")

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
        "serving": {"px_s": px_srv, "ms_per_frame": dt_srv / n_srv * 1e3,
                    "mean_batch_frames": st_srv["mean_batch_frames"],
                    "p50_ms": st_srv["p50_ms"], "p99_ms": st_srv["p99_ms"]},
        "plain": {"px_s": px_pl, "ms_per_frame": dt_pl / n_pl * 1e3,
                  "p50_ms": st_pl["p50_ms"], "p99_ms": st_pl["p99_ms"]},
        "speedup_serving_vs_plain": px_srv / px_pl,
        "fused_points_per_s": fused_per_s,
        "frame_sizes": {"P": P, "M": M_mean, "S": S_mean, "R": R_mean, "key_bits": key_bits},
        "latency": latency,
        "kernels": kernels,
        "roofline": roofline,
        "frame_roofline": frame_roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
