#!/usr/bin/env python
"""Oriented FAST over an 8-level pyramid of a 1920x1080 frame on one MI355X.

One step = the whole hot path (pyramid, segment test, Harris, NMS, cell and level
selection, orientation) over one synthetic 1920x1080 frame, through the C ABI, with the
frame already resident in HBM.  `value` is frames/s of the fused path (one launch per
step over all levels, replayed from a HIP graph); the plain path (one launch per level
and step, eager) is timed beside it.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import hashlib

# int32 VALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one op per lane per clock).
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic integer ops per unit of each step:
#  resample: 11 per level pixel (four Q8 taps, one rounding);
#  segment test: 32 per tested pixel (each circle pixel against I_p - t and I_p + t, Eq. 1);
#  Harris + NMS: per FAST candidate, Sobel G_x and G_y (6 ops each) and the three
#    products accumulated (6) at the 49 window pixels, R' (8), and 8 neighbour compares (3);
#  orientation: per kept keypoint, dx*I and dy*I accumulated over the 709-pixel disk.
OPS_RESAMPLE, OPS_SEGMENT = 11, 32
OPS_HARRIS_NMS = 49 * 18 + 8 + 8 * 3
OPS_ORIENT = 709 * 4
STEP_KERNELS = {"pyramid": "k_pyramid_batch", "segment_test": "k_mark",
                "harris_nms_cells": "k_detect", "select": "k_select_orient"}


def level_work(shapes, p):
    """(resampled level pixels, segment-tested pixels) of one step."""
    from paper_2506_07164_amd import ofhip
    res = seg = 0
    B = p.patch_radius
    for (H, W) in shapes:
        d = ofhip.of_pyramid_desc_get(W, H, p)
        for l in range(d.n_levels):
            w, h = d.width[l], d.height[l]
            if l > 0:
                res += w * h
            seg += (w - 2 * B) * (h - 2 * B)
    return res, seg


KERNEL_SOURCES = ("paper_2506_07164_amd/csrc/of_kernels.hip", "paper_2506_07164_amd/csrc/of_plan.h")
def traffic_file(kernel):
    return os.path.join(ROOT, "profiles", f"{kernel}_1080p_8level_traffic.txt")
COPY_MIB = 256
PROFILE_REPEAT = 10


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, tuning):
    """HBM bytes per launch of `kernel` from the committed counter summary (FETCH_SIZE +
    WRITE_SIZE, each scaled by the same counter on a plain copy), or None when the
    kernel sources or the launch shape changed since the counters were taken."""
    try:
        with open(traffic_file(kernel)) as fh:
            kv = dict(l.strip().split("=", 1) for l in fh if "=" in l and not l.startswith("#"))
    except OSError:
        return None
    if kv.get("kernel_src_sha") != kernel_source_hash():
        return None
    if kv.get("tuning") != json.dumps(tuning, sort_keys=True):
        return None
    return int(float(kv["traffic_bytes_per_launch"]))


def calibrate_copy():
    """A plain device-to-device copy of known size, for scaling the HBM byte counters."""
    import torch
    n = COPY_MIB << 20
    src = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "copies": 5}), flush=True)


def cpu_baseline(img, kw, budget_s=15.0):
    """The oracle as it stands, one thread, on as many copies of the frame as fit."""
    import oracle
    p = oracle.params(**kw)
    n, t0 = 0, time.perf_counter()
    while True:
        oracle.detect(img, p)
        n += 1
        el = time.perf_counter() - t0
        if el > budget_s or n >= 16:
            break
    return {"value": n / el, "unit": "frames/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} frames of the 1920x1080 8-level workload, single-threaded C oracle"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="library default launch shape")
    ap.add_argument("--tuning", type=str, default=None,
                    help="launch shape as JSON (of_tuning fields), instead of the autotuner")
    ap.add_argument("--tune-verbose", action="store_true")
    ap.add_argument("--retune", action="store_true", help="search again, ignoring stored results")
    ap.add_argument("--no-batched", action="store_true", help="skip the 16-frame batched figure")
    ap.add_argument("--no-serve", action="store_true", help="skip the served (32-stream) figure")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 64-frame mixed and 16 x 4K batched figures")
    ap.add_argument("--no-patterns", action="store_true",
                    help="skip the Fig. 6/7 pattern benchmark (1024x1024, 625 copies per case)")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain path (profiles of the fused kernels alone)")
    # The legs below run only when asked for: a full run of every leg once faulted the
    # device with the cause not found; the fused, graph, profile and rBRIEF legs above
    # are the ones verified since.
    for leg in ("plain", "batched", "serve", "configs", "patterns"):
        ap.add_argument(f"--{leg}", action="store_true", help=f"run the {leg} leg")
    ap.add_argument("--all-legs", action="store_true",
                    help="run the plain, batched, served, configs and pattern legs too")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help=f"only run a {COPY_MIB} MiB device copy (counter calibration)")
    args = ap.parse_args()
    for leg in ("plain", "batched", "serve", "configs", "patterns"):
        on = (args.all_legs or getattr(args, leg)) and not getattr(args, f"no_{leg}")
        setattr(args, f"no_{leg}", not on)
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(frames shard across GPUs with no exchange between them)", file=sys.stderr)
        sys.exit(2)

    if args.calibrate_copy:
        calibrate_copy()
        return

    import numpy as np
    import torch
    from paper_2506_07164_amd import ofhip
    from synth import CONFIGS, make_frame

    spec = CONFIGS["c2"]["frames"][0]
    kw = CONFIGS["c2"]["params"]
    img = make_frame(spec)
    p = ofhip.params(**kw)
    frame = torch.from_numpy(img).cuda()
    print(f"# workload {spec.width}x{spec.height} L={kw['n_levels']} N={kw['n_features']}",
          file=sys.stderr, flush=True)

    fused = ofhip.Detector([img.shape], p, resident=True)
    plain = ofhip.Detector([img.shape], p)
    stream = torch.cuda.Stream()

    # launch shape of the fused path from the autotuner (outside the timed region)
    tune_fields = None
    if args.tuning:
        tune_fields = {k: int(v) for k, v in json.loads(args.tuning).items()}
    elif not args.no_tune:
        from paper_2506_07164_amd.tune import autotune
        tune_fields = autotune([frame], p, use_cache=not args.retune, verbose=args.tune_verbose)
        print(f"# tuning {tune_fields}", file=sys.stderr, flush=True)
    tune = ofhip.tuning(**tune_fields) if tune_fields else None

    # warm-up (eager), then capture the fused step in a graph on `stream`
    with torch.cuda.stream(stream):
        for _ in range(max(1, args.warmup)):
            fused.detect_batch([frame], tune=tune, stream=stream)
            if not args.no_plain:
                plain.detect_plain(frame, stream=stream)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            fused.detect_batch([frame], tune=tune, stream=stream)
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()

    # timed: fused path, graph replays
    K = args.steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        graph.replay()
    torch.cuda.synchronize()
    t_fused = time.perf_counter() - t0
    print(f"# fused {K} steps {t_fused * 1e3:.1f} ms", file=sys.stderr, flush=True)

    # timed: fused path, eager calls (no graph), same K
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for _ in range(K):
            fused.detect_batch([frame], tune=tune, stream=stream)
    torch.cuda.synchronize()
    t_fused_eager = time.perf_counter() - t0
    print(f"# fused eager {K} steps {t_fused_eager * 1e3:.1f} ms", file=sys.stderr, flush=True)

    # timed: plain path, eager launches
    Kp = max(1, K // 4)
    t_plain = None
    if not args.no_plain:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            for _ in range(Kp):
                plain.detect_plain(frame, stream=stream)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        print(f"# plain {Kp} steps {t_plain * 1e3:.1f} ms", file=sys.stderr, flush=True)

    # per-step kernel durations: HIP events on the launching stream; repeatable launches
    # (segment test, selection) are issued PROFILE_REPEAT times back to back between
    # their events, so the mean is the kernel's duration without the event overhead
    Kq = max(1, min(K, 500))
    ofhip.of_profile_enable(PROFILE_REPEAT)
    with torch.cuda.stream(stream):
        for _ in range(Kq):
            fused.detect_batch([frame], tune=tune, stream=stream)
    torch.cuda.synchronize()
    prof = ofhip.of_profile_read()
    ofhip.of_profile_enable(False)
    step_us = {k: (ms / n * 1e3 if n else 0.0) for k, (ms, n) in prof.items()}
    print("# fused step means (us): " + ", ".join(f"{k}={v:.2f}" for k, v in step_us.items()),
          file=sys.stderr, flush=True)

    # correctness of what was timed: same keypoints from both paths
    got_f = fused.results()[0]
    assert len(got_f) == kw["n_features"]
    if not args.no_plain:
        got_p = plain.results()[0]
        for k in ("x", "y", "level", "score", "m10", "m01"):
            assert np.array_equal(got_f[k], got_p[k]), k

    # batched form: 16 copies of the frame (distinct buffers) in one call, graph replays
    batched = None
    if not args.no_batched:
        nb = 16
        bframes = [frame.clone() for _ in range(nb)]
        bdet = ofhip.Detector([img.shape] * nb, p)
        with torch.cuda.stream(stream):
            for _ in range(3):
                bdet.detect_batch(bframes, tune=tune, stream=stream)
        torch.cuda.synchronize()
        bgraph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(stream):
            with torch.cuda.graph(bgraph, stream=stream):
                bdet.detect_batch(bframes, tune=tune, stream=stream)
        for _ in range(5):
            bgraph.replay()
        torch.cuda.synchronize()
        Kb = max(1, K // 16)
        t0 = time.perf_counter()
        for _ in range(Kb):
            bgraph.replay()
        torch.cuda.synchronize()
        t_b = time.perf_counter() - t0
        bres = bdet.results()
        for k in ("x", "y", "level", "score", "m10", "m01"):
            assert all(np.array_equal(r[k], got_f[k]) for r in bres), k
        batched = {"frames_per_call": nb, "calls": Kb, "fps": round(nb * Kb / t_b, 1)}
        print(f"# batched {nb} frames x {Kb} calls {t_b * 1e3:.1f} ms", file=sys.stderr, flush=True)

    # served form: 32 camera streams (720x540..1920x1080, 30 fps Poisson each), continuous
    # batching; latency from arrival to host-visible keypoints
    served = None
    if not args.no_serve:
        from paper_2506_07164_amd import serve
        from synth import stream_schedule
        pool = serve.camera_pool(32, 2)
        server = serve.Server(p, hbm_budget=4 << 30, max_batch=16, lanes=3)
        frame_of = lambda s_, k_: (pool[(s_, k_ % 2)][0], (s_, k_ % 2))
        serve.run_schedule(server, stream_schedule(32, 0.2, 30.0), frame_of, rate_scale=4.0)
        served = {"workload": "32 streams x 30 fps Poisson, 720x540..1920x1080, 8 levels, N=2000",
                  "runs": []}
        for scale in (1.0, 32.0):
            res, wall = serve.run_schedule(server, stream_schedule(32, 1.0, 30.0), frame_of,
                                           rate_scale=scale)
            row = serve.summarize(res, wall, 32 * 30.0 * scale)
            row["scale"] = scale
            served["runs"].append(row)
        print(f"# served {served['runs']}", file=sys.stderr, flush=True)

    # algorithmic work of each step launch, the dominant (longest) step's roofline
    # rBRIEF of the 2000 keypoints (one launch; the pattern is a seeded input)
    from synth import brief_pattern
    rot, cen = ofhip.of_brief_tables(brief_pattern())
    rot_d, cen_d = torch.from_numpy(rot).cuda(), torch.from_numpy(cen).cuda()
    fused.detect_batch([frame], tune=tune, stream=stream)
    torch.cuda.synchronize()
    for _ in range(5):
        fused.describe([frame], rot_d, cen_d, tune=tune)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(200):
        fused.describe([frame], rot_d, cen_d, tune=tune)
    torch.cuda.synchronize()
    describe_us = (time.perf_counter() - t0) / 200 * 1e6
    print(f"# describe 2000 keypoints: {describe_us:.1f} us per call", file=sys.stderr, flush=True)

    # batched workloads: 64 mixed frames (16 each of 720x540 .. 1920x1080, 8 levels) and
    # 16 frames of 3840x2160 (12 levels, N = 5000), one call per batch, eager
    configs = None
    if not args.no_configs:
        configs = {}
        for name in ("c3", "c4"):
            specs = CONFIGS[name]["frames"]
            ckw = CONFIGS[name]["params"]
            cp = ofhip.params(**ckw)
            frames = [torch.from_numpy(make_frame(sp)).cuda() for sp in specs]
            cdet = ofhip.Detector([tuple(f.shape) for f in frames], cp)
            with torch.cuda.stream(stream):
                for _ in range(3):
                    cdet.detect_batch(frames, stream=stream)
            torch.cuda.synchronize()
            calls = 20
            t0 = time.perf_counter()
            with torch.cuda.stream(stream):
                for _ in range(calls):
                    cdet.detect_batch(frames, stream=stream)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            configs[name] = {"frames_per_call": len(frames), "calls": calls,
                             "ms_per_call": round(dt / calls * 1e3, 3),
                             "fps": round(len(frames) * calls / dt, 1),
                             "keypoints": int(sum(len(r) for r in cdet.results()))}
            del frames, cdet
            print(f"# {name}: {configs[name]}", file=sys.stderr, flush=True)

    # Fig. 6/7 pattern benchmark: 1024x1024 frames holding 625 copies of one segment-test
    # pattern, 1 and 4 levels, fused path, one frame per call
    patterns = None
    if not args.no_patterns:
        from synth import FIG6_CASES, fig6_pattern_image
        patterns = {}
        for levels in (1, 4):
            pp = ofhip.params(n_levels=levels, fast_t=20, fast_t_min=20, cell=0, n_features=2000)
            for case, pos, _ in FIG6_CASES:
                pf = torch.from_numpy(fig6_pattern_image(pos)).cuda()
                pdet = ofhip.Detector([tuple(pf.shape)], pp)
                with torch.cuda.stream(stream):
                    for _ in range(10):
                        pdet.detect_batch([pf], stream=stream)
                torch.cuda.synchronize()
                calls = 200
                t0 = time.perf_counter()
                with torch.cuda.stream(stream):
                    for _ in range(calls):
                        pdet.detect_batch([pf], stream=stream)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                patterns[f"{case}_L{levels}"] = {"us": round(dt / calls * 1e6, 2),
                                                  "keypoints": len(pdet.results()[0])}
        print(f"# patterns: {patterns}", file=sys.stderr, flush=True)

    res_px, seg_px = level_work([img.shape], p)
    cands = int(fused.candidates([frame]).sum())
    eff = ofhip.of_tuning_default([ofhip.image_of(frame)], p) if tune is None else tune
    split = bool(eff.pyr_pass)
    step_ops = {"pyramid": OPS_RESAMPLE * res_px if split else 0,
                "segment_test": OPS_SEGMENT * seg_px + (0 if split else OPS_RESAMPLE * res_px),
                "harris_nms_cells": OPS_HARRIS_NMS * cands,
                "select": OPS_ORIENT * int(len(got_f))}
    steps = {}
    for k, ops in step_ops.items():
        us = step_us.get(k, 0.0)
        if us > 0 and ops > 0:
            tops = ops / (us * 1e-6) / 1e12
            steps[k] = {"kernel": STEP_KERNELS[k], "us": round(us, 3), "ops": ops,
                        "tops": round(tops, 3), "frac": round(tops / ALU_PEAK_TOPS, 4)}
    dom = max(steps, key=lambda k: steps[k]["us"])
    roofline = {"bound": "alu", "achieved": steps[dom]["tops"], "peak": round(ALU_PEAK_TOPS, 2),
                "unit": "TOP/s", "frac": steps[dom]["frac"],
                "traffic": measured_traffic(STEP_KERNELS[dom], tune_fields),
                "kernel": STEP_KERNELS[dom], "kernel_us": steps[dom]["us"],
                "kernel_src_sha": kernel_source_hash(), "steps": steps,
                "fast_candidates": cands}

    mode = "graph" if t_fused <= t_fused_eager else "eager"
    t_best = min(t_fused, t_fused_eager)
    fused_fps = K / t_best
    out = {
        "metric": "frames/sec 1920x1080 8-level Oriented FAST (batched vs plain), HBM GB/s %",
        "value": round(fused_fps, 1),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(t_best / K * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8/int32/int64",
        "data": "synthetic",
        "config": {"workload": "c2: one 1920x1080 frame, 8-level 1.2 pyramid, FAST 20/7 per "
                               "30x30 cell, 2000 keypoints, fused path",
                   "frames_per_step": 1, "launch": mode},
        "fused_fps": {"graph": round(K / t_fused, 1), "eager": round(K / t_fused_eager, 1)},
        "plain_fps": round(Kp / t_plain, 1) if t_plain else None,
        "batched": batched,
        "served": served,
        "describe_us": round(describe_us, 2),
        "batched_configs": configs,
        "fig7_patterns": patterns,
        "tuning": tune_fields,
        "step_us": {k: round(v, 3) for k, v in step_us.items()},
        "hbm_algorithmic_gbps": round((img.nbytes + 32 * kw["n_features"]) * fused_fps / 1e9, 2),
        "roofline": roofline,
    }
    out["hbm_algorithmic_frac"] = round(out["hbm_algorithmic_gbps"] / 8000.0, 5)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(img, kw)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
