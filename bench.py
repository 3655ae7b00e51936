#!/usr/bin/env python
"""Oriented FAST over an 8-level pyramid of a 1920x1080 frame on one MI355X.

One step = the whole hot path (pyramid, segment test, Harris, NMS, cell and level
selection, orientation) over one synthetic 1920x1080 frame, through the C ABI, with the
frame already resident in HBM.  `value` is frames/s of the fused path (one launch per
step over all levels): K steps between two device synchronisations, the faster of eager
calls and HIP-graph replays.  Beside it, each measured with HIP events on the launching
stream (median of at least 50 runs after 10 warm-ups):

* the plain path (one launch per level and step) on the same frame;
* batched calls: 16 copies of the 1080p frame, the 64-frame mixed batch, 16 frames of
  3840x2160 at 12 levels, and the single 640x480 level with 500 keypoints;
* the served form (32 camera streams, continuous batching): p50/p99 latency at the
  offered 960 frames/s and saturated;
* the Fig. 6/7 pattern frames (1024x1024, 625 copies of one pattern, 1 and 4 levels);
* rBRIEF of the 2000 keypoints;
* per-step kernel durations and the roofline of the longest step;
* the CPU oracle: one thread on the 1080p frame, and frame-parallel over the host's
  cores on the 64-frame and 16 x 4K batches.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# int32 VALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one op per lane per clock).
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
HBM_PEAK_GBPS = 8000.0
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
KERNEL_SOURCES = ("paper_2506_07164_amd/csrc/of_kernels.hip", "paper_2506_07164_amd/csrc/of_plan.h")
COPY_MIB = 256
PROFILE_REPEAT = 10
EVENT_RUNS = 50   # timed runs per leg (median reported)
EVENT_WARMUP = 10


def log(msg):
    print(msg, file=sys.stderr, flush=True)


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


def traffic_file(kernel):
    return os.path.join(ROOT, "profiles", f"{kernel}_1080p_8level_traffic.txt")


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


def event_median_ms(run, stream, runs=EVENT_RUNS, warmup=EVENT_WARMUP):
    """Median milliseconds of `run()` (which queues work on `stream`) over `runs` runs,
    each bracketed by HIP events recorded on `stream`."""
    import torch
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            run()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(runs)]
    with torch.cuda.stream(stream):
        for a, b in evs:
            a.record(stream)
            run()
            b.record(stream)
    torch.cuda.synchronize()
    return statistics.median(a.elapsed_time(b) for a, b in evs)


def capture(run, stream):
    """A HIP graph of `run()` captured on `stream` (after one eager call)."""
    import torch
    with torch.cuda.stream(stream):
        run()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(g, stream=stream):
            run()
    torch.cuda.synchronize()
    return g


def cpu_worker_count():
    """Host threads for the frame-parallel oracle: the cores this process may use, at
    most 16 (a one-GPU machine's share of its host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


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
    return {"value": round(n / el, 4), "unit": "frames/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} runs of the 1920x1080 8-level frame, single-threaded C oracle",
            "cpu": cpu_model()}


def cpu_baseline_parallel(name, imgs, kw):
    """The oracle on every frame of a batch, one frame per thread across the host's
    cores (the C oracle releases the interpreter lock while it runs)."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    p = oracle.params(**kw)
    workers = cpu_worker_count()
    t0 = time.perf_counter()
    with ThreadPoolExecutor(workers) as ex:
        list(ex.map(lambda im: oracle.detect(im, p), imgs))
    el = time.perf_counter() - t0
    return {"value": round(len(imgs) / el, 4), "unit": "frames/s", "cores": workers,
            "kind": "oracle", "sample": f"the {len(imgs)}-frame {name} batch once, one frame "
                                        f"per thread on {workers} threads", "cpu": cpu_model()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="library default launch shape")
    ap.add_argument("--tuning", type=str, default=None,
                    help="launch shape as JSON (of_tuning fields), instead of the autotuner")
    ap.add_argument("--tune-verbose", action="store_true")
    ap.add_argument("--retune", action="store_true", help="search again, ignoring stored results")
    for leg in ("plain", "batched", "serve", "configs", "patterns", "describe"):
        ap.add_argument(f"--no-{leg}", action="store_true", help=f"skip the {leg} leg")
    ap.add_argument("--fused-only", action="store_true",
                    help="only the fused leg and its profile (for profilers)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help=f"only run a {COPY_MIB} MiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.fused_only:
        for leg in ("plain", "batched", "serve", "configs", "patterns", "describe"):
            setattr(args, f"no_{leg}", True)
        args.no_cpu_baseline = True
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
    log(f"# workload {spec.width}x{spec.height} L={kw['n_levels']} N={kw['n_features']}")

    fused = ofhip.Detector([img.shape], p, resident=True)
    stream = torch.cuda.Stream()

    # launch shape of the fused path from the autotuner (outside the timed region)
    tune_fields = None
    if args.tuning:
        tune_fields = {k: int(v) for k, v in json.loads(args.tuning).items()}
    elif not args.no_tune:
        from paper_2506_07164_amd.tune import autotune
        tune_fields = autotune([frame], p, use_cache=not args.retune, verbose=args.tune_verbose)
        log(f"# tuning {tune_fields}")
    tune = ofhip.tuning(**tune_fields) if tune_fields else None

    def fused_step():
        fused.detect_batch([frame], tune=tune, stream=stream)

    # warm-up (eager), then capture the fused step in a graph on `stream`
    with torch.cuda.stream(stream):
        for _ in range(max(1, args.warmup)):
            fused_step()
    torch.cuda.synchronize()
    graph = capture(fused_step, stream)
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()

    # timed: exactly K steps between two synchronisations, eager calls then graph replays
    K = args.steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for _ in range(K):
            fused_step()
    torch.cuda.synchronize()
    t_eager = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for _ in range(K):
            graph.replay()
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t0
    log(f"# fused {K} steps: eager {t_eager * 1e3:.2f} ms, graph {t_graph * 1e3:.2f} ms")
    got_f = fused.results()[0]
    assert len(got_f) == kw["n_features"]

    with torch.cuda.stream(stream):
        fused_ev_ms = event_median_ms(fused_step, stream)
        fused_graph_ev_ms = event_median_ms(graph.replay, stream)

    # plain path: one launch per level and step
    plain_leg = None
    if not args.no_plain:
        plain = ofhip.Detector([img.shape], p)
        ms = event_median_ms(lambda: plain.detect_plain(frame, stream=stream), stream)
        got_p = plain.results()[0]
        for k in ("x", "y", "level", "score", "m10", "m01"):
            assert np.array_equal(got_f[k], got_p[k]), k
        plain_leg = {"ms_median": round(ms, 4), "fps": round(1e3 / ms, 1)}
        log(f"# plain {plain_leg}")
        del plain

    # per-step kernel durations: HIP events attached to each dispatch on its stream;
    # repeatable launches are issued PROFILE_REPEAT times back to back between their
    # events, so the mean is the kernel's duration without the event overhead
    Kq = 200
    ofhip.of_profile_enable(PROFILE_REPEAT)
    with torch.cuda.stream(stream):
        for _ in range(Kq):
            fused_step()
    torch.cuda.synchronize()
    prof = ofhip.of_profile_read()
    ofhip.of_profile_enable(False)
    step_us = {k: (ms / n * 1e3 if n else 0.0) for k, (ms, n) in prof.items()}
    log("# fused step means (us): " + ", ".join(f"{k}={v:.2f}" for k, v in step_us.items()))
    assert len(fused.results()[0]) == kw["n_features"]

    # batched calls, each a graph replay of one of_detect_batch call
    batched = None
    if not args.no_batched or not args.no_configs:
        batched = {}
        cases = []
        if not args.no_batched:
            cases.append(("b16_1080p", [spec] * 16, kw, True))
        if not args.no_configs:
            cases += [("c3_mixed64", CONFIGS["c3"]["frames"], CONFIGS["c3"]["params"], False),
                      ("c4_4k16", CONFIGS["c4"]["frames"], CONFIGS["c4"]["params"], False),
                      ("c1_640x480", CONFIGS["c1"]["frames"], CONFIGS["c1"]["params"], False)]
        for name, specs, ckw, same in cases:
            cp = ofhip.params(**ckw)
            frames = ([frame.clone() for _ in specs] if same else
                      [torch.from_numpy(make_frame(sp)).cuda() for sp in specs])
            cdet = ofhip.Detector([tuple(f.shape) for f in frames], cp, resident=True)
            if same:
                ctune = tune
            elif args.no_tune:
                ctune = None
            else:  # the workload's shipped launch shape (else the library default)
                from paper_2506_07164_amd.tune import autotune
                ctune = ofhip.tuning(**autotune(frames, cp))
            run = lambda: cdet.detect_batch(frames, tune=ctune, stream=stream)
            g = capture(run, stream)
            ms = event_median_ms(g.replay, stream)
            ms_eager = event_median_ms(run, stream)
            res = cdet.results()
            if same:
                for k in ("x", "y", "level", "score", "m10", "m01"):
                    assert all(np.array_equal(r[k], got_f[k]) for r in res), k
            batched[name] = {"frames_per_call": len(frames), "ms_median": round(ms, 4),
                             "ms_median_eager": round(ms_eager, 4),
                             "fps": round(len(frames) * 1e3 / ms, 1),
                             "keypoints": int(sum(len(r) for r in res))}
            log(f"# {name}: {batched[name]}")
            del frames, cdet, g
        torch.cuda.synchronize()

    # served form: 32 camera streams (720x540..1920x1080, 30 fps Poisson each), continuous
    # batching; latency from arrival to host-visible keypoints
    served = None
    if not args.no_serve:
        from paper_2506_07164_amd import serve
        from synth import stream_schedule
        pool = serve.camera_pool(32, 2)
        server = serve.Server(p, hbm_budget=4 << 30, max_batch=16, lanes=3)
        server.warm(sorted({tuple(v[0].shape) for v in pool.values()}))
        frame_of = lambda s_, k_: (pool[(s_, k_ % 2)][0], (s_, k_ % 2))
        serve.run_schedule(server, stream_schedule(32, 0.2, 30.0), frame_of, rate_scale=4.0)
        served = {"workload": "32 streams x 30 fps Poisson, 720x540..1920x1080, 8 levels, N=2000",
                  "runs": []}
        for scale in (1.0, 32.0):
            res, wall = serve.run_schedule(server, stream_schedule(32, 1.0, 30.0), frame_of,
                                           rate_scale=scale)
            assert all(r.status == "ok" for r in res)
            row = serve.summarize(res, wall, 32 * 30.0 * scale)
            row["scale"] = scale
            row["resident_mib"] = round(server.resident / 2**20, 1)
            served["runs"].append(row)
        log(f"# served {served['runs']}")
        del pool, server

    # rBRIEF of the 2000 keypoints (one launch; the pattern is a seeded input)
    describe_us = None
    if not args.no_describe:
        from synth import brief_pattern
        rot, cen = ofhip.of_brief_tables(brief_pattern())
        rot_d, cen_d = torch.from_numpy(rot).cuda(), torch.from_numpy(cen).cuda()
        fused_step()
        torch.cuda.synchronize()
        describe_us = 1e3 * event_median_ms(
            lambda: fused.describe([frame], rot_d, cen_d, tune=tune, stream=stream), stream)
        log(f"# describe 2000 keypoints: {describe_us:.1f} us per call")

    # Fig. 6/7 pattern benchmark: 1024x1024 frames holding 625 copies of one segment-test
    # pattern, 1 and 4 levels, one frame per call
    patterns = None
    if not args.no_patterns:
        from synth import FIG6_CASES, fig6_pattern_image
        patterns = {}
        for levels in (1, 4):
            pp = ofhip.params(n_levels=levels, fast_t=20, fast_t_min=20, cell=0, n_features=2000)
            for case, pos, _ in FIG6_CASES:
                pf = torch.from_numpy(fig6_pattern_image(pos)).cuda()
                pdet = ofhip.Detector([tuple(pf.shape)], pp, resident=True)
                ms = event_median_ms(lambda: pdet.detect_batch([pf], stream=stream), stream)
                patterns[f"{case}_L{levels}"] = {"us": round(ms * 1e3, 2),
                                                  "keypoints": len(pdet.results()[0])}
                del pdet
        log(f"# patterns: {patterns}")

    # roofline of the longest step
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

    mode = "graph" if t_graph <= t_eager else "eager"
    t_best = min(t_graph, t_eager)
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
        "fused": {"fps_eager": round(K / t_eager, 1), "fps_graph": round(K / t_graph, 1),
                  "ms_median_eager": round(fused_ev_ms, 4),
                  "ms_median_graph": round(fused_graph_ev_ms, 4)},
        "plain": plain_leg,
        "batched": batched,
        "served": served,
        "describe_us": round(describe_us, 2) if describe_us else None,
        "fig7_patterns": patterns,
        "tuning": tune_fields,
        "step_us": {k: round(v, 3) for k, v in step_us.items()},
        "hbm_algorithmic_gbps": round((img.nbytes + 32 * kw["n_features"]) * fused_fps / 1e9, 2),
        "roofline": roofline,
    }
    out["hbm_algorithmic_frac"] = round(out["hbm_algorithmic_gbps"] / HBM_PEAK_GBPS, 5)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(img, kw)
        log(f"# cpu baseline {out['cpu_baseline']}")
        par = {}
        for name in ("c3", "c4"):
            imgs = [make_frame(s) for s in CONFIGS[name]["frames"]]
            par[name] = cpu_baseline_parallel(name, imgs, CONFIGS[name]["params"])
            log(f"# cpu baseline {name}: {par[name]}")
        out["cpu_baseline_batched"] = par
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
