"""Ablation ladder: the gain of each design decision of the segment test and the Harris
score, measured on the pyramid levels of the 64-frame mixed batch.

Every level of every frame is built with of_pyramid_build, then each variant of a step
(of_ablate_fast / of_ablate_harris) runs over all of them, 64 levels per launch.  The
time per frame is the summed duration of the kernels themselves (HIP events attached to
each dispatch); the elapsed time of the launch sequence is reported beside it.  Harris runs at the FAST corners (t = 20) of each level.
The table gives each rung's time and its gain over the rung before and over the first,
in the manner of the paper's step-wise table (Table 4).

Run ``python -m paper_2506_07164_amd.ablation``; prints one JSON line.
"""
from __future__ import annotations

import json
import sys

from . import ofhip

FAST_LADDER = [("branchy, global reads", "branchy"), ("bit masks, global reads", "masks"),
               ("bit masks, LDS tile", "masks_lds"),
               ("LDS tile + compass pre-test + bit masks", "masks_pretest_lds"),
               ("LDS tile + compass pre-test + min/max windows", "minmax_lds")]
HARRIS_LADDER = [("2D Sobel, thread per candidate", "2d"),
                 ("separable Sobel, thread per candidate", "separable"),
                 ("8 lanes per candidate, one window row each", "groups")]


def build_levels(frames, p, stream):
    """Device pyramid levels of every frame: list of (tensor, OfImage)."""
    import torch
    levels = []
    for f in frames:
        H, W = f.shape
        d = ofhip.of_pyramid_desc_get(W, H, p)
        buf = torch.empty(d.total_bytes, dtype=torch.uint8, device="cuda")
        ofhip.of_pyramid_build(ofhip.image_of(f), p, buf.data_ptr(), stream)
        for l in range(d.n_levels):
            if l == 0:
                levels.append((f, ofhip.image_of(f)))
            else:
                w, h, s = d.width[l], d.height[l], d.stride[l]
                view = buf[d.offset[l]: d.offset[l] + s * h].view(h, s)
                levels.append((view, ofhip.OfImage(view.data_ptr(), w, h, s)))
    return levels


def timed(fn, reps, step):
    """(kernel us, wall us) per rep: the summed durations of the kernels themselves (HIP
    events attached to their dispatches) and the elapsed time of the launch sequence."""
    import torch
    fn()
    torch.cuda.synchronize()
    ofhip.of_profile_read()
    ofhip.of_profile_enable(1)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record(torch.cuda.current_stream())
    for _ in range(reps):
        fn()
    e.record(torch.cuda.current_stream())
    e.synchronize()
    prof = ofhip.of_profile_read()
    ofhip.of_profile_enable(0)
    return prof[step][0] / reps * 1e3, s.elapsed_time(e) / reps * 1e3


def ladder(rows):
    out, first, prev = [], None, None
    for label, (us, wall) in rows:
        first = us if first is None else first
        out.append({"rung": label, "kernel_us_per_frame": round(us, 2),
                    "launch_sequence_us_per_frame": round(wall, 2),
                    "gain_vs_previous_pct": None if prev is None else round(100 * (prev - us) / prev, 1),
                    "gain_vs_first_pct": round(100 * (first - us) / first, 1)})
        prev = us
    return out


def main(reps=5):
    import numpy as np
    import torch
    from synth import CONFIGS, make_frame
    specs = CONFIGS["c3"]["frames"]
    kw = CONFIGS["c3"]["params"]
    p = ofhip.params(**kw)
    stream = torch.cuda.current_stream().cuda_stream
    frames = [torch.from_numpy(make_frame(s)).cuda() for s in specs]
    levels = build_levels(frames, p, stream)
    torch.cuda.synchronize()
    outs = [torch.empty((lv.height, lv.width), dtype=torch.uint8, device="cuda")
            for _, lv in levels]
    B, t = p.patch_radius, p.fast_t
    lvs = [lv for _, lv in levels]
    chunks = [slice(i, i + 64) for i in range(0, len(lvs), 64)]
    fast = []
    for label, name in FAST_LADDER:
        v = ofhip.AB_FAST[name]

        def run():
            for c in chunks:
                ofhip.of_ablate_fast(lvs[c], t, B, v, [o.data_ptr() for o in outs[c]], stream)
        k_us, w_us = timed(run, reps, "ablate_fast")
        fast.append((label, (k_us / len(frames), w_us / len(frames))))
    # candidates for Harris: the FAST corners of each level (production variant's map)
    for c in chunks:
        ofhip.of_ablate_fast(lvs[c], t, B, ofhip.AB_FAST["minmax_lds"],
                             [o.data_ptr() for o in outs[c]], stream)
    pos, ncand = [], 0
    for o in outs:
        yx = torch.nonzero(o).to(torch.int64)
        pk = ((yx[:, 0] << 16) | yx[:, 1]).to(torch.int32).contiguous()
        pos.append(pk)
        ncand += pk.numel()
    scores = [torch.empty(max(1, q.numel()), dtype=torch.int64, device="cuda") for q in pos]
    harris = []

    def run_points(v):
        for c in chunks:
            ofhip.of_ablate_harris(lvs[c], [q.data_ptr() for q in pos[c]],
                                   [q.numel() for q in pos[c]], v,
                                   [sc.data_ptr() for sc in scores[c]], stream)
    for label, name in HARRIS_LADDER:
        v = ofhip.AB_HARRIS[name]
        k_us, w_us = timed(lambda: run_points(v), reps, "ablate_harris")
        harris.append((label, (k_us / len(frames), w_us / len(frames))))
    dense = [torch.empty((lv.height, lv.width), dtype=torch.int64, device="cuda") for lv in lvs]

    def run_dense():
        for c in chunks:
            ofhip.of_ablate_harris(lvs[c], None, None, ofhip.AB_HARRIS["dense_sliding"],
                                   [d.data_ptr() for d in dense[c]], stream)
    dense_k, dense_w = timed(run_dense, reps, "ablate_harris")
    # the point-wise variants agree with each other and with the dense map
    ref = None
    for label, name in HARRIS_LADDER:
        run_points(ofhip.AB_HARRIS[name])
        got = torch.cat([sc[: q.numel()] for q, sc in zip(pos, scores)]).cpu().numpy()
        ref = got if ref is None else ref
        assert np.array_equal(got, ref), name
    got = torch.cat([d.view(-1)[(q.to(torch.int64) >> 16) * d.shape[1] + (q.to(torch.int64) & 0xffff)]
                     for q, d in zip(pos, dense)]).cpu().numpy()
    assert np.array_equal(got, ref), "dense"
    res = {"workload": "64 mixed frames (16 each of 720x540, 1080x720, 1440x1080, 1920x1080), "
                       "all 8 levels (scale 6/5), FAST t = 20, border 15",
           "levels": len(levels), "fast_corners_per_frame": round(ncand / len(frames), 1),
           "fast": ladder(fast), "harris": ladder(harris),
           "harris_dense_sliding": {"kernel_us_per_frame": round(dense_k / len(frames), 2),
                                    "launch_sequence_us_per_frame": round(dense_w / len(frames), 2)}}
    print(json.dumps(res), flush=True)
    return res


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 5)
