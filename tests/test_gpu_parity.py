"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit for bit.

Keypoints, moments and R' must match exactly and in order; angles within 1e-5 rad.
Every case prints its name before touching the GPU."""
import numpy as np
import pytest

import oracle
from oracle_pool import detect_many
from parity import assert_same_keypoints
from synth import CONFIGS, FrameSpec, fig6_pattern_image, make_frame

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def hip():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_07164_amd import ofhip
    ofhip.lib()
    return ofhip


def _kw(**kw):
    base = dict(n_levels=8, fast_t=20, fast_t_min=7, cell=30, n_features=2000)
    base.update(kw)
    return base


def run_batch(hip, imgs, kw, tune=None):
    frames = [torch.from_numpy(i).cuda() for i in imgs]
    det = hip.Detector([i.shape for i in imgs], hip.params(**kw))
    det.detect_batch(frames, tune=tune)
    return det.results()


def shipped_tuning(hip, name):
    """The launch shape shipped for benchmark workload `name` on this device (what the
    benchmark runs it with), or None when none is shipped for this device."""
    import json
    from paper_2506_07164_amd import tune
    cfg = CONFIGS[name]
    shapes = [(s.height, s.width) for s in cfg["frames"]]
    with open(tune.SHIPPED) as fh:
        entry = json.load(fh).get(tune._key(shapes, hip.params(**cfg["params"]), tune.device_key()))
    return hip.tuning(**entry["tuning"]) if entry else None


def run_plain(hip, img, kw):
    frame = torch.from_numpy(img).cuda()
    det = hip.Detector([img.shape], hip.params(**kw))
    det.detect_plain(frame)
    return det.results()[0]


# ------------------------------------------------------------ segment test --

def test_segment_test_all_masks(hip):
    """All 2^16 bright and dark circle masks, differences exactly t (inclusive) and
    t - 1 (not classified), through the kernel's segment-test routine."""
    log("case: segment test, 2^16 masks x 2 polarities")
    masks = np.arange(1 << 16, dtype=np.uint32)
    bits = ((masks[:, None] >> np.arange(16)) & 1).astype(np.int32)
    expect = np.array([oracle.run9(int(m)) for m in masks], dtype=np.uint8)
    for sign in (+1, -1):
        circ = np.empty((len(masks), 17), np.uint8)
        circ[:, 0] = 128
        circ[:, 1:] = 128 + sign * 20 * bits
        dev = torch.from_numpy(circ).cuda()
        out = torch.empty(len(masks), dtype=torch.uint8, device="cuda")
        for t_lo, t_hi, want_lo, want_hi in [(20, 20, expect, expect), (7, 21, expect, 0 * expect),
                                             (20, 255, expect, 0 * expect)]:
            hip.of_test_segment(dev.data_ptr(), len(masks), t_lo, t_hi, out.data_ptr(),
                                hip.stream_ptr())
            got = out.cpu().numpy()
            assert np.array_equal(got & 1, want_lo), (sign, t_lo)
            assert np.array_equal(got >> 1, want_hi), (sign, t_hi)


def test_segment_test_random(hip):
    log("case: segment test, random circles and thresholds")
    rng = np.random.Generator(np.random.PCG64(5))
    n = 20000
    circ = rng.integers(0, 256, (n, 17)).astype(np.uint8)
    circ[: n // 2, 1:] = np.clip(circ[: n // 2, :1].astype(int) + rng.integers(-40, 41, (n // 2, 16)),
                                 0, 255)
    dev = torch.from_numpy(circ).cuda()
    out = torch.empty(n, dtype=torch.uint8, device="cuda")
    import bruteforce as bf
    for t_lo, t_hi in [(7, 20), (1, 1), (30, 90)]:
        hip.of_test_segment(dev.data_ptr(), n, t_lo, t_hi, out.data_ptr(), hip.stream_ptr())
        got = out.cpu().numpy()
        for i in range(0, n, 7):
            patch = np.zeros((7, 7), np.uint8)
            patch[3, 3] = circ[i, 0]
            for k, (dx, dy) in enumerate(bf.CIRCLE):
                patch[3 + dy, 3 + dx] = circ[i, 1 + k]
            assert (got[i] & 1) == oracle.segment_test(patch, 3, 3, t_lo), (i, t_lo)
            assert (got[i] >> 1) == oracle.segment_test(patch, 3, 3, t_hi), (i, t_hi)


# ----------------------------------------------------------------- pyramid --

@pytest.mark.parametrize("W,H,L,pad", [(1920, 1080, 8, 0), (641, 479, 4, 3), (3840, 2160, 12, 0)])
def test_pyramid_build(hip, W, H, L, pad):
    log(f"case: pyramid {W}x{H} L={L} pad={pad}")
    img = make_frame(FrameSpec(W, H, 11, 50, 3.0))
    host = np.zeros((H, W + pad), np.uint8)
    host[:, :W] = img
    dev = torch.from_numpy(host).cuda()[:, :W]
    kw = _kw(n_levels=L, n_features=2000 if L < 12 else 5000)
    p = hip.params(**kw)
    d = hip.of_pyramid_desc_get(W, H, p)
    buf = torch.zeros(d.total_bytes, dtype=torch.uint8, device="cuda")
    hip.of_pyramid_build(hip.image_of(dev), p, buf.data_ptr(), hip.stream_ptr())
    host_buf = buf.cpu().numpy()
    ref = oracle.pyramid(img, oracle.params(**kw))
    for l in range(L):
        lv = host_buf[d.offset[l]: d.offset[l] + d.stride[l] * d.height[l]]
        lv = lv.reshape(d.height[l], d.stride[l])[:, : d.width[l]]
        assert np.array_equal(lv, ref[l]), f"level {l}"


# ------------------------------------------------------- detection: small --

SMALL = [(96, 80, 1), (97, 83, 2), (150, 126, 3), (320, 240, 3), (641, 479, 4), (64, 64, 1)]
PARAMS = [dict(cell=30, fast_t_min=7), dict(cell=0, fast_t_min=20), dict(cell=16, fast_t_min=9),
          dict(cell=0, fast_t_min=5)]


@pytest.mark.parametrize("W,H,seed", SMALL)
@pytest.mark.parametrize("pk", range(len(PARAMS)))
def test_small_frames_plain_and_batch(hip, W, H, seed, pk):
    L = 1 if min(W, H) < 100 else (2 if min(W, H) < 200 else 4)
    kw = _kw(n_levels=L, n_features=400, **PARAMS[pk])
    log(f"case: small {W}x{H} seed={seed} {kw}")
    img = make_frame(FrameSpec(W, H, seed, 12, 3.0))
    ref = oracle.detect(img, oracle.params(**kw))
    assert_same_keypoints(run_plain(hip, img, kw), ref, "plain")
    assert_same_keypoints(run_batch(hip, [img], kw)[0], ref, "batch")


# Widest and tallest frames the calls accept, each shorter or narrower than one tile of
# either detection kernel, and the most levels: the last level of the 480x480 frame is
# 31x31, one valid pixel.  With 60 features the levels from 9 up have a quota of 0.
EXTREME = [(16384, 40, 1, 1000, 0), (40, 16384, 1, 1000, 1), (480, 480, 16, 2000, 2),
           (480, 480, 16, 60, 3)]


@pytest.mark.parametrize("W,H,L,N,seed", EXTREME)
def test_extreme_sizes(hip, W, H, L, N, seed):
    kw = _kw(n_levels=L, n_features=N)
    log(f"case: extreme {W}x{H} {kw}")
    img = make_frame(FrameSpec(W, H, seed, max(12, max(W, H) // 40), 2.0, 40.0))
    ref = oracle.detect(img, oracle.params(**kw))
    assert len(ref) > 0
    assert_same_keypoints(run_batch(hip, [img], kw)[0], ref, "batch")
    assert_same_keypoints(run_plain(hip, img, kw), ref, "plain")


@pytest.mark.parametrize("W", [286, 287])
def test_rank_cap_and_largest_quota(hip, W):
    """One whole-level cell over uniform noise with a quota of 4096, the most a level
    takes, and more survivors than that.  The 286x286 frame has exactly 16384 candidate
    slots (one per 2x2 block of its 256x256 valid region), the most the rank-count
    selection takes; 287x286 has one more column of blocks and goes to the radix select
    with appended candidates."""
    kw = _kw(n_levels=1, cell=0, fast_t_min=20, n_features=4096)
    log(f"case: rank cap, {W}x286 noise {kw}")
    img = np.random.default_rng(W).integers(0, 256, (286, W), dtype=np.uint8)
    ref = oracle.detect(img, oracle.params(**kw))
    assert len(ref) == 4096
    assert_same_keypoints(run_batch(hip, [img], kw)[0], ref, "batch")
    assert_same_keypoints(run_plain(hip, img, kw), ref, "plain")


def test_smallest_frame(hip):
    """31x31, the smallest frame the calls accept: one valid pixel, (15, 15)."""
    img = np.full((31, 31), 60, np.uint8)
    img[14:26, 14:26] = 170
    for cell in (30, 0):
        kw = _kw(n_levels=1, cell=cell, n_features=4)
        log(f"case: smallest frame {kw}")
        ref = oracle.detect(img, oracle.params(**kw))
        assert len(ref) == 1
        assert_same_keypoints(run_batch(hip, [img], kw)[0], ref, "batch")
        assert_same_keypoints(run_plain(hip, img, kw), ref, "plain")


def test_batch_of_extremes(hip):
    """One batch holding the smallest frame, the widest, the tallest and a 640x480 frame:
    each frame's keypoints equal the oracle's for that frame alone."""
    sq = np.full((31, 31), 60, np.uint8)
    sq[14:26, 14:26] = 170
    imgs = [sq, make_frame(FrameSpec(16384, 40, 11, 400, 2.0, 40.0)),
            make_frame(FrameSpec(40, 16384, 12, 400, 2.0, 40.0)),
            make_frame(FrameSpec(640, 480, 13, 30, 3.0))]
    kw = _kw(n_levels=1, n_features=1000)
    log(f"case: batch of extremes {[i.shape for i in imgs]} {kw}")
    got = run_batch(hip, imgs, kw)
    for i, img in enumerate(imgs):
        assert_same_keypoints(got[i], oracle.detect(img, oracle.params(**kw)), f"frame {i}")


# Scales and patch radii other than 6/5 and 15: the radius is also the detection border,
# and radii above 15 take the moments' multi-pass path.
SCALES_RADII = [(641, 479, 4, 2, 1, 8), (641, 479, 6, 8, 7, 20), (320, 240, 3, 3, 2, 4),
                (641, 479, 3, 6, 5, 31), (1920, 1080, 8, 6, 5, 48)]


@pytest.mark.parametrize("W,H,L,num,den,r", SCALES_RADII)
def test_other_scales_and_radii(hip, W, H, L, num, den, r):
    kw = _kw(n_levels=L, scale_num=num, scale_den=den, patch_radius=r, n_features=1000)
    log(f"case: scale {num}/{den} radius {r} {W}x{H} {kw}")
    img = make_frame(FrameSpec(W, H, 20 + r, 40, 3.0))
    ref = oracle.detect(img, oracle.params(**kw))
    assert {int(k) for k in ref["level"]} == set(range(L))
    assert_same_keypoints(run_batch(hip, [img], kw)[0], ref, "batch")
    assert_same_keypoints(run_plain(hip, img, kw), ref, "plain")


def test_more_features_than_candidates(hip):
    kw = _kw(n_levels=2, n_features=4000, cell=30)
    log(f"case: quota above candidates {kw}")
    img = make_frame(FrameSpec(200, 160, 3, 6, 2.0))
    ref = oracle.detect(img, oracle.params(**kw))
    assert len(ref) < 4000
    assert_same_keypoints(run_batch(hip, [img], kw)[0], ref, "batch")
    assert_same_keypoints(run_plain(hip, img, kw), ref, "plain")


def test_constant_and_square(hip):
    log("case: constant frame and the square example")
    kw = _kw(n_levels=1, cell=0, fast_t_min=20, n_features=500)
    const = np.full((120, 140), 77, np.uint8)
    assert len(run_batch(hip, [const], kw)[0]) == 0
    assert len(run_plain(hip, const, kw)) == 0
    sq = np.full((64, 64), 60, np.uint8)
    sq[20:44, 20:44] = 160
    got = run_batch(hip, [sq], kw)[0]
    assert [(int(k["x"]), int(k["y"])) for k in got] == [(21, 21), (42, 21), (21, 42), (42, 42)]
    assert set(got["score"].tolist()) == {45_358_400_000_000}


def test_equal_scores_across_cells(hip):
    """Every 30x30 cell holds the same square, so all cell winners tie on R' and the
    level's top N is decided by (y, x) alone, on the rank path with the level staged in
    LDS and without it (a level too large to stage)."""
    tile = np.full((30, 30), 70, np.uint8)
    tile[9:21, 9:21] = 170
    for reps, kw in (((9, 12), _kw(n_levels=1, cell=30, fast_t_min=20, n_features=40)),
                     ((60, 80), _kw(n_levels=1, cell=30, fast_t_min=20, n_features=1500))):
        img = np.ascontiguousarray(np.tile(tile, reps))
        log(f"case: equal scores, {img.shape} {kw}")
        ref = oracle.detect(img, oracle.params(**kw))
        assert len(set(ref["score"].tolist())) <= 4
        assert_same_keypoints(run_batch(hip, [img], kw)[0], ref, "batch")
        assert_same_keypoints(run_plain(hip, img, kw), ref, "plain")
    # three copies of the large case in one call: counting work past the few-frame budget,
    # so its level (4,800 slots, every winner tied) takes the radix select with the ties
    # settled by position
    log(f"case: equal scores, 3 x {img.shape}, radix select")
    for i, got in enumerate(run_batch(hip, [img] * 3, kw)):
        assert_same_keypoints(got, ref, f"batch copy {i}")


@pytest.mark.parametrize("L,N", [(1, 4000), (4, 8000), (1, 2000), (4, 2000)])
def test_fig6_pattern_frames(hip, L, N):
    from test_oracle_pins import _fig6_cases
    for case, pos, corner in _fig6_cases():
        kw = _kw(n_levels=L, cell=0, fast_t_min=20, n_features=N)
        log(f"case: fig6 {case} L={L}")
        img = fig6_pattern_image(pos)
        ref = oracle.detect(img, oracle.params(**kw))
        assert_same_keypoints(run_batch(hip, [img], kw)[0], ref, f"fig6 {case}")
        assert_same_keypoints(run_plain(hip, img, kw), ref, f"fig6 {case} plain")


def test_strided_and_unaligned_frames(hip):
    kw = _kw(n_levels=3, n_features=600)
    log("case: strided / unaligned frames")
    imgs = [make_frame(FrameSpec(331, 250, 40 + i, 20, 3.0)) for i in range(3)]
    host = np.zeros((3, 250, 400), np.uint8)
    for i in range(3):
        host[i, :, 1 + i: 1 + i + 331] = imgs[i]
    dev = torch.from_numpy(host).cuda()
    frames = [dev[i, :, 1 + i: 1 + i + 331] for i in range(3)]
    det = hip.Detector([im.shape for im in imgs], hip.params(**kw))
    det.detect_batch(frames)
    res = det.results()
    refs = [oracle.detect(im, oracle.params(**kw)) for im in imgs]
    for i in range(3):
        assert_same_keypoints(res[i], refs[i], f"strided {i}")
    det1 = hip.Detector([imgs[1].shape], hip.params(**kw))
    det1.detect_plain(frames[1])
    assert_same_keypoints(det1.results()[0], refs[1], "strided plain")


# ------------------------------------------------- detection: the workloads --

def test_c1_plain_and_batch(hip):
    spec = CONFIGS["c1"]["frames"][0]
    kw = CONFIGS["c1"]["params"]
    log(f"case: c1 {spec}")
    img = make_frame(spec)
    ref = oracle.detect(img, oracle.params(**kw))
    assert len(ref) > 50
    assert_same_keypoints(run_plain(hip, img, kw), ref, "c1 plain")
    assert_same_keypoints(run_batch(hip, [img], kw)[0], ref, "c1 batch")
    t = shipped_tuning(hip, "c1")
    if t is not None:
        log("case: c1 batch, shipped launch shape")
        assert_same_keypoints(run_batch(hip, [img], kw, t)[0], ref, "c1 batch (shipped shape)")


def test_c2_plain_and_fused(hip):
    spec = CONFIGS["c2"]["frames"][0]
    kw = CONFIGS["c2"]["params"]
    log(f"case: c2 {spec}")
    img = make_frame(spec)
    ref = oracle.detect(img, oracle.params(**kw))
    assert len(ref) == 2000
    assert_same_keypoints(run_plain(hip, img, kw), ref, "c2 plain")
    assert_same_keypoints(run_batch(hip, [img], kw)[0], ref, "c2 fused")


@pytest.mark.parametrize("tune", [dict(mark_grid=0, det_grid=0), dict(mark_words=1, mark_rows=4),
                                  dict(mark_words=2, mark_rows=64, det_cells_x=8, det_cells_y=1),
                                  dict(det_cells_x=1, det_cells_y=1, mark_grid=7, det_grid=3),
                                  dict(pyr_pass=1), dict(pyr_pass=1, mark_words=1, mark_rows=8,
                                                         mark_grid=64),
                                  dict(mark_order=1), dict(mark_order=1, mark_words=2, mark_rows=48),
                                  dict(mark_order=1, mark_words=3, mark_rows=5, pyr_pass=1),
                                  dict(det_order=1),
                                  dict(mark_order=1, det_order=1, mark_words=2, mark_rows=56),
                                  dict(mark_order=1, det_order=1, det_cells_x=2, det_cells_y=3,
                                       mark_rows=7)])
def test_c2_tunings_agree(hip, tune):
    spec = CONFIGS["c2"]["frames"][0]
    kw = CONFIGS["c2"]["params"]
    log(f"case: c2 tuning {tune}")
    img = make_frame(spec)
    ref = oracle.detect(img, oracle.params(**kw))
    assert_same_keypoints(run_batch(hip, [img], kw, hip.tuning(**tune))[0], ref, str(tune))


def _dense_noise_frame(W=400, H=300, seed=31):
    """Left half uniform noise over 0..255 (the compass pre-test at t = 7 passes about 9
    pixels in 10), right half 128 +- 10 (few t = 20 corners: cells fall back to t = 7)."""
    rng = np.random.default_rng(seed)
    img = rng.integers(0, 256, (H, W), dtype=np.int32)
    img[:, W // 2:] = 128 + rng.integers(-10, 11, (H, W - W // 2))
    return img.astype(np.uint8)


@pytest.mark.parametrize("rows", [5, 6, 9, 13])
@pytest.mark.parametrize("words", [2, 3, 4])
def test_dense_noise_segment_tiles(hip, words, rows):
    """Segment-test tiles whose rows are not a multiple of the 4 waves, on a frame where
    almost every pixel passes the pre-test: each wave's queue fills to its worst case."""
    kw = _kw(n_levels=3, n_features=600)
    tune = dict(mark_words=words, mark_rows=rows)
    log(f"case: dense noise 400x300 {kw} {tune}")
    img = _dense_noise_frame()
    ref = oracle.detect(img, oracle.params(**kw))
    assert len(ref) > 500
    assert_same_keypoints(run_batch(hip, [img], kw, hip.tuning(**tune))[0], ref, str(tune))


@pytest.mark.parametrize("tune", [dict(det_w=8, det_h=8), dict(det_w=64, det_h=32),
                                  dict(det_w=64, det_h=16, pyr_pass=1, det_grid=5),
                                  dict(det_w=64, det_h=32, mark_order=1, det_order=1),
                                  dict(det_w=8, det_h=10, mark_rows=9, det_order=1)])
def test_whole_level_cell_tunings_agree(hip, tune):
    """cell = 0 (one cell per level, K = N_l): output slots per 2x2 block, any tiling."""
    kw = _kw(n_levels=3, cell=0, fast_t=8, fast_t_min=8, n_features=400)
    spec = FrameSpec(641, 479, 5, 60, 2.0, texture_amp=6)
    log(f"case: whole-level cells {spec} {tune}")
    img = make_frame(spec)
    ref = oracle.detect(img, oracle.params(**kw))
    assert len(ref) == 400
    assert_same_keypoints(run_batch(hip, [img], kw, hip.tuning(**tune))[0], ref, str(tune))


@pytest.mark.parametrize("cell", [8, 64, 100, 128])
def test_cell_sizes(hip, cell):
    """Default launch shapes across cell sizes: narrow cells (many per tile) to cells
    wider than a tile budget of 240 pixels (one cell per tile, no per-survivor cell)."""
    kw = _kw(n_levels=3, cell=cell, n_features=600)
    spec = FrameSpec(700, 500, 11 + cell, 80, 2.5)
    log(f"case: cell {cell} {spec}")
    img = make_frame(spec)
    ref = oracle.detect(img, oracle.params(**kw))
    assert_same_keypoints(run_batch(hip, [img], kw)[0], ref, f"cell {cell} batch")
    assert_same_keypoints(run_plain(hip, img, kw), ref, f"cell {cell} plain")


def test_c3_batch(hip):
    specs = CONFIGS["c3"]["frames"]
    kw = CONFIGS["c3"]["params"]
    log(f"case: c3 batch of {len(specs)}")
    refs = detect_many(specs, kw)
    imgs = [make_frame(s) for s in specs]
    res = run_batch(hip, imgs, kw)
    for i, (g, r) in enumerate(zip(res, refs)):
        assert_same_keypoints(g, r, f"c3 frame {i}")
    log("case: c3 batch, separate pyramid pass")
    res = run_batch(hip, imgs, kw, hip.tuning(pyr_pass=1))
    for i, (g, r) in enumerate(zip(res, refs)):
        assert_same_keypoints(g, r, f"c3 frame {i} (pyramid pass)")
    log("case: c3 batch, XCD-band tile order")
    res = run_batch(hip, imgs, kw, hip.tuning(mark_order=1, det_order=1))
    for i, (g, r) in enumerate(zip(res, refs)):
        assert_same_keypoints(g, r, f"c3 frame {i} (bands)")
    t = shipped_tuning(hip, "c3")
    if t is not None:
        log("case: c3 batch, shipped launch shape")
        res = run_batch(hip, imgs, kw, t)
        for i, (g, r) in enumerate(zip(res, refs)):
            assert_same_keypoints(g, r, f"c3 frame {i} (shipped shape)")


def test_c4_batch(hip):
    specs = CONFIGS["c4"]["frames"]
    kw = CONFIGS["c4"]["params"]
    log(f"case: c4 batch of {len(specs)}")
    refs = detect_many(specs, kw)
    imgs = [make_frame(s) for s in specs]
    res = run_batch(hip, imgs, kw)
    for i, (g, r) in enumerate(zip(res, refs)):
        assert_same_keypoints(g, r, f"c4 frame {i}")
    t = shipped_tuning(hip, "c4")
    if t is not None:
        log("case: c4 batch, shipped launch shape")
        res = run_batch(hip, imgs, kw, t)
        for i, (g, r) in enumerate(zip(res, refs)):
            assert_same_keypoints(g, r, f"c4 frame {i} (shipped shape)")


def test_batch_equals_alone(hip):
    kw = _kw(n_levels=4, n_features=800)
    log("case: batch vs alone")
    specs = [FrameSpec(w, h, 70 + i, 40, 2.5) for i, (w, h) in
             enumerate([(400, 300), (257, 199), (512, 384), (333, 333)])]
    imgs = [make_frame(s) for s in specs]
    together = run_batch(hip, imgs, kw)
    for i, img in enumerate(imgs):
        alone = run_batch(hip, [img], kw)[0]
        assert_same_keypoints(together[i], alone, f"frame {i} in batch")
        assert_same_keypoints(alone, oracle.detect(img, oracle.params(**kw)), f"frame {i}")


def test_graph_replay(hip):
    """The batched sequence captured in a HIP graph: every replay (with eager work and
    syncs in between, and new frame contents) equals the eager result."""
    kw = CONFIGS["c2"]["params"]
    log("case: graph capture and replay")
    specs = [FrameSpec(960, 540, 90 + i, 60, 3.0) for i in range(4)]
    imgs = [make_frame(s) for s in specs]
    slots = [torch.empty_like(torch.from_numpy(imgs[0])).cuda() for _ in range(2)]
    det = hip.Detector([imgs[0].shape] * 2, hip.params(**kw))
    for s, im in zip(slots, imgs[:2]):
        s.copy_(torch.from_numpy(im))
    torch.cuda.synchronize()
    det.detect_batch(slots)  # warm-up, loads the kernels
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(g, stream=stream):
            det.detect_batch(slots, stream=stream)
    refs = {i: oracle.detect(imgs[i], oracle.params(**kw)) for i in range(4)}
    for rep, pair in enumerate([(0, 1), (2, 3), (1, 0), (3, 2)]):
        for s, i in zip(slots, pair):
            s.copy_(torch.from_numpy(imgs[i]))
        x = torch.randn(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        res = det.results()
        for k, i in enumerate(pair):
            assert_same_keypoints(res[k], refs[i], f"replay {rep} slot {k}")
        del x


def test_graph_replay_sixteen_frames(hip):
    """Sixteen copies of the 1080p 8-level frame in one call (more entries than the
    arguments carry, so the kernels read the workspace's prefix tables), captured in a
    HIP graph with its planning launch and replayed with eager work in between: every
    frame of every replay equals the oracle."""
    spec, kw = CONFIGS["c2"]["frames"][0], CONFIGS["c2"]["params"]
    log("case: graph replay, 16 x 1080p in one call")
    img = make_frame(spec)
    ref = oracle.detect(img, oracle.params(**kw))
    frames = [torch.from_numpy(img).cuda() for _ in range(16)]
    det = hip.Detector([img.shape] * 16, hip.params(**kw))
    det.detect_batch(frames)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(g, stream=stream):
            det.detect_batch(frames, stream=stream)
    for rep in range(3):
        det.counts.zero_()
        x = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, r in enumerate(det.results()):
            assert_same_keypoints(r, ref, f"replay {rep} frame {i}")
        del x


@pytest.mark.parametrize("which", ["c2", "cell0"])
def test_candidate_counts_match_oracle(hip, which):
    """FAST candidates per level (pixels of the valid region passing the segment test at
    their cell's threshold), read back with of_candidate_counts, equal the oracle's."""
    if which == "c2":
        spec, kw = CONFIGS["c2"]["frames"][0], CONFIGS["c2"]["params"]
    else:
        spec, kw = FrameSpec(641, 479, 5, 60, 2.0, texture_amp=6), \
            _kw(n_levels=3, cell=0, fast_t=8, fast_t_min=8, n_features=400)
    log(f"case: candidate counts {which}")
    img = make_frame(spec)
    p = oracle.params(**kw)
    want = [int(oracle.level_detect(lvl, p, level=l)["cand"].sum())
            for l, lvl in enumerate(oracle.pyramid(img, p))]
    frame = torch.from_numpy(img).cuda()
    det = hip.Detector([img.shape], hip.params(**kw))
    det.detect_batch([frame])
    assert det.candidates([frame])[0].tolist() == want
    det.detect_plain(frame)
    assert det.candidates([frame])[0].tolist() == want


@pytest.mark.parametrize("which", ["c2", "whole-level cells, appended candidates"])
def test_profiling_repeats_keep_results(hip, which):
    """of_profile_enable(n > 1) issues repeatable launches n times back to back for
    timing, the Harris/NMS launch included (its candidate counters are divided back):
    keypoints and candidate counts stay those of the oracle, batched and plain."""
    if which == "c2":
        spec, kw = CONFIGS["c2"]["frames"][0], CONFIGS["c2"]["params"]
    else:  # levels past the rank cap: tiles append their survivors to a counted list
        spec, kw = FrameSpec(700, 500, 9, 80, 2.0, texture_amp=6), \
            _kw(n_levels=2, cell=0, fast_t=8, fast_t_min=8, n_features=3000)
    log(f"case: profiling repeats, {which}")
    img = make_frame(spec)
    p = oracle.params(**kw)
    ref = oracle.detect(img, p)
    want = [int(oracle.level_detect(lvl, p, level=l)["cand"].sum())
            for l, lvl in enumerate(oracle.pyramid(img, p))]
    frame = torch.from_numpy(img).cuda()
    det = hip.Detector([img.shape], hip.params(**kw))
    hip.of_profile_enable(4)
    try:
        det.detect_batch([frame])
        got, counts = det.results()[0], det.candidates([frame])[0].tolist()
        det.detect_plain(frame)
        got_plain, counts_plain = det.results()[0], det.candidates([frame])[0].tolist()
        prof = hip.of_profile_read()
    finally:
        hip.of_profile_enable(0)
    assert prof["harris_nms_cells"][1] > 0
    assert_same_keypoints(got, ref, f"{which} batched, profiled")
    assert_same_keypoints(got_plain, ref, f"{which} plain, profiled")
    assert counts == want and counts_plain == want


def test_resident_plan(hip):
    """plan_resident: identical results call after call (state left zeroed for the next
    call), in a graph with new frame contents, with persistent grids; an overwritten
    workspace yields count -1 instead of a result."""
    kw = CONFIGS["c2"]["params"]
    log("case: resident plan")
    specs = [FrameSpec(960, 540, 120 + i, 60, 3.0) for i in range(3)]
    imgs = [make_frame(s) for s in specs]
    refs = [oracle.detect(i, oracle.params(**kw)) for i in imgs]
    slot = torch.from_numpy(imgs[0]).cuda()
    det = hip.Detector([imgs[0].shape], hip.params(**kw), resident=True)
    for k in range(3):
        slot.copy_(torch.from_numpy(imgs[k]))
        det.detect_batch([slot])
        assert_same_keypoints(det.results()[0], refs[k], f"resident call {k}")
    for tune in (dict(mark_grid=64, det_grid=32), dict(mark_order=1, pyr_pass=1),
                 dict(mark_order=1, det_order=1)):
        for k in range(2):
            slot.copy_(torch.from_numpy(imgs[k]))
            det.detect_batch([slot], tune=hip.tuning(**tune))
            assert_same_keypoints(det.results()[0], refs[k], f"resident {tune} {k}")
    stream = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        det.detect_batch([slot], stream=stream)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=stream):
            det.detect_batch([slot], stream=stream)
    for k in (2, 0, 1):
        slot.copy_(torch.from_numpy(imgs[k]))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert_same_keypoints(det.results()[0], refs[k], f"resident graph replay {k}")
    det.ws.zero_()
    det.detect_batch([slot])
    assert det.counts.cpu().tolist() == [-1]
    plain = hip.Detector([imgs[0].shape], hip.params(**kw))
    plain.ws = det.ws  # a non-resident call on the same workspace re-plans it
    plain.detect_batch([slot])
    assert_same_keypoints(plain.results()[0], refs[1], "after re-plan")
