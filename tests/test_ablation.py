"""Ablation-ladder kernels (GPU): every variant of a step gives the oracle's result.

FAST variants against the oracle's segment test at every pixel; Harris variants against
the oracle's R' at candidate positions (and the dense map at sampled positions)."""
import numpy as np
import pytest

import oracle
from synth import CONFIGS, FrameSpec, make_frame

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


def _level(ofhip, img, pad=0):
    H, W = img.shape
    dev = torch.zeros((H, W + pad), dtype=torch.uint8, device="cuda")
    dev[:, :W] = torch.from_numpy(img).cuda()
    return dev, ofhip.OfImage(dev.data_ptr(), W, H, W + pad)


def _fast_ref(img, t, border):
    H, W = img.shape
    if border == 15:
        p = oracle.params(n_levels=1, fast_t=t, fast_t_min=t, cell=0, n_features=1)
        return oracle.level_detect(img, p)["cand"]
    ref = np.zeros((H, W), np.uint8)
    for y in range(border, H - border):
        for x in range(border, W - border):
            ref[y, x] = oracle.segment_test(img, x, y, t)
    return ref


@pytest.mark.parametrize("shape,t,border,pad", [((160, 200), 20, 15, 0), ((97, 131), 7, 3, 5),
                                                ((64, 70), 1, 3, 3)])
def test_fast_variants_equal_oracle(hip, shape, t, border, pad):
    img = make_frame(FrameSpec(shape[1], shape[0], 31 + t, 30, 2.0, texture_amp=8))
    log(f"case: ablate fast {shape} t={t} border={border}")
    ref = _fast_ref(img, t, border)
    assert ref.sum() > 10
    dev, lv = _level(hip, img, pad)
    out = torch.empty(shape, dtype=torch.uint8, device="cuda")
    for name, v in hip.AB_FAST.items():
        out.fill_(7)
        hip.of_ablate_fast([lv], t, border, v, [out.data_ptr()], 0)
        np.testing.assert_array_equal(out.cpu().numpy(), ref, err_msg=name)


def test_fast_variants_on_the_1080p_frame(hip):
    img = make_frame(CONFIGS["c2"]["frames"][0])
    log("case: ablate fast 1080p")
    ref = _fast_ref(img, 20, 15)
    dev, lv = _level(hip, img)
    out = torch.empty(img.shape, dtype=torch.uint8, device="cuda")
    for name, v in hip.AB_FAST.items():
        hip.of_ablate_fast([lv], 20, 15, v, [out.data_ptr()], 0)
        np.testing.assert_array_equal(out.cpu().numpy(), ref, err_msg=name)


def test_fast_variants_batched_over_levels(hip):
    """One launch over all levels of a pyramid equals the per-level oracle maps."""
    from paper_2506_07164_amd.ablation import build_levels
    img = make_frame(FrameSpec(500, 380, 77, 60, 2.0, texture_amp=8))
    kw = dict(n_levels=5, fast_t=12, fast_t_min=12, cell=0, n_features=10)
    log("case: ablate fast batched over 5 levels")
    frame = torch.from_numpy(img).cuda()
    levels = build_levels([frame], hip.params(**kw), 0)
    refs = [oracle.level_detect(l, oracle.params(**kw), level=i)["cand"]
            for i, l in enumerate(oracle.pyramid(img, oracle.params(**kw)))]
    for name, v in hip.AB_FAST.items():
        outs = [torch.full((lv.height, lv.width), 7, dtype=torch.uint8, device="cuda")
                for _, lv in levels]
        hip.of_ablate_fast([lv for _, lv in levels], 12, 15, v, [o.data_ptr() for o in outs], 0)
        for i, (o, r) in enumerate(zip(outs, refs)):
            np.testing.assert_array_equal(o.cpu().numpy(), r, err_msg=f"{name} level {i}")


def test_harris_variants_equal_oracle(hip):
    img = make_frame(FrameSpec(180, 150, 44, 30, 3.0, texture_amp=8))
    H, W = img.shape
    log("case: ablate harris")
    rng = np.random.default_rng(5)
    xs = rng.integers(0, W, 600)
    ys = rng.integers(0, H, 600)
    xs[:4], ys[:4] = [4, W - 5, 3, W - 4], [4, H - 5, 10, 10]  # edges: in, in, out, out
    pos = torch.from_numpy(((ys.astype(np.uint32) << 16) | xs.astype(np.uint32))).cuda()
    want = np.array([oracle.harris(img, int(x), int(y)) if 4 <= x < W - 4 and 4 <= y < H - 4
                     else 0 for x, y in zip(xs, ys)], np.int64)
    dev, lv = _level(hip, img, 3)
    out = torch.empty(600, dtype=torch.int64, device="cuda")
    out2 = torch.empty(600, dtype=torch.int64, device="cuda")
    for name, v in hip.AB_HARRIS.items():
        if name == "dense_sliding":
            continue
        out.fill_(123)
        hip.of_ablate_harris([lv, lv], [pos.data_ptr(), pos.data_ptr()], [600, 300], v,
                             [out.data_ptr(), out2.data_ptr()], 0)
        np.testing.assert_array_equal(out.cpu().numpy(), want, err_msg=name)
        np.testing.assert_array_equal(out2.cpu().numpy()[:300], want[:300], err_msg=name)
    dense = torch.full((H, W), 123, dtype=torch.int64, device="cuda")
    hip.of_ablate_harris([lv], None, None, hip.AB_HARRIS["dense_sliding"], [dense.data_ptr()], 0)
    d = dense.cpu().numpy()
    np.testing.assert_array_equal(d[ys, xs], want)
    assert (d[:4] == 0).all() and (d[:, -4:] == 0).all()
