"""The C-ABI library loads and exports every entry point of include/of.h, and its
host-only calls (validation, geometry, workspace sizing) behave.  No GPU needed."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2506_07164_amd import ofhip

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "of.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(of_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ofhip.LIB_PATH):
        import paper_2506_07164_amd.build as b
        b.build()
    return ofhip.lib()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert {"of_pyramid_build", "of_detect", "of_detect_batch"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(lib):
    for s in (ofhip.OF_OK, ofhip.OF_EINVAL, ofhip.OF_ENOSPACE, ofhip.OF_EHIP):
        assert lib.of_status_string(s)


def test_pyramid_desc_matches_oracle_geometry(lib):
    for (W, H, L) in [(1920, 1080, 8), (3840, 2160, 12), (641, 479, 3), (720, 540, 8)]:
        p = ofhip.params(n_levels=L, n_features=2000 if L < 12 else 5000)
        d = ofhip.of_pyramid_desc_get(W, H, p)
        g = oracle.geometry(W, H, oracle.params(n_levels=L, n_features=p.n_features))
        assert list(d.width[:L]) == g["width"].tolist()
        assert list(d.height[:L]) == g["height"].tolist()
        assert list(d.quota[:L]) == g["quota"].tolist()
        for l in range(L):
            assert d.stride[l] >= d.width[l] and d.stride[l] % 64 == 0
            assert d.offset[l] % 256 == 0
        assert d.total_bytes >= d.offset[L - 1] + d.stride[L - 1] * d.height[L - 1]


def test_validation_rejects_bad_arguments(lib):
    good = ofhip.params()
    img = ofhip.OfImage(None, 1920, 1080, 1920)
    assert ofhip.of_workspace_size([img], good) > 0
    bad = [dict(n_levels=0), dict(n_levels=17), dict(fast_t=0), dict(fast_t_min=21),
           dict(cell=7), dict(cell=129), dict(harris_block=5), dict(patch_radius=3),
           dict(scale_num=5, scale_den=5), dict(n_features=0)]
    for kw in bad:
        with pytest.raises(ofhip.OfError) as e:
            ofhip.of_workspace_size([img], ofhip.params(**kw))
        assert e.value.status == ofhip.OF_EINVAL, kw
    # a level smaller than 2 * patch_radius + 1
    with pytest.raises(ofhip.OfError):
        ofhip.of_workspace_size([ofhip.OfImage(None, 30, 400, 30)], ofhip.params(n_levels=1))
    # level quota above 4096
    with pytest.raises(ofhip.OfError):
        ofhip.of_workspace_size([img], ofhip.params(n_levels=1, n_features=5000))
    # batch size limits
    with pytest.raises(ofhip.OfError):
        ofhip.of_workspace_size([], good)
    with pytest.raises(ofhip.OfError):
        ofhip.of_workspace_size([img] * 65, good)


def test_detect_argument_errors_before_any_launch(lib):
    p = ofhip.params(n_levels=1, cell=0, n_features=100, fast_t_min=20)
    img = ofhip.OfImage(0x1000, 64, 64, 64)
    # null workspace / output / capacity below n_features: rejected on the host
    assert lib.of_detect(ctypes.byref(img), ctypes.byref(p), None, 0, 0x1000, 100, 0x1000, None) \
        == ofhip.OF_EINVAL
    assert lib.of_detect(ctypes.byref(img), ctypes.byref(p), 0x1000, 1 << 30, 0x1000, 99, 0x1000,
                         None) == ofhip.OF_EINVAL
    # workspace too small
    assert lib.of_detect(ctypes.byref(img), ctypes.byref(p), 0x1000, 16, 0x1000, 100, 0x1000,
                         None) == ofhip.OF_ENOSPACE
    # stride below width, or at 2^24 (the kernels' rows are 24-bit multiplies)
    for bad in (ofhip.OfImage(0x1000, 64, 64, 63), ofhip.OfImage(0x1000, 64, 64, 1 << 24)):
        assert lib.of_detect(ctypes.byref(bad), ctypes.byref(p), 0x1000, 1 << 30, 0x1000, 100,
                             0x1000, None) == ofhip.OF_EINVAL
    # a frame spanning more than 2^31 - 1 bytes (the resample's 32-bit offsets); the
    # largest stride that still fits is accepted by the host-only size query
    p1 = ofhip.params(n_levels=1, cell=0, n_features=100, fast_t_min=20)
    tall = ofhip.OfImage(0x1000, 64, 16384, 131080)
    assert 131080 * 16383 + 64 > 2**31 - 1 >= 131079 * 16383 + 64
    assert lib.of_detect(ctypes.byref(tall), ctypes.byref(p1), 0x1000, 1 << 40, 0x1000, 100,
                         0x1000, None) == ofhip.OF_EINVAL
    assert lib.of_pyramid_build(ctypes.byref(tall), ctypes.byref(p1), 0x1000, None) \
        == ofhip.OF_EINVAL
    assert ofhip.of_workspace_size([ofhip.OfImage(None, 64, 16384, 131079)], p1) > 0
    # tuning outside its ranges
    imgs = (ofhip.OfImage * 1)(img)
    offs = (ctypes.c_int64 * 1)(0)
    for kw in (dict(mark_words=5), dict(mark_rows=65), dict(det_w=300), dict(det_h=4),
               dict(det_w=129), dict(det_h=33)):
        t = ofhip.tuning(**kw)
        assert lib.of_detect_batch(imgs, 1, ctypes.byref(p), 0x1000, 1 << 30, 0x1000, offs, 100,
                                   0x1000, ctypes.byref(t), None) == ofhip.OF_EINVAL, kw
    assert lib.of_test_segment(None, 4, 7, 20, 0x1000, None) == ofhip.OF_EINVAL


def test_workspace_independent_of_tuning_and_monotone(lib):
    p = ofhip.params()
    a = ofhip.of_workspace_size([ofhip.OfImage(None, 1920, 1080, 1920)], p)
    b = ofhip.of_workspace_size([ofhip.OfImage(None, 1920, 1080, 1920)] * 2, p)
    assert b > a > 1920 * 1080


def test_default_tuning_valid_for_every_cell_size(lib):
    """The library's default launch shape fits its LDS limits for every accepted cell
    size: a call with a too-small workspace gets past tuning and stops at ENOSPACE."""
    img = ofhip.OfImage(0x1000, 1000, 800, 1024)
    imgs = (ofhip.OfImage * 1)(img)
    offs = (ctypes.c_int64 * 1)(0)
    for cell in [0] + list(range(8, 129)):
        p = ofhip.params(n_levels=3, cell=cell, n_features=500)
        st = lib.of_detect_batch(imgs, 1, ctypes.byref(p), 0x1000, 16, 0x1000, offs, 500, 0x1000,
                                 None, None)
        assert st == ofhip.OF_ENOSPACE, (cell, st)


def test_ablation_entry_points_validate_before_launch(lib):
    img = ofhip.OfImage(0x1000, 64, 48, 64)
    bad_img = ofhip.OfImage(0x1000, 64, 48, 32)
    one = (ctypes.c_void_p * 1)(0x1000)
    null = (ctypes.c_void_p * 1)(None)
    for lv, t, b, v in ((bad_img, 20, 15, 0), (img, 0, 15, 0), (img, 256, 15, 0),
                        (img, 20, 2, 0), (img, 20, 15, 5), (img, 20, 15, -1)):
        arr = (ofhip.OfImage * 1)(lv)
        assert lib.of_ablate_fast(arr, 1, t, b, v, one, None) == ofhip.OF_EINVAL, (t, b, v)
    arr = (ofhip.OfImage * 1)(img)
    assert lib.of_ablate_fast(None, 1, 20, 15, 0, one, None) == ofhip.OF_EINVAL
    assert lib.of_ablate_fast(arr, 0, 20, 15, 0, one, None) == ofhip.OF_EINVAL
    assert lib.of_ablate_fast(arr, 65, 20, 15, 0, one, None) == ofhip.OF_EINVAL
    assert lib.of_ablate_fast(arr, 1, 20, 15, 0, null, None) == ofhip.OF_EINVAL
    cnt = (ctypes.c_int32 * 1)(10)
    neg = (ctypes.c_int32 * 1)(-1)
    zero = (ctypes.c_int32 * 1)(0)
    assert lib.of_ablate_harris(arr, 1, one, cnt, 4, one, None) == ofhip.OF_EINVAL
    assert lib.of_ablate_harris(arr, 1, None, cnt, 0, one, None) == ofhip.OF_EINVAL
    assert lib.of_ablate_harris(arr, 1, null, cnt, 0, one, None) == ofhip.OF_EINVAL
    assert lib.of_ablate_harris(arr, 1, one, neg, 0, one, None) == ofhip.OF_EINVAL
    bad = (ofhip.OfImage * 1)(bad_img)
    assert lib.of_ablate_harris(bad, 1, None, None, 3, one, None) == ofhip.OF_EINVAL
    # nothing to score: returns before any launch
    assert lib.of_ablate_harris(arr, 1, null, zero, 0, one, None) == ofhip.OF_OK


def test_brief_tables_match_the_oracle(lib):
    """The library's steered tables (its own host code) equal the oracle's."""
    import oracle
    from synth import brief_pattern
    for seed in (4242, 7):
        pat = brief_pattern(seed)
        got = ofhip.of_brief_tables(pat)
        want = oracle.brief_tables(pat)
        np.testing.assert_array_equal(got[0], want[0])
        np.testing.assert_array_equal(got[1], want[1])


def test_describe_validates_before_launch(lib):
    p = ofhip.params(n_levels=2, cell=30, n_features=100)
    imgs = (ofhip.OfImage * 1)(ofhip.OfImage(0x1000, 200, 150, 200))
    offs = (ctypes.c_int64 * 1)(0)
    ok = [imgs, 1, ctypes.byref(p), None, 0x1000, 0x1000, offs, 0x1000, 0x1000, 0x1000, 0x1000,
          None]
    for k in (4, 5, 6, 7, 8, 9, 10):  # each device pointer / host array null in turn
        args = list(ok)
        args[k] = None
        assert lib.of_describe(*args) == ofhip.OF_EINVAL, k
    args = list(ok)
    args[1] = 0
    assert lib.of_describe(*args) == ofhip.OF_EINVAL
    bad = ofhip.tuning(mark_words=9)
    args = list(ok)
    args[3] = ctypes.byref(bad)
    assert lib.of_describe(*args) == ofhip.OF_EINVAL
    # a detection border below the descriptor's 15-pixel patch radius
    small_r = ofhip.params(n_levels=2, cell=30, n_features=100, patch_radius=14)
    args = list(ok)
    args[2] = ctypes.byref(small_r)
    assert lib.of_describe(*args) == ofhip.OF_EINVAL
    # stride below width; a frame spanning more than 2^31 - 1 bytes
    for im in (ofhip.OfImage(0x1000, 200, 150, 199), ofhip.OfImage(0x1000, 200, 150, 1 << 30)):
        args = list(ok)
        args[0] = (ofhip.OfImage * 1)(im)
        assert lib.of_describe(*args) == ofhip.OF_EINVAL


def test_library_geometry_matches_hand_derived_fixture(lib):
    """The library's level sizes and quotas (of_pyramid_desc_get) for the workloads of
    tests/golden/level_geometry.txt."""
    from test_oracle_pins import level_geometry_fixture
    for name, W, H, L, N, cell, widths, heights, quotas, _, _ in level_geometry_fixture():
        d = ofhip.of_pyramid_desc_get(W, H, ofhip.params(n_levels=L, n_features=N, cell=cell))
        assert list(d.width[:L]) == widths, name
        assert list(d.height[:L]) == heights, name
        assert list(d.quota[:L]) == quotas, name
