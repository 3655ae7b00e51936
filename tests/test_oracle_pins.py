"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Closed forms, hand-derived worked examples, invariants, the paper's Fig. 6 cases and a
pure-Python brute force written from different formulations (tests/bruteforce.py).
"""
import math
import os

import numpy as np
import pytest

import bruteforce as bf
import oracle
from synth import FrameSpec, make_frame, fig6_pattern_image

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng_img(H, W, seed, lo=0, hi=256):
    return np.random.Generator(np.random.PCG64(seed)).integers(lo, hi, (H, W)).astype(np.uint8)


# ------------------------------------------------------------- segment test --

def test_run9_closed_form_count():
    """Masks with a cyclic run of >= 9 ones among 16: 1 (all ones) + 16 (one zero)
    + sum_{L=9..14} 16 * 2^(14-L) (a maximal run of L ones bounded by two zeros,
    the other 14-L positions free) = 1 + 16 + 1008 = 1025."""
    expected = 1 + 16 + sum(16 * 2 ** (14 - L) for L in range(9, 15))
    assert expected == 1025
    got = sum(oracle.run9(m) for m in range(1 << 16))
    assert got == expected


def test_run9_matches_binary_encoding_formulation():
    """Sec. 5.1's binary encoding (Alg. 2): extend the 16 bits with their own low 8 bits
    to 24 bits, then test the low 9 bits against 0x1FF over 16 right shifts."""
    for m in range(1 << 16):
        ext = m | ((m & 0xFF) << 16)
        alg = any(((ext >> k) & 0x1FF) == 0x1FF for k in range(16))
        assert alg == oracle.run9(m), hex(m)


def test_compass_prefilter_is_necessary():
    """Any 9 contiguous positions hold two cyclically adjacent compass points
    (0,4), (4,8), (8,12) or (12,0): (b0|b8)&(b4|b12) never rejects a corner mask."""
    for m in range(1 << 16):
        if oracle.run9(m):
            b = [(m >> i) & 1 for i in (0, 4, 8, 12)]
            assert (b[0] | b[2]) & (b[1] | b[3])


def test_diagonal_prefilter_is_necessary():
    """Likewise for the diagonal points (2,6), (6,10), (10,14), (14,2): the segment test's
    second pre-test stage, (b2|b10)&(b6|b14), never rejects a corner mask either."""
    for m in range(1 << 16):
        if oracle.run9(m):
            b = [(m >> i) & 1 for i in (2, 6, 10, 14)]
            assert (b[0] | b[2]) & (b[1] | b[3])


def test_odd_position_prefilters_are_necessary():
    """Likewise for the two sets of odd positions, (1,5,9,13) and (3,7,11,15) (0-based
    from the top, clockwise): nine consecutive positions hold two points of every residue
    class mod 4 that are adjacent in the class, so (b1|b9)&(b5|b13) and (b3|b11)&(b7|b15)
    never reject a corner mask (the segment test's third pre-test stage)."""
    for m in range(1 << 16):
        if oracle.run9(m):
            b = [(m >> i) & 1 for i in range(16)]
            assert (b[1] | b[9]) & (b[5] | b[13])
            assert (b[3] | b[11]) & (b[7] | b[15])


def test_pretests_hold_per_polarity():
    """The pre-tests in the min/max form the segment-test tiles evaluate (the compass
    pairs and the diagonal pairs, each as min(max(a, a'), max(b, b')) >= p + t for bright
    and max(min(..), min(..)) <= p - t for dark) are necessary per polarity: a corner of
    either polarity passes both pre-tests of that polarity.  Random circles, centres and
    thresholds."""
    rng = np.random.Generator(np.random.PCG64(17))
    n = 40000
    p = rng.integers(0, 256, n)
    c = np.clip(p[:, None] + rng.integers(-60, 61, (n, 16)), 0, 255)
    t = rng.integers(1, 40, n)
    comp, diag = (0, 4, 8, 12), (2, 6, 10, 14)  # positions 1/5/9/13 and 3/7/11/15
    odd_a, odd_b = (1, 5, 9, 13), (3, 7, 11, 15)  # the third stage's two sets
    for i in range(n):
        ci, pi, ti = c[i], int(p[i]), int(t[i])
        for sign in (+1, -1):
            mask = sum(1 << k for k in range(16) if sign * (int(ci[k]) - pi) >= ti)
            if not oracle.run9(mask):
                continue
            for a, b, a2, b2 in (comp, diag, odd_a, odd_b):
                if sign > 0:
                    assert min(max(ci[a], ci[a2]), max(ci[b], ci[b2])) >= pi + ti
                else:
                    assert max(min(ci[a], ci[a2]), min(ci[b], ci[b2])) <= pi - ti


def _fig6_cases():
    cases = []
    with open(os.path.join(GOLDEN, "fig6_patterns.txt")) as f:
        for line in f:
            line = line.split("#")[0].split()
            if line:
                cases.append((line[0], [int(v) for v in line[1].split(",")], line[2] == "1"))
    return cases


def test_fig6_cases_of_the_generator_match_the_fixture():
    """The benchmark's input list (synth) holds the same patterns as the cited fixture."""
    from synth import FIG6_CASES
    assert [(c, tuple(p), bool(k)) for c, p, k in _fig6_cases()] == list(FIG6_CASES)


@pytest.mark.parametrize("case,pos,corner", _fig6_cases())
def test_fig6_patterns(case, pos, corner):
    img = np.full((9, 9), 100, np.uint8)
    for p in pos:
        dx, dy = bf.CIRCLE[p - 1]
        img[4 + dy, 4 + dx] = 200
    assert oracle.segment_test(img, 4, 4, 20) == corner
    assert bf.is_corner(img, 4, 4, 20) == corner


def test_segment_test_thresholds_inclusive():
    """Eq. (1) classifies with <= and >=: a difference of exactly t counts."""
    img = np.full((9, 9), 100, np.uint8)
    for p in range(1, 10):
        dx, dy = bf.CIRCLE[p - 1]
        img[4 + dy, 4 + dx] = 120
    assert oracle.segment_test(img, 4, 4, 20)
    assert not oracle.segment_test(img, 4, 4, 21)
    img2 = 255 - img
    assert oracle.segment_test(img2, 4, 4, 20)  # dark run, difference exactly 20


def test_fig6_tiled_image_counts():
    """1024x1024 frame with 625 copies of each Fig. 6 pattern: the copies are identical
    and isolated, so the corner count is 625 times the count of one copy."""
    p = oracle.params(n_levels=1, fast_t=20, fast_t_min=20, cell=0, n_features=65536)
    for case, pos, corner in _fig6_cases():
        img = fig6_pattern_image(pos)
        r = oracle.level_detect(img, p, 0, 65536, 65536)
        one = fig6_pattern_image(pos, size=41, copies=1)
        r1 = oracle.level_detect(one, p, 0, 65536, 65536)
        assert r["cand"].sum() == 625 * r1["cand"].sum()
        assert bool(r1["cand"][20, 20]) == corner


# ------------------------------------------------------- worked example: square --

def _square():
    img = np.full((64, 64), 60, np.uint8)
    img[20:44, 20:44] = 160
    return img


def test_square_fast_corners():
    """Hand count: an inside pixel at offset (a, b) from a square corner sees
    16 - #{circle points with dx >= -a, dy >= -b} dark circle pixels; that is >= 9
    exactly for the offsets (0,0),(1,0),(2,0),(0,1),(1,1),(0,2).  Straight edges
    give 7 contiguous pixels and no outside pixel sees 9 bright ones: 24 corners."""
    img = _square()
    p = oracle.params(n_levels=1, fast_t=20, fast_t_min=20, cell=0, n_features=500)
    r = oracle.level_detect(img, p, 0, 500, 500)
    offs = [(0, 0), (1, 0), (2, 0), (0, 1), (1, 1), (0, 2)]
    expected = set()
    for a, b in offs:
        expected |= {(20 + a, 20 + b), (43 - a, 20 + b), (20 + a, 43 - b), (43 - a, 43 - b)}
    got = {(int(x), int(y)) for y, x in zip(*np.nonzero(r["cand"]))}
    assert got == expected and len(got) == 24


def test_square_harris_and_nms():
    """Hand derivation at (21,21): G_x = 100 * c(y) on columns 19 and 20 with
    c = 0,1,3,4,4,... for y = 18,19,20,21,... (and symmetrically for G_y), so over the
    7x7 window Sxx = Syy = 2 * (1 + 9 + 4*16) * 10^4 = 1,480,000 and
    Sxy = (1 + 3 + 3 + 9) * 10^4 = 160,000.  R' = 25 (Sxx Syy - Sxy^2) - (Sxx+Syy)^2
    = 45,358,400,000,000.  Likewise (20,20): Sxx = Syy = 1,160,000 -> 27,617,600,000,000;
    (22,20): Sxx = 1,160,000, Syy = 1,800,000 -> 42,798,400,000,000;
    (21,20): Sxx = 1,160,000, Syy = 1,480,000 -> 35,310,400,000,000.
    (21,21) is a neighbour of all five others, so NMS keeps one pixel per corner."""
    img = _square()
    R = lambda sxx, syy, sxy: 25 * (sxx * syy - sxy * sxy) - (sxx + syy) ** 2
    assert R(1_480_000, 1_480_000, 160_000) == 45_358_400_000_000
    assert oracle.harris(img, 21, 21) == 45_358_400_000_000
    assert oracle.harris(img, 20, 20) == R(1_160_000, 1_160_000, 160_000) == 27_617_600_000_000
    assert oracle.harris(img, 22, 20) == R(1_160_000, 1_800_000, 160_000) == 42_798_400_000_000
    assert oracle.harris(img, 21, 20) == R(1_160_000, 1_480_000, 160_000) == 35_310_400_000_000
    p = oracle.params(n_levels=1, fast_t=20, fast_t_min=20, cell=0, n_features=500)
    r = oracle.level_detect(img, p, 0, 500, 500)
    surv = {(int(x), int(y)) for y, x in zip(*np.nonzero(r["surv"]))}
    assert surv == {(21, 21), (42, 21), (21, 42), (42, 42)}
    kp = oracle.detect(img, p)
    assert len(kp) == 4
    assert set(kp["score"].tolist()) == {45_358_400_000_000}
    # equal scores: ties go to smaller y, then smaller x
    assert [(int(k["x"]), int(k["y"])) for k in kp] == [(21, 21), (42, 21), (21, 42), (42, 42)]


# --------------------------------------------------------------- Harris -------

def test_harris_constant_and_edge():
    """A constant window gives 0.  A vertical step of height h gives G_y = 0 and
    G_x = 4h on the two columns beside the step, so Sxx = 2 * 7 * (4h)^2,
    Syy = Sxy = 0 and R' = -Sxx^2."""
    img = np.full((20, 20), 77, np.uint8)
    assert oracle.harris(img, 10, 10) == 0
    h = 50
    img[:, 10:] = 77 + h
    sxx = 2 * 7 * (4 * h) ** 2
    assert oracle.harris(img, 10, 10) == -sxx * sxx
    assert oracle.harris(img, 9, 10) == -sxx * sxx


@pytest.mark.parametrize("seed", range(4))
def test_harris_separable_and_mirror(seed):
    """2D kernels (oracle) equal the separable form of Eq. (4) and the sliding
    column-sum form of Alg. 3 (brute force), and R' is unchanged by mirroring the image
    (a sign flip of G_x)."""
    img = _rng_img(24, 24, seed)
    R = bf.harris_map(img)
    S = bf.harris_sliding(img)
    mir = np.ascontiguousarray(img[:, ::-1])
    for y in range(4, 20):
        for x in range(4, 20):
            v = oracle.harris(img, x, y)
            assert v == R(x, y)
            assert v == S(x, y)
            assert v == oracle.harris(mir, 23 - x, y)


# --------------------------------------------------------------- pyramid ------

def test_level_sizes_closed_form():
    g = oracle.geometry(1920, 1080, oracle.params())
    want = [(int(math.floor(1920 / 1.2 ** l + 0.5)), int(math.floor(1080 / 1.2 ** l + 0.5)))
            for l in range(8)]
    assert list(zip(g["width"].tolist(), g["height"].tolist())) == want
    assert bf.level_sizes(1920, 1080, 8) == want
    assert g["quota"].sum() == 2000
    A = g["width"].astype(np.int64) * g["height"]
    for l in range(1, 8):  # floor of the proportional share
        assert g["quota"][l] <= 2000 * A[l] / A.sum() < g["quota"][l] + 1


def level_geometry_fixture():
    """Rows of tests/golden/level_geometry.txt: (name, W, H, levels, N, cell, widths,
    heights, quotas, cells, K)."""
    rows = []
    with open(os.path.join(GOLDEN, "level_geometry.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            head, *cols = [c.strip() for c in line.split("|")]
            name, W, H, L, N, cell = head.split()
            rows.append((name, int(W), int(H), int(L), int(N), int(cell),
                         *[[int(v) for v in c.split(",")] for c in cols]))
    return rows


@pytest.mark.parametrize("row", level_geometry_fixture(), ids=lambda r: r[0])
def test_level_quotas_cells_and_keep_counts(row):
    """Level sizes, area quotas N_l, cell counts and per-cell keep counts K_l of the
    workloads against the hand-derived fixture."""
    name, W, H, L, N, cell, widths, heights, quotas, cells, K = row
    g = oracle.geometry(W, H, oracle.params(n_levels=L, n_features=N, cell=cell))
    assert g["width"].tolist() == widths
    assert g["height"].tolist() == heights
    assert g["quota"].tolist() == quotas
    assert g["n_cells"].tolist() == cells
    assert g["k_cell"].tolist() == K


def test_resample_identity_and_constant():
    img = _rng_img(31, 37, 7)
    assert np.array_equal(oracle.resample(img, 37, 31), img)
    c = np.full((50, 60), 123, np.uint8)
    assert np.all(oracle.resample(c, 41, 37) == 123)


def test_resample_ramp_and_float_bilinear():
    """A horizontal ramp I = 2x + 10 resampled must equal round(2 sx + 10) up to the
    1/256 weight quantisation (|err| <= 2/512 + 1/2 -> within 1 of the exact value);
    random images stay within 1.5 of float64 bilinear (weights off by <= 1/512)."""
    W, H = 100, 20
    ramp = np.tile((2 * np.arange(W) + 10).astype(np.uint8), (H, 1))
    Wl, Hl = 83, 17
    out = oracle.resample(ramp, Wl, Hl)
    sx = ((2 * np.arange(Wl) + 1) * W - Wl) / (2 * Wl)
    exact = 2 * sx + 10
    assert np.all(np.abs(out[0].astype(float) - exact) <= 1.0)
    img = _rng_img(60, 70, 3)
    Wl, Hl = 58, 50
    out = oracle.resample(img, Wl, Hl).astype(float)
    sx = ((2 * np.arange(Wl) + 1) * 70 - Wl) / (2 * Wl)
    sy = ((2 * np.arange(Hl) + 1) * 60 - Hl) / (2 * Hl)
    x0 = np.floor(sx).astype(int); fx = sx - x0; x1 = np.minimum(x0 + 1, 69)
    y0 = np.floor(sy).astype(int); fy = sy - y0; y1 = np.minimum(y0 + 1, 59)
    I = img.astype(float)
    ref = ((1 - fy)[:, None] * ((1 - fx) * I[y0][:, x0] + fx * I[y0][:, x1])
           + fy[:, None] * ((1 - fx) * I[y1][:, x0] + fx * I[y1][:, x1]))
    assert np.max(np.abs(out - ref)) <= 1.5


@pytest.mark.parametrize("seed", range(3))
def test_resample_matches_exact_rational_bruteforce(seed):
    img = _rng_img(40, 52, 10 + seed)
    for Wl, Hl in [(43, 33), (36, 28), (25, 19)]:
        assert np.array_equal(oracle.resample(img, Wl, Hl), bf.resample(img, Wl, Hl))


def test_resample_commutes_with_flip_and_transpose():
    img = _rng_img(53, 71, 11)
    for Wl, Hl in [(59, 44), (49, 37), (41, 31)]:
        a = oracle.resample(img, Wl, Hl)
        assert np.array_equal(oracle.resample(np.ascontiguousarray(img[:, ::-1]), Wl, Hl), a[:, ::-1])
        assert np.array_equal(oracle.resample(np.ascontiguousarray(img[::-1]), Wl, Hl), a[::-1])
        assert np.array_equal(oracle.resample(np.ascontiguousarray(img.T), Hl, Wl), a.T)


# ----------------------------------------------------------- orientation -------

def test_disk_and_ramp_moments():
    """The r = 15 disk has 709 pixels (row half-widths floor(sqrt(225 - dy^2))).  For a
    horizontal ramp I = a + b x the moments are m10 = b * sum dx^2 = b * sum_dy
    h(h+1)(2h+1)/3 and m01 = 0, so the angle is 0 (b > 0) or pi (b < 0)."""
    hw = [math.isqrt(225 - dy * dy) for dy in range(-15, 16)]
    assert sum(2 * h + 1 for h in hw) == 709
    sdx2 = sum(h * (h + 1) * (2 * h + 1) // 3 for h in hw)
    W = 40
    for b in (1, 2, -1):
        row = (100 + b * (np.arange(W) - 20)).astype(np.uint8)
        img = np.tile(row, (W, 1))
        m10, m01 = oracle.moments(img, 20, 20, 15)
        assert (m10, m01) == (b * sdx2, 0)
        assert (m10, m01) == bf.moments(img, 20, 20, 15)
        vert = np.ascontiguousarray(img.T)
        assert oracle.moments(vert, 20, 20, 15) == (0, b * sdx2)


# ------------------------------------------------------------- invariants ------

def test_constant_image_has_no_keypoints():
    img = np.full((200, 240), 93, np.uint8)
    p = oracle.params(n_levels=4, n_features=500)
    assert len(oracle.detect(img, p)) == 0
    for lvl in oracle.pyramid(img, p):
        assert np.all(lvl == 93)


def _no_tied_neighbours(r):
    s, c = r["score"], r["cand"].astype(bool)
    H, W = c.shape
    for dy, dx in [(0, 1), (1, -1), (1, 0), (1, 1)]:
        a = c[max(0, -dy):H - max(0, dy), max(0, -dx):W - max(0, dx)]
        b = c[max(0, dy):, max(0, dx):][:a.shape[0], :a.shape[1]]
        sa = s[max(0, -dy):H - max(0, dy), max(0, -dx):W - max(0, dx)]
        sb = s[max(0, dy):, max(0, dx):][:a.shape[0], :a.shape[1]]
        if np.any(a & b & (sa == sb)):
            return False
    return True


def test_rotation_invariance():
    """A 90-degree clockwise turn (x, y) -> (H-1-y, x) maps candidates, scores and
    survivors onto each other exactly, at every pyramid level (the resample commutes
    with flips and transposition); moments map as (m10, m01) -> (-m01, m10)."""
    img = make_frame(FrameSpec(150, 126, 5, 12, 4.0))
    rot = np.ascontiguousarray(np.rot90(img, k=-1))  # clockwise
    H = img.shape[0]
    p = oracle.params(n_levels=3, cell=0, fast_t=20, fast_t_min=20, n_features=65536)
    L0, L1 = oracle.pyramid(img, p), oracle.pyramid(rot, p)
    total = 0
    for l in range(3):
        assert np.array_equal(np.rot90(L0[l], k=-1), L1[l])
        a = oracle.level_detect(L0[l], p, l, 65536, 65536)
        b = oracle.level_detect(L1[l], p, l, 65536, 65536)
        assert _no_tied_neighbours(a)
        for key in ("cand", "surv", "score"):
            assert np.array_equal(np.rot90(a[key], k=-1), b[key]), key
        total += a["surv"].sum()
    assert total > 20
    ka, kb = oracle.detect(img, p), oracle.detect(rot, p)
    assert len(ka) == len(kb) == total
    ma = {(int(k["level"]), L0[k["level"]].shape[0] - 1 - int(k["y"]), int(k["x"])): (int(k["m10"]), int(k["m01"]), float(k["angle"])) for k in ka}
    for k in kb:
        m10, m01, ang = ma[(int(k["level"]), int(k["x"]), int(k["y"]))]
        assert (int(k["m10"]), int(k["m01"])) == (-m01, m10)
        d = (float(k["angle"]) - ang - math.pi / 2) % (2 * math.pi)
        assert min(d, 2 * math.pi - d) < 1e-12


# ------------------------------------------------------------ brute force ------

@pytest.mark.parametrize("W,H,seed,L,cell,N", [
    (64, 56, 1, 1, 0, 40), (72, 64, 2, 2, 30, 60), (90, 76, 3, 2, 30, 30),
    (80, 80, 4, 3, 16, 100)])
def test_pipeline_matches_bruteforce(W, H, seed, L, cell, N):
    img = make_frame(FrameSpec(W, H, seed, 10, 3.0))
    p = oracle.params(n_levels=L, cell=cell, n_features=N, fast_t=20, fast_t_min=7)
    got = oracle.detect(img, p)
    want = bf.detect(img, L, 20, 7, cell, N)
    assert len(got) == len(want) > 0
    for g, w in zip(got, want):
        assert (int(g["x"]), int(g["y"]), int(g["level"]), int(g["m10"]), int(g["m01"])) == w[:5]
        assert int(g["score"]) == w[6]
        assert abs(float(g["angle"]) - w[5]) < 1e-12


@pytest.mark.parametrize("cell", [30, 0])
def test_smallest_frame_one_valid_pixel(cell):
    """A 31x31 frame, the smallest the calls accept, has one pixel outside the 15-pixel
    border: (15, 15).  A bright square with its corner there gives exactly one keypoint;
    the frame is symmetric under transposition, so m10 = m01 and the angle is pi/4."""
    img = np.full((31, 31), 60, np.uint8)
    img[14:26, 14:26] = 170
    p = oracle.params(n_levels=1, cell=cell, n_features=4, fast_t=20, fast_t_min=7)
    got = oracle.detect(img, p)
    want = bf.detect(img, 1, 20, 7, cell, 4)
    assert len(got) == len(want) == 1
    g = got[0]
    assert (int(g["x"]), int(g["y"]), int(g["m10"]), int(g["m01"])) == want[0][:2] + want[0][3:5]
    assert (int(g["x"]), int(g["y"])) == (15, 15) and int(g["m10"]) == int(g["m01"]) > 0
    assert int(g["score"]) == want[0][6] > 0
    assert abs(float(g["angle"]) - math.pi / 4) < 1e-6
    assert len(oracle.detect(np.full((31, 31), 60, np.uint8), p)) == 0


@pytest.mark.parametrize("W,H,seed,L,cell,N,num,den,B", [
    (72, 64, 5, 2, 30, 40, 2, 1, 8), (90, 80, 6, 3, 16, 60, 8, 7, 20),
    (60, 52, 7, 2, 30, 30, 3, 2, 4)])
def test_pipeline_other_scales_and_radii(W, H, seed, L, cell, N, num, den, B):
    """Scales 2, 8/7 and 3/2 with patch radii (and detection borders) 8, 20 and 4 against
    the brute-force pipeline: level sizes, border, disk and moments all follow them."""
    img = make_frame(FrameSpec(W, H, seed, 10, 3.0))
    p = oracle.params(n_levels=L, scale_num=num, scale_den=den, cell=cell, n_features=N,
                      fast_t=20, fast_t_min=7, patch_radius=B)
    got = oracle.detect(img, p)
    want = bf.detect(img, L, 20, 7, cell, N, B, num, den)
    assert len(got) == len(want) > 0
    assert {int(g["level"]) for g in got} == set(range(L))
    for g, w in zip(got, want):
        assert (int(g["x"]), int(g["y"]), int(g["level"]), int(g["m10"]), int(g["m01"])) == w[:5]
        assert int(g["score"]) == w[6]
        assert abs(float(g["angle"]) - w[5]) < 1e-12


def test_level_stage_maps_match_bruteforce():
    img = make_frame(FrameSpec(96, 80, 9, 14, 3.0))
    p = oracle.params(n_levels=1, cell=30, n_features=1000, fast_t=20, fast_t_min=7)
    r = oracle.level_detect(img, p, 0, 2, 1000)
    cand, surv, kept = bf.level_keypoints(img, 20, 7, 30, 2, 1000)
    assert {(int(x), int(y)) for y, x in zip(*np.nonzero(r["cand"]))} == cand
    assert {(int(x), int(y)) for y, x in zip(*np.nonzero(r["surv"]))} == {(x, y) for _, y, x in surv}
    assert [(int(k["score"]), int(k["y"]), int(k["x"])) for k in r["keypoints"]] == kept


def test_cell_fallback_only_adds_points():
    """Segment-test corner sets shrink as t grows, so the fallback threshold only adds
    candidates: every t=20 corner is a t=7 corner."""
    img = make_frame(FrameSpec(120, 100, 21, 20, 3.0))
    for y in range(3, 97):
        for x in range(3, 117):
            if oracle.segment_test(img, x, y, 20):
                assert oracle.segment_test(img, x, y, 7)


def test_param_validation():
    assert oracle.check(640, 480, oracle.params(n_levels=1))
    assert not oracle.check(640, 480, oracle.params(n_levels=0))
    assert not oracle.check(640, 480, oracle.params(fast_t_min=21))
    assert not oracle.check(640, 480, oracle.params(harris_block=5))
    assert oracle.check(31, 31, oracle.params(n_levels=1))
    assert not oracle.check(30, 31, oracle.params(n_levels=1))  # narrower than 2*15+1
    assert oracle.check(640, 480, oracle.params(n_levels=16))  # level 15 is 42x31
    assert not oracle.check(600, 460, oracle.params(n_levels=16))  # level 15 is 39x30
    assert not oracle.check(640, 480, oracle.params(n_levels=17))


# ------------------------------------------------------------------ rBRIEF ------

def test_brief_tables_closed_forms():
    """Bin 0 is the pattern itself, bin 15 its exact negation (180 degrees); bin 5 (60
    degrees, cos = 1/2) rounds the half-way values to even, written out by hand."""
    from synth import brief_pattern
    pat = np.array([[1, 0, 2, 0], [0, 1, -3, 2]] + [[0, 0, 0, 0]] * 254, np.int8)
    rot, cen = oracle.brief_tables(pat)
    assert (rot[0] == pat).all() and (rot[15] == -pat).all()
    assert tuple(cen[0]) == (16384, 0) and tuple(cen[15]) == (-16384, 0)
    assert tuple(cen[5]) == (8192, 14189)                       # round(2^14 (1/2, sqrt(3)/2))
    # (1,0) -> (0.5, 0.866) -> (0, 1); (2,0) -> (1, 1.732) -> (1, 2)
    assert rot[5, 0].tolist() == [0, 1, 1, 2]
    # 240 degrees: (1,0) -> (-0.5, -0.866) -> (0, -1) (ties to even in both directions)
    assert rot[20, 0].tolist() == [0, -1, -1, -2]
    assert (rot[15:] == -rot[:15]).all() and (cen[15:] == -cen[:15]).all()
    # (0,1) -> (-0.866, 0.5) -> (-1, 0); (-3,2) -> (-1.5-1.732, -2.598+1) -> (-3, -2)
    assert rot[5, 1].tolist() == [-1, 0, -3, -2]
    real = brief_pattern()
    assert (np.abs(real.astype(int)) <= 13).all()
    assert ((real[:, 0::2].astype(int) ** 2 + real[:, 1::2].astype(int) ** 2) <= 169).all()
    rr, _ = oracle.brief_tables(real)
    assert (np.abs(rr.astype(int)) <= 13).all()


def _kp(x, y, m10, m01):
    a = np.zeros(1, oracle.KEYPOINT_DTYPE)
    a["x"], a["y"], a["m10"], a["m01"] = x, y, m10, m01
    return a


def test_brief_descriptor_closed_forms():
    """A constant patch sets no bit; on a horizontal ramp (smoothing keeps it a ramp)
    the bits of bin 0 are x1 < x2, on a vertical ramp y1 < y2."""
    from synth import brief_pattern
    pat = brief_pattern()
    rot, cen = oracle.brief_tables(pat)
    bits = lambda d: np.unpackbits(d[0], bitorder="little")
    flat = np.full((40, 40), 90, np.uint8)
    assert not oracle.describe(flat, _kp(20, 20, 5, 0), rot, cen).any()
    ramp_x = np.tile(np.arange(40, dtype=np.uint8) + 10, (40, 1))
    ramp_y = np.ascontiguousarray(ramp_x.T)
    np.testing.assert_array_equal(bits(oracle.describe(ramp_x, _kp(20, 20, 7, 0), rot, cen)),
                                  (pat[:, 0] < pat[:, 2]).astype(np.uint8))
    np.testing.assert_array_equal(bits(oracle.describe(ramp_y, _kp(20, 20, 7, 0), rot, cen)),
                                  (pat[:, 1] < pat[:, 3]).astype(np.uint8))


def test_brief_bins_and_180_degree_rotation():
    """The bin follows the angle of (m10, m01) in 12 degree steps; rotating the image by
    180 degrees (and negating the moments) leaves the descriptor unchanged."""
    from synth import brief_pattern
    rot, cen = oracle.brief_tables(brief_pattern())
    rng = np.random.default_rng(3)
    img = rng.integers(0, 256, (48, 52), dtype=np.uint8)
    img180 = np.ascontiguousarray(img[::-1, ::-1])
    for k in range(30):
        a = 2 * np.pi * k / 30 + 0.05
        m10, m01 = int(round(1e5 * np.cos(a))), int(round(1e5 * np.sin(a)))
        d = oracle.describe(img, _kp(25, 22, m10, m01), rot, cen)
        # the same descriptor as from the table of bin k directly
        t = rot[k].astype(int)
        assert d[0].tolist() == oracle.describe(img, _kp(25, 22, int(cen[k][0]),
                                                         int(cen[k][1])), rot, cen)[0].tolist()
        d180 = oracle.describe(img180, _kp(52 - 1 - 25, 48 - 1 - 22, -m10, -m01), rot, cen)
        np.testing.assert_array_equal(d, d180)


def test_brief_smoothing_matches_library_convolution():
    """The tests compare 5x5 binomial sums; scipy's correlate gives the same comparisons."""
    from scipy.ndimage import correlate
    from synth import brief_pattern
    pat = brief_pattern()
    rot, cen = oracle.brief_tables(pat)
    rng = np.random.default_rng(9)
    img = rng.integers(0, 256, (60, 64), dtype=np.uint8)
    w = np.array([1, 4, 6, 4, 1])
    S = correlate(img.astype(np.int64), np.outer(w, w), mode="constant")
    for (x, y, m10, m01) in [(30, 30, 100, 3), (20, 40, -50, 80), (44, 17, 0, -9)]:
        d = oracle.describe(img, _kp(x, y, m10, m01), rot, cen)
        k = int(np.argmax(m10 * cen[:, 0].astype(np.int64) + m01 * cen[:, 1].astype(np.int64)))
        t = rot[k].astype(int)
        want = (S[y + t[:, 1], x + t[:, 0]] < S[y + t[:, 3], x + t[:, 2]]).astype(np.uint8)
        np.testing.assert_array_equal(np.unpackbits(d[0], bitorder="little"), want)
