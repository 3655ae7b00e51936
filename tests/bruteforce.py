"""Pure-Python brute force of the detector for tiny images (pins the C oracle).

Written from different formulations than the oracle so that a slip in one does not
repeat in the other:

* pyramid      -- exact rational source positions with ``fractions.Fraction``; the
                  weight is Python's round() of 256 * fraction (round half to even);
* segment test -- circle pixels classified per Eq. (1), then a substring search for
                  nine '1' characters in the doubled classification string;
* Harris       -- the separable form of Eq. (4): G_x = [1 2 1]^T * ([-1 0 1] * I),
                  G_y = [-1 0 1]^T * ([1 2 1] * I), computed as whole-image passes;
* NMS/select   -- explicit neighbour comparisons and Python tuple sorting;
* orientation  -- direct double loops and math.atan2.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

CIRCLE = [(0, -3), (1, -3), (2, -2), (3, -1), (3, 0), (3, 1), (2, 2), (1, 3),
          (0, 3), (-1, 3), (-2, 2), (-3, 1), (-3, 0), (-3, -1), (-2, -2), (-1, -3)]


def level_sizes(W, H, L, num=6, den=5):
    out = []
    for l in range(L):
        s = Fraction(num, den) ** l
        # round half up of W / s
        out.append((int(math.floor(Fraction(W) / s + Fraction(1, 2))),
                    int(math.floor(Fraction(H) / s + Fraction(1, 2)))))
    return out


def resample(img, Wl, Hl):
    H, W = img.shape
    out = np.zeros((Hl, Wl), np.uint8)
    I = img.astype(np.int64)

    def tap(n_src, n_dst, i):
        pos = Fraction(2 * i + 1, 2) * Fraction(n_src, n_dst) - Fraction(1, 2)
        i0 = math.floor(pos)
        w = round(256 * (pos - i0))  # half to even
        return i0, min(i0 + 1, n_src - 1), w

    cols = [tap(W, Wl, x) for x in range(Wl)]
    rows = [tap(H, Hl, y) for y in range(Hl)]
    for y, (y0, y1, wy) in enumerate(rows):
        for x, (x0, x1, wx) in enumerate(cols):
            acc = ((256 - wy) * (256 - wx) * I[y0, x0] + (256 - wy) * wx * I[y0, x1]
                   + wy * (256 - wx) * I[y1, x0] + wy * wx * I[y1, x1])
            out[y, x] = (acc + 32768) >> 16
    return out


def is_corner(img, x, y, t):
    p = int(img[y, x])
    cls = ""
    for dx, dy in CIRCLE:
        v = int(img[y + dy, x + dx])
        cls += "b" if v >= p + t else ("d" if v <= p - t else "s")
    twice = cls + cls
    return "b" * 9 in twice or "d" * 9 in twice


def sobel_separable(img):
    I = img.astype(np.int64)
    H, W = I.shape
    hx = np.zeros_like(I)  # [-1 0 1] along x
    hs = np.zeros_like(I)  # [1 2 1] along x
    hx[:, 1:-1] = I[:, 2:] - I[:, :-2]
    hs[:, 1:-1] = I[:, :-2] + 2 * I[:, 1:-1] + I[:, 2:]
    gx = np.zeros_like(I)
    gy = np.zeros_like(I)
    gx[1:-1, :] = hx[:-2, :] + 2 * hx[1:-1, :] + hx[2:, :]  # [1 2 1] along y
    gy[1:-1, :] = hs[2:, :] - hs[:-2, :]                    # [-1 0 1] along y
    return gx, gy


def harris_map(img, r=3):
    gx, gy = sobel_separable(img)
    H, W = img.shape
    out = {}

    def R(x, y):
        if (x, y) not in out:
            sl = (slice(y - r, y + r + 1), slice(x - r, x + r + 1))
            a = int((gx[sl] * gx[sl]).sum())
            b = int((gy[sl] * gy[sl]).sum())
            c = int((gx[sl] * gy[sl]).sum())
            out[(x, y)] = 25 * (a * b - c * c) - (a + b) ** 2
        return out[(x, y)]
    return R


def harris_sliding(img, r=3):
    """R' map by sliding column sums: per column, running sums of the products over
    2r+1 rows, then running sums of those column sums over 2r+1 columns (the structure
    of Alg. 3, written from its description)."""
    gx, gy = sobel_separable(img)
    H, W = img.shape
    n = 2 * r + 1
    prods = [gx * gx, gy * gy, gx * gy]
    boxes = []
    for p in prods:
        col = np.zeros((H, W), np.int64)
        acc = np.zeros(W, np.int64)
        for y in range(H):
            acc += p[y]
            if y >= n:
                acc -= p[y - n]
            col[y] = acc            # rows y-n+1 .. y
        box = np.zeros((H, W), np.int64)
        for y in range(H):
            run = 0
            for x in range(W):
                run += int(col[y, x])
                if x >= n:
                    run -= int(col[y, x - n])
                box[y, x] = run     # columns x-n+1 .. x
        boxes.append(box)

    def R(x, y):
        a, b, c = (int(bx[y + r, x + r]) for bx in boxes)
        return 25 * (a * b - c * c) - (a + b) ** 2
    return R


def level_keypoints(lvl, t_hi, t_lo, cell, K, N, B=15):
    """Candidates, survivors and the kept keypoints [(R', y, x)] of one level."""
    Hl, Wl = lvl.shape
    cs = cell if cell > 0 else max(Wl, Hl)
    valid = [(x, y) for y in range(B, Hl - B) for x in range(B, Wl - B)]
    has_hi = set()
    for x, y in valid:
        if is_corner(lvl, x, y, t_hi):
            has_hi.add((x // cs, y // cs))
    cand = set()
    for x, y in valid:
        t = t_hi if (x // cs, y // cs) in has_hi else t_lo
        if is_corner(lvl, x, y, t):
            cand.add((x, y))
    R = harris_map(lvl)
    surv = []
    for (x, y) in cand:
        mine = (-R(x, y), y, x)
        ok = True
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                q = (x + dx, y + dy)
                if (dx or dy) and q in cand and (-R(*q), q[1], q[0]) < mine:
                    ok = False
        if ok:
            surv.append(mine)
    by_cell = {}
    for k in surv:
        by_cell.setdefault((k[2] // cs, k[1] // cs), []).append(k)
    kept = []
    for ks in by_cell.values():
        kept += sorted(ks)[:K]
    kept = sorted(kept)[:N]
    return cand, surv, [(-s, y, x) for s, y, x in kept]


def moments(lvl, x, y, r=15):
    m10 = m01 = 0
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            if dx * dx + dy * dy <= r * r:
                v = int(lvl[y + dy, x + dx])
                m10 += dx * v
                m01 += dy * v
    return m10, m01


def detect(img, L, t_hi, t_lo, cell, N, B=15, num=6, den=5):
    H, W = img.shape
    sizes = level_sizes(W, H, L, num, den)
    areas = [w * h for w, h in sizes]
    quota = [0] * L
    for l in range(1, L):
        quota[l] = (N * areas[l]) // sum(areas)
    quota[0] = N - sum(quota[1:])
    out = []
    for l, (w, h) in enumerate(sizes):
        lvl = img if l == 0 else resample(img, w, h)
        ncells = (-(-w // cell)) * (-(-h // cell)) if cell > 0 else 1
        K = max(1, -(-quota[l] // ncells))
        _, _, kept = level_keypoints(lvl, t_hi, t_lo, cell, K, quota[l], B)
        for R, y, x in kept:
            m10, m01 = moments(lvl, x, y, B)
            out.append((x, y, l, m10, m01, math.atan2(m01, m10), R))
    return out
