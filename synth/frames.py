"""Seeded synthetic grey frames shared by the CPU oracle, the GPU path and the bench.

This module only draws pixels. It holds none of the detector's arithmetic, so the
oracle and the HIP path can both take their inputs from it without sharing code.

The paper measures on eight natural photographs (720x540 up to 1920x1080) that are
not available; these frames stand in for them with the same resolutions and a
controllable feature density.  Recipe (one frame):

1. background: a linear ramp between two intensities drawn from U{30..225}, along a
   random direction, spanning the whole frame;
2. ``n_shapes`` filled shapes painted in order, each a rectangle or a triangle with
   probability 1/2: box sides U{8..min(W,H)//6}, box origin uniform inside the
   frame, fill U{0..255}; a triangle has three vertices uniform in its box and
   covers a pixel when the pixel centre is inside (or on an edge);
3. optionally a low-contrast sinusoidal texture ``amp * sin(2 pi (fx x + fy y) + phi)``
   with period U[6, 40] px along a random direction;
4. additive Gaussian noise N(0, sigma^2).

All of it is summed in float64 and rounded once (half to even) and clipped to
[0, 255].  Random numbers come from numpy's PCG64 seeded with ``seed``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = ["FrameSpec", "make_frame", "make_frames", "fig6_pattern_image",
           "stream_schedule", "CONFIGS"]


@dataclass(frozen=True)
class FrameSpec:
    width: int
    height: int
    seed: int
    n_shapes: int = 150
    sigma: float = 3.0
    texture_amp: float = 0.0


def _ramp(rng: np.random.Generator, W: int, H: int) -> np.ndarray:
    a = float(rng.integers(30, 226))
    b = float(rng.integers(30, 226))
    theta = rng.uniform(0.0, 2.0 * math.pi)
    ux, uy = math.cos(theta), math.sin(theta)
    xs = np.arange(W, dtype=np.float64) + 0.5
    ys = np.arange(H, dtype=np.float64) + 0.5
    proj = ux * xs[None, :] + uy * ys[:, None]
    lo, hi = proj.min(), proj.max()
    t = (proj - lo) / max(hi - lo, 1e-12)
    return a + (b - a) * t


def _paint_shapes(rng: np.random.Generator, img: np.ndarray, n_shapes: int) -> None:
    H, W = img.shape
    smax = max(8, min(W, H) // 6)
    for _ in range(n_shapes):
        is_tri = rng.random() < 0.5
        bw = int(rng.integers(8, smax + 1))
        bh = int(rng.integers(8, smax + 1))
        x0 = int(rng.integers(0, max(1, W - bw + 1)))
        y0 = int(rng.integers(0, max(1, H - bh + 1)))
        fill = float(rng.integers(0, 256))
        if not is_tri:
            img[y0:y0 + bh, x0:x0 + bw] = fill
            continue
        vx = rng.uniform(x0, x0 + bw, size=3)
        vy = rng.uniform(y0, y0 + bh, size=3)
        xs = np.arange(x0, x0 + bw, dtype=np.float64) + 0.5
        ys = np.arange(y0, y0 + bh, dtype=np.float64) + 0.5
        px = xs[None, :]
        py = ys[:, None]

        def edge(ax, ay, bx, by):
            return (bx - ax) * (py - ay) - (by - ay) * (px - ax)

        e0 = edge(vx[0], vy[0], vx[1], vy[1])
        e1 = edge(vx[1], vy[1], vx[2], vy[2])
        e2 = edge(vx[2], vy[2], vx[0], vy[0])
        inside = ((e0 >= 0) & (e1 >= 0) & (e2 >= 0)) | ((e0 <= 0) & (e1 <= 0) & (e2 <= 0))
        sub = img[y0:y0 + bh, x0:x0 + bw]
        sub[inside] = fill


def make_frame(spec: FrameSpec) -> np.ndarray:
    """Return an (H, W) uint8 C-contiguous frame for ``spec``."""
    W, H = spec.width, spec.height
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    img = _ramp(rng, W, H)
    _paint_shapes(rng, img, spec.n_shapes)
    if spec.texture_amp > 0.0:
        period = rng.uniform(6.0, 40.0)
        theta = rng.uniform(0.0, 2.0 * math.pi)
        phi = rng.uniform(0.0, 2.0 * math.pi)
        fx, fy = math.cos(theta) / period, math.sin(theta) / period
        xs = np.arange(W, dtype=np.float64)
        ys = np.arange(H, dtype=np.float64)
        img += spec.texture_amp * np.sin(2.0 * math.pi * (fx * xs[None, :] + fy * ys[:, None]) + phi)
    if spec.sigma > 0.0:
        img += rng.normal(0.0, spec.sigma, size=(H, W))
    out = np.clip(np.rint(img), 0, 255).astype(np.uint8)
    return np.ascontiguousarray(out)


def make_frames(specs) -> list[np.ndarray]:
    return [make_frame(s) for s in specs]


# Circle positions 1..16 of the segment test, clockwise from the top, y down.
_CIRCLE = [(0, -3), (1, -3), (2, -2), (3, -1), (3, 0), (3, 1), (2, 2), (1, 3),
           (0, 3), (-1, 3), (-2, 2), (-3, 1), (-3, 0), (-3, -1), (-2, -2), (-1, -3)]


# The five segment-test patterns of Fig. 6 as read from its caption: case, bright circle
# positions (1..16 clockwise from the top), and whether the centre is a FAST-9 corner.
FIG6_CASES = (
    ("a", (1, 2, 3, 4, 5, 6, 7, 8, 9), True),
    ("b", (6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 1), True),
    ("c", (12, 13, 14, 15, 16, 1, 2, 3, 4), True),
    ("d", (1, 2, 3, 4, 5, 6, 7, 8), False),
    ("e", (1, 3, 5, 7, 9, 11, 13, 15), False),
)


def fig6_pattern_image(bright_positions, size: int = 1024, copies: int = 25,
                       base: int = 100, bright: int = 200) -> np.ndarray:
    """Tile ``copies x copies`` copies of one segment-test pattern over a flat frame.

    ``bright_positions`` are circle positions numbered 1..16 clockwise from the top;
    each copy sets those circle pixels around its centre to ``bright`` on a flat
    ``base`` background (the centre keeps ``base``).  Copies sit on a regular grid of
    pitch ``size // copies`` so neighbouring copies never overlap.
    """
    img = np.full((size, size), base, dtype=np.uint8)
    pitch = size // copies
    off = pitch // 2
    for cy in range(copies):
        for cx in range(copies):
            x, y = cx * pitch + off, cy * pitch + off
            for p in bright_positions:
                dx, dy = _CIRCLE[p - 1]
                img[y + dy, x + dx] = bright
    return img


# rBRIEF input.  ORB's learned test pattern is not available, so the 256 point pairs are
# drawn here (BRIEF's isotropic Gaussian sampling, sigma = 31/5), kept inside the disk of
# radius 13 so that every rotation plus the 5x5 smoothing stays within the border of 15.
BRIEF_RADIUS = 13


def brief_pattern(seed: int = 4242) -> np.ndarray:
    """256 test pairs (x1, y1, x2, y2), int8, every point inside the disk of radius 13."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.zeros((256, 4), np.int8)
    for i in range(256):
        for j in (0, 2):
            while True:
                p = np.rint(rng.normal(0.0, 31.0 / 5.0, 2))
                if p[0] * p[0] + p[1] * p[1] <= BRIEF_RADIUS * BRIEF_RADIUS:
                    break
            out[i, j], out[i, j + 1] = int(p[0]), int(p[1])
    return out


def stream_schedule(n_streams: int, duration_s: float, rate_hz: float, seed: int = 3000):
    """Poisson arrivals for ``n_streams`` cameras: list of (t_arrival, stream, frame_idx)."""
    events = []
    for s in range(n_streams):
        rng = np.random.Generator(np.random.PCG64(seed + s))
        t, k = 0.0, 0
        while True:
            t += rng.exponential(1.0 / rate_hz)
            if t >= duration_s:
                break
            events.append((t, s, k))
            k += 1
    events.sort()
    return events


def _sigma_for(seed: int) -> float:
    rng = np.random.Generator(np.random.PCG64(seed ^ 0x5EED))
    return float(rng.uniform(1.0, 6.0))


_MIXED = [(720, 540), (1080, 720), (1440, 1080), (1920, 1080)]


def _c3_specs():
    specs = []
    for i, (w, h) in enumerate(_MIXED):
        for j in range(16):
            seed = 1000 + i * 16 + j
            specs.append(FrameSpec(w, h, seed, 150, _sigma_for(seed)))
    return specs


def stream_frame_spec(stream: int, k: int) -> FrameSpec:
    w, h = _MIXED[stream % 4]
    seed = (3000 + stream) * 1_000_003 + k
    return FrameSpec(w, h, seed, 150, _sigma_for(seed))


# Workload recipes; detector parameters live with the configs that use them.
CONFIGS = {
    "c1": dict(frames=[FrameSpec(640, 480, 1, 40, 3.0)],
               params=dict(n_levels=1, fast_t=20, fast_t_min=20, cell=0, n_features=500)),
    "c2": dict(frames=[FrameSpec(1920, 1080, 2, 150, 3.0)],
               params=dict(n_levels=8, fast_t=20, fast_t_min=7, cell=30, n_features=2000)),
    "c3": dict(frames=_c3_specs(),
               params=dict(n_levels=8, fast_t=20, fast_t_min=7, cell=30, n_features=2000)),
    "c4": dict(frames=[FrameSpec(3840, 2160, 2000 + i, 600, 3.0, 8.0) for i in range(16)],
               params=dict(n_levels=12, fast_t=20, fast_t_min=7, cell=30, n_features=5000)),
    "c5": dict(frames=None,
               params=dict(n_levels=8, fast_t=20, fast_t_min=7, cell=30, n_features=2000)),
}
