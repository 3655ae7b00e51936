"""CPU oracle for Oriented FAST over an image pyramid (TEST INFRASTRUCTURE).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this package.  The detector product never does: it shares no code with it.

This module is a thin ctypes wrapper over ``ofref.c`` (plain C99, one thread, exact
integers); every definition and reading lives there.  The shared library is compiled
with gcc on first use when it is not already built.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboforacle.so")
_SRC = os.path.join(_HERE, "ofref.c")

__all__ = ["build", "Params", "params", "KEYPOINT_DTYPE", "check", "geometry", "resample",
           "pyramid", "run9", "segment_test", "harris", "moments", "level_detect", "detect"]


def build(force: bool = False) -> str:
    """Compile liboforacle.so with gcc (always when ``force``)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC", _SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "n_levels", "scale_num", "scale_den", "fast_t", "fast_t_min", "cell",
        "n_features", "harris_block", "patch_radius")]


KEYPOINT_DTYPE = np.dtype([("x", "<i4"), ("y", "<i4"), ("level", "<i4"), ("m10", "<i4"),
                           ("m01", "<i4"), ("pad", "<i4"), ("angle", "<f8"), ("score", "<i8")])

_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        lib = ctypes.CDLL(build())
        P = ctypes.POINTER
        u8p, i32p, i64p = P(ctypes.c_uint8), P(ctypes.c_int32), P(ctypes.c_int64)
        vp = ctypes.c_void_p
        i32 = ctypes.c_int32
        lib.ofref_check.argtypes = [i32, i32, P(Params)]
        lib.ofref_geometry.argtypes = [i32, i32, P(Params), i32p, i32p, i32p, i32p, i32p]
        lib.ofref_resample.argtypes = [u8p, i32, i32, i32, u8p, i32, i32]
        lib.ofref_resample.restype = None
        lib.ofref_run9.argtypes = [ctypes.c_uint32]
        lib.ofref_segment_test.argtypes = [u8p, i32, i32, i32, i32]
        lib.ofref_harris.argtypes = [u8p, i32, i32, i32, i32]
        lib.ofref_harris.restype = ctypes.c_int64
        lib.ofref_moments.argtypes = [u8p, i32, i32, i32, i32, i32p, i32p]
        lib.ofref_moments.restype = None
        i8p = ctypes.POINTER(ctypes.c_int8)
        lib.ofref_brief_tables.argtypes = [i8p, i8p, i32p]
        lib.ofref_brief_tables.restype = None
        lib.ofref_describe.argtypes = [u8p, i32, i32, i32, i32, i32, i8p, i32p,
                                       ctypes.POINTER(ctypes.c_uint8)]
        lib.ofref_describe.restype = None
        lib.ofref_level_detect.argtypes = [u8p, i32, i32, i32, P(Params), i32, i32, i32,
                                           u8p, u8p, i64p, u8p, vp]
        lib.ofref_pyramid_level.argtypes = [u8p, i32, i32, i32, P(Params), i32, u8p]
        lib.ofref_detect.argtypes = [u8p, i32, i32, i32, P(Params), vp, i32]
        _lib_handle = lib
    return _lib_handle


def params(n_levels=8, scale_num=6, scale_den=5, fast_t=20, fast_t_min=7, cell=30,
           n_features=2000, harris_block=7, patch_radius=15) -> Params:
    return Params(n_levels, scale_num, scale_den, fast_t, fast_t_min, cell, n_features,
                  harris_block, patch_radius)


def _u8(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _img(img):
    img = np.asarray(img)
    assert img.dtype == np.uint8 and img.ndim == 2
    if not img.flags.c_contiguous:
        img = np.ascontiguousarray(img)
    return img


def check(W: int, H: int, p: Params) -> bool:
    return _lib().ofref_check(W, H, ctypes.byref(p)) == 0


def geometry(W: int, H: int, p: Params) -> dict:
    L = p.n_levels
    arrs = {k: np.zeros(16, np.int32) for k in ("width", "height", "quota", "k_cell", "n_cells")}
    ptr = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    n = _lib().ofref_geometry(W, H, ctypes.byref(p), ptr(arrs["width"]), ptr(arrs["height"]),
                              ptr(arrs["quota"]), ptr(arrs["k_cell"]), ptr(arrs["n_cells"]))
    if n < 0:
        raise ValueError("oracle rejects the parameters / frame size")
    return {k: v[:L].copy() for k, v in arrs.items()}


def resample(img, Wl: int, Hl: int) -> np.ndarray:
    img = _img(img)
    H, W = img.shape
    out = np.empty((Hl, Wl), np.uint8)
    _lib().ofref_resample(_u8(img), W, H, img.strides[0], _u8(out), Wl, Hl)
    return out


def pyramid(img, p: Params) -> list:
    img = _img(img)
    H, W = img.shape
    g = geometry(W, H, p)
    levels = [img.copy()]
    for l in range(1, p.n_levels):
        levels.append(resample(img, int(g["width"][l]), int(g["height"][l])))
    return levels


def run9(mask16: int) -> bool:
    return bool(_lib().ofref_run9(mask16 & 0xFFFF))


def segment_test(img, x: int, y: int, t: int) -> bool:
    img = _img(img)
    return bool(_lib().ofref_segment_test(_u8(img), img.strides[0], x, y, t))


def harris(img, x: int, y: int, block: int = 7) -> int:
    img = _img(img)
    return int(_lib().ofref_harris(_u8(img), img.strides[0], x, y, block))


def moments(img, x: int, y: int, r: int = 15):
    img = _img(img)
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _lib().ofref_moments(_u8(img), img.strides[0], x, y, r, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def brief_tables(pattern):
    """(rot [30, 256, 4] int8, centres [30, 2] int32): the steered copies of `pattern`."""
    pattern = np.ascontiguousarray(pattern, dtype=np.int8)
    rot = np.zeros((30, 256, 4), np.int8)
    centres = np.zeros((30, 2), np.int32)
    _lib().ofref_brief_tables(pattern.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                              rot.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                              centres.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return rot, centres


def describe(img, keypoints, rot, centres) -> np.ndarray:
    """rBRIEF of each keypoint (fields x, y, m10, m01) on level image `img`: (n, 32) uint8."""
    img = _img(img)
    rot = np.ascontiguousarray(rot, dtype=np.int8)
    centres = np.ascontiguousarray(centres, dtype=np.int32)
    out = np.zeros((len(keypoints), 32), np.uint8)
    for i, kp in enumerate(keypoints):
        _lib().ofref_describe(_u8(img), img.strides[0], int(kp["x"]), int(kp["y"]),
                              int(kp["m10"]), int(kp["m01"]),
                              rot.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                              centres.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              out[i].ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    return out


def level_detect(lvl, p: Params, level: int = 0, k_cell: int | None = None,
                 n_keep: int | None = None) -> dict:
    """Run the per-level stages on one level image; returns maps and the level keypoints."""
    lvl = _img(lvl)
    Hl, Wl = lvl.shape
    cs = p.cell if p.cell > 0 else max(Wl, Hl)
    ncx, ncy = -(-Wl // cs), -(-Hl // cs)
    if k_cell is None:
        k_cell = max(1, -(-p.n_features // (ncx * ncy))) if p.cell > 0 else p.n_features
    if n_keep is None:
        n_keep = p.n_features
    cand = np.zeros((Hl, Wl), np.uint8)
    surv = np.zeros((Hl, Wl), np.uint8)
    score = np.zeros((Hl, Wl), np.int64)
    flags = np.zeros((ncy, ncx), np.uint8)
    out = np.zeros(max(1, n_keep), KEYPOINT_DTYPE)
    n = _lib().ofref_level_detect(
        _u8(lvl), Wl, Hl, lvl.strides[0], ctypes.byref(p), level, k_cell, n_keep, _u8(cand),
        _u8(surv), score.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _u8(flags),
        out.ctypes.data)
    if n < 0:
        raise ValueError("oracle level_detect failed")
    return dict(cand=cand, surv=surv, score=score, flags=flags, keypoints=out[:n].copy())


def detect(img, p: Params) -> np.ndarray:
    """Whole pipeline; structured array with KEYPOINT_DTYPE in canonical order."""
    img = _img(img)
    H, W = img.shape
    out = np.zeros(p.n_features, KEYPOINT_DTYPE)
    n = _lib().ofref_detect(_u8(img), W, H, img.strides[0], ctypes.byref(p), out.ctypes.data,
                            p.n_features)
    if n < 0:
        raise ValueError("oracle rejects the parameters / frame size")
    return out[:n].copy()
