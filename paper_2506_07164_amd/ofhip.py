"""Python binding of the C ABI in include/of.h (argument marshalling only).

Every function of the header has a ctypes twin with the same name; the helpers below
take torch tensors for device memory and the current torch stream.  All detection work
runs in libof_hip.so; if that library is missing this module raises instead of falling
back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libof_hip.so")

OF_OK, OF_EINVAL, OF_ENOSPACE, OF_EHIP = 0, -1, -2, -3
OF_MAX_LEVELS = 16
OF_MAX_BATCH = 64


class OfImage(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("stride", ctypes.c_int32)]


class OfParams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "n_levels", "scale_num", "scale_den", "fast_t", "fast_t_min", "cell", "n_features",
        "harris_block", "patch_radius")]


class OfKeypoint(ctypes.Structure):
    _fields_ = [("x", ctypes.c_int32), ("y", ctypes.c_int32), ("level", ctypes.c_int32),
                ("m10", ctypes.c_int32), ("m01", ctypes.c_int32), ("angle", ctypes.c_float),
                ("score", ctypes.c_int64)]


class OfPyramidDesc(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32),
                ("width", ctypes.c_int32 * 16), ("height", ctypes.c_int32 * 16),
                ("stride", ctypes.c_int32 * 16), ("quota", ctypes.c_int32 * 16),
                ("offset", ctypes.c_int64 * 16), ("total_bytes", ctypes.c_int64)]


class OfTuning(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "mark_words", "mark_rows", "det_cells_x", "det_cells_y", "det_w", "det_h",
        "mark_grid", "det_grid", "pyr_pass", "mark_order", "plan_resident", "det_order")]


KEYPOINT_DTYPE = np.dtype([("x", "<i4"), ("y", "<i4"), ("level", "<i4"), ("m10", "<i4"),
                           ("m01", "<i4"), ("angle", "<f4"), ("score", "<i8")])
assert KEYPOINT_DTYPE.itemsize == ctypes.sizeof(OfKeypoint) == 32

_lib = None


def lib() -> ctypes.CDLL:
    """Load libof_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first "
                               "(python -m paper_2506_07164_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp, i32, i64p = ctypes.c_void_p, ctypes.c_int32, P(ctypes.c_int64)
        L.of_pyramid_desc_get.argtypes = [i32, i32, P(OfParams), P(OfPyramidDesc)]
        L.of_pyramid_build.argtypes = [P(OfImage), P(OfParams), vp, vp]
        L.of_workspace_size.argtypes = [P(OfImage), i32, P(OfParams), P(ctypes.c_size_t)]
        L.of_detect.argtypes = [P(OfImage), P(OfParams), vp, ctypes.c_size_t, vp, i32, vp, vp]
        L.of_detect_batch.argtypes = [P(OfImage), i32, P(OfParams), vp, ctypes.c_size_t, vp,
                                      i64p, i32, vp, P(OfTuning), vp]
        L.of_detect_batch_scratch.argtypes = [P(OfImage), i32, P(OfParams), vp, i64p, i32, vp,
                                              P(OfTuning), vp]
        L.of_tuning_default.argtypes = [P(OfImage), i32, P(OfParams), P(OfTuning)]
        L.of_test_segment.argtypes = [vp, i32, i32, i32, vp, vp]
        L.of_candidate_counts.argtypes = [P(OfImage), i32, P(OfParams), vp, vp, vp]
        L.of_brief_tables.argtypes = [vp, vp, vp]
        L.of_describe.argtypes = [P(OfImage), i32, P(OfParams), P(OfTuning), vp, vp, i64p, vp,
                                  vp, vp, vp, vp]
        L.of_ablate_fast.argtypes = [P(OfImage), i32, i32, i32, i32, P(vp), vp]
        L.of_ablate_harris.argtypes = [P(OfImage), i32, P(vp), P(i32), i32, P(vp), vp]
        L.of_profile_enable.argtypes = [ctypes.c_int]
        L.of_profile_read.argtypes = [P(ctypes.c_double), i64p, i32]
        L.of_status_string.argtypes = [ctypes.c_int]
        L.of_status_string.restype = ctypes.c_char_p
        L.of_last_hip_error.argtypes = []
        _lib = L
    return _lib


class OfError(RuntimeError):
    def __init__(self, status: int, what: str):
        msg = lib().of_status_string(status).decode()
        if status == OF_EHIP:
            msg += f" (hipError {lib().of_last_hip_error()})"
        super().__init__(f"{what}: {msg}")
        self.status = status


def _check(status: int, what: str) -> None:
    if status != OF_OK:
        raise OfError(status, what)


def params(n_levels=8, scale_num=6, scale_den=5, fast_t=20, fast_t_min=7, cell=30,
           n_features=2000, harris_block=7, patch_radius=15) -> OfParams:
    return OfParams(n_levels, scale_num, scale_den, fast_t, fast_t_min, cell, n_features,
                    harris_block, patch_radius)


def tuning(**kw) -> OfTuning:
    t = OfTuning()
    t.mark_grid = -1
    t.det_grid = -1
    t.pyr_pass = -1
    t.mark_order = -1
    t.plan_resident = -1
    t.det_order = -1
    for k, v in kw.items():
        setattr(t, k, v)
    return t


# ------------------------------------------------------------- C-ABI twins --

def of_pyramid_desc_get(width: int, height: int, p: OfParams) -> OfPyramidDesc:
    d = OfPyramidDesc()
    _check(lib().of_pyramid_desc_get(width, height, ctypes.byref(p), ctypes.byref(d)),
           "of_pyramid_desc_get")
    return d


def of_workspace_size(images, p: OfParams) -> int:
    arr = (OfImage * len(images))(*images)
    n = ctypes.c_size_t()
    _check(lib().of_workspace_size(arr, len(images), ctypes.byref(p), ctypes.byref(n)),
           "of_workspace_size")
    return n.value


def of_tuning_default(images, p: OfParams) -> OfTuning:
    arr = (OfImage * len(images))(*images)
    t = OfTuning()
    _check(lib().of_tuning_default(arr, len(images), ctypes.byref(p), ctypes.byref(t)),
           "of_tuning_default")
    return t


def of_pyramid_build(image: OfImage, p: OfParams, levels_ptr: int, stream: int) -> None:
    _check(lib().of_pyramid_build(ctypes.byref(image), ctypes.byref(p), levels_ptr, stream),
           "of_pyramid_build")


def of_detect(image: OfImage, p: OfParams, ws_ptr: int, ws_bytes: int, out_ptr: int, cap: int,
              count_ptr: int, stream: int) -> None:
    _check(lib().of_detect(ctypes.byref(image), ctypes.byref(p), ws_ptr, ws_bytes, out_ptr,
                           cap, count_ptr, stream), "of_detect")


def of_detect_batch(images, p: OfParams, ws_ptr: int, ws_bytes: int, out_ptr: int, out_offsets,
                    cap_per_frame: int, counts_ptr: int, tune: OfTuning | None, stream: int) -> None:
    n = len(images)
    arr = (OfImage * n)(*images)
    offs = (ctypes.c_int64 * n)(*[int(o) for o in out_offsets])
    _check(lib().of_detect_batch(arr, n, ctypes.byref(p), ws_ptr, ws_bytes, out_ptr, offs,
                                 cap_per_frame, counts_ptr,
                                 ctypes.byref(tune) if tune is not None else None, stream),
           "of_detect_batch")


OF_SCRATCH_BYTES = 64 * 1024 * 1024


def of_detect_batch_scratch(images, p: OfParams, out_ptr: int, out_offsets, cap_per_frame: int,
                            counts_ptr: int, tune: OfTuning | None, stream: int) -> None:
    n = len(images)
    arr = (OfImage * n)(*images)
    offs = (ctypes.c_int64 * n)(*[int(o) for o in out_offsets])
    _check(lib().of_detect_batch_scratch(arr, n, ctypes.byref(p), out_ptr, offs, cap_per_frame,
                                         counts_ptr, ctypes.byref(tune) if tune is not None
                                         else None, stream), "of_detect_batch_scratch")


def of_candidate_counts(images, p: OfParams, ws_ptr: int, out_ptr: int, stream: int) -> None:
    n = len(images)
    arr = (OfImage * n)(*images)
    _check(lib().of_candidate_counts(arr, n, ctypes.byref(p), ws_ptr, out_ptr, stream),
           "of_candidate_counts")


def of_brief_tables(pattern):
    """(rot [30, 256, 4] int8, centres [30, 2] int32) for a 256 x 4 int8 test pattern."""
    pattern = np.ascontiguousarray(pattern, dtype=np.int8)
    assert pattern.shape == (256, 4)
    rot = np.zeros((30, 256, 4), np.int8)
    centres = np.zeros((30, 2), np.int32)
    _check(lib().of_brief_tables(pattern.ctypes.data, rot.ctypes.data, centres.ctypes.data),
           "of_brief_tables")
    return rot, centres


def of_describe(images, p: OfParams, tune, ws_ptr: int, kps_ptr: int, kp_offsets, counts_ptr: int,
                rot_ptr: int, centres_ptr: int, desc_ptr: int, stream: int) -> None:
    n = len(images)
    arr = (OfImage * n)(*images)
    offs = (ctypes.c_int64 * n)(*[int(o) for o in kp_offsets])
    _check(lib().of_describe(arr, n, ctypes.byref(p), ctypes.byref(tune) if tune is not None
                             else None, ws_ptr, kps_ptr, offs, counts_ptr, rot_ptr,
                             centres_ptr, desc_ptr, stream), "of_describe")


AB_FAST = {"branchy": 0, "masks": 1, "masks_lds": 2, "minmax_lds": 3, "masks_pretest_lds": 4}
AB_HARRIS = {"2d": 0, "separable": 1, "groups": 2, "dense_sliding": 3}


def of_ablate_fast(levels, t: int, border: int, variant: int, out_ptrs, stream: int) -> None:
    """levels: OfImage list (device images); out_ptrs: device uint8 maps, one per level."""
    n = len(levels)
    arr = (OfImage * n)(*levels)
    outs = (ctypes.c_void_p * n)(*out_ptrs)
    _check(lib().of_ablate_fast(arr, n, t, border, variant, outs, stream), "of_ablate_fast")


def of_ablate_harris(levels, pos_ptrs, counts, variant: int, out_ptrs, stream: int) -> None:
    """pos_ptrs/counts: device (y << 16 | x) arrays and their lengths, one per level (None
    for the dense variant); out_ptrs: device int64 outputs."""
    n = len(levels)
    arr = (OfImage * n)(*levels)
    outs = (ctypes.c_void_p * n)(*out_ptrs)
    pp = (ctypes.c_void_p * n)(*pos_ptrs) if pos_ptrs is not None else None
    cc = (ctypes.c_int32 * n)(*counts) if counts is not None else None
    _check(lib().of_ablate_harris(arr, n, pp, cc, variant, outs, stream), "of_ablate_harris")


def of_test_segment(circles_ptr: int, n: int, t_lo: int, t_hi: int, out_ptr: int,
                    stream: int) -> None:
    _check(lib().of_test_segment(circles_ptr, n, t_lo, t_hi, out_ptr, stream), "of_test_segment")


OF_PROFILE_STEPS = 8
PROFILE_STEP_NAMES = ["prologue", "pyramid", "segment_test", "harris_nms_cells", "select",
                      "select_lists", "ablate_fast", "ablate_harris"]


def of_profile_enable(on) -> None:
    """False/0 off, True/1 events per step launch, n > 1 also repeats each repeatable
    launch n times between its events (kernel-only durations)."""
    _check(lib().of_profile_enable(int(on)), "of_profile_enable")


def of_profile_read():
    """{step name: (total ms, launches)} since the last read (waits for the events)."""
    ms = (ctypes.c_double * OF_PROFILE_STEPS)()
    n = (ctypes.c_int64 * OF_PROFILE_STEPS)()
    _check(lib().of_profile_read(ms, n, OF_PROFILE_STEPS), "of_profile_read")
    return {PROFILE_STEP_NAMES[i]: (ms[i], n[i]) for i in range(OF_PROFILE_STEPS)}


# ----------------------------------------------------------- torch helpers --

def _torch():
    import torch
    return torch


def image_of(t) -> OfImage:
    """OfImage describing a 2-D uint8 CUDA tensor (rows may be strided)."""
    assert t.dtype == _torch().uint8 and t.dim() == 2 and t.is_cuda and t.stride(1) == 1
    return OfImage(t.data_ptr(), t.shape[1], t.shape[0], t.stride(0))


def stream_ptr(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def alloc_workspace(images, p: OfParams, device="cuda"):
    torch = _torch()
    n = of_workspace_size(images, p)
    return torch.empty(n, dtype=torch.uint8, device=device)


def keypoints_to_numpy(raw, count: int) -> np.ndarray:
    """View a (cap, 32) uint8 tensor of of_keypoint records as a structured array."""
    a = raw[:count].cpu().numpy()
    return np.ascontiguousarray(a).view(KEYPOINT_DTYPE).reshape(-1)


class Detector:
    """Owns a workspace and output buffers for repeated detection on fixed shapes."""

    def __init__(self, shapes, p: OfParams, device="cuda", resident: bool = False):
        """resident: the workspace belongs to this detector alone, so batched calls keep
        their plan resident (of_tuning.plan_resident) and skip re-planning."""
        torch = _torch()
        self.p = p
        self.resident = resident
        self.shapes = list(shapes)  # [(H, W), ...]
        self.n = len(self.shapes)
        dummy = [OfImage(None, w, h, w) for h, w in self.shapes]
        self.ws = alloc_workspace(dummy, p, device)
        self.cap = p.n_features
        self.out = torch.empty((self.n * self.cap, 32), dtype=torch.uint8, device=device)
        self.counts = torch.zeros(self.n, dtype=torch.int32, device=device)
        self.offsets = [i * self.cap for i in range(self.n)]

    def detect_plain(self, frame, stream=None):
        assert self.n == 1
        of_detect(image_of(frame), self.p, self.ws.data_ptr(), self.ws.numel(),
                  self.out.data_ptr(), self.cap, self.counts.data_ptr(), stream_ptr(stream))

    def _tune(self, tune):
        if not self.resident:
            return tune
        t = OfTuning()
        ctypes.memmove(ctypes.byref(t), ctypes.byref(tune if tune is not None else tuning()),
                       ctypes.sizeof(OfTuning))
        t.plan_resident = 1
        return t

    def detect_batch(self, frames, tune: OfTuning | None = None, stream=None):
        assert len(frames) == self.n
        of_detect_batch([image_of(f) for f in frames], self.p, self.ws.data_ptr(),
                        self.ws.numel(), self.out.data_ptr(), self.offsets, self.cap,
                        self.counts.data_ptr(), self._tune(tune), stream_ptr(stream))

    def candidates(self, frames, stream=None):
        """FAST candidates per (frame, level) of the last detection (synchronises)."""
        torch = _torch()
        out = torch.zeros(self.n * self.p.n_levels, dtype=torch.int32, device=self.ws.device)
        of_candidate_counts([image_of(f) for f in frames], self.p, self.ws.data_ptr(),
                            out.data_ptr(), stream_ptr(stream))
        return out.cpu().numpy().reshape(self.n, self.p.n_levels)

    def describe(self, frames, rot, centres, tune: OfTuning | None = None, stream=None):
        """rBRIEF of the last detection's keypoints: device (n * cap, 32) uint8; rot and
        centres are device tensors from of_brief_tables."""
        torch = _torch()
        desc = torch.zeros((self.n * self.cap, 32), dtype=torch.uint8, device=self.ws.device)
        of_describe([image_of(f) for f in frames], self.p, self._tune(tune), self.ws.data_ptr(),
                    self.out.data_ptr(), self.offsets, self.counts.data_ptr(), rot.data_ptr(),
                    centres.data_ptr(), desc.data_ptr(), stream_ptr(stream))
        return desc

    def results(self):
        """Per frame, a structured numpy array of its keypoints (synchronises)."""
        counts = self.counts.cpu().tolist()
        out = self.out.cpu().numpy()
        res = []
        for i, c in enumerate(counts):
            a = out[self.offsets[i]:self.offsets[i] + c]
            res.append(np.ascontiguousarray(a).view(KEYPOINT_DTYPE).reshape(-1))
        return res
