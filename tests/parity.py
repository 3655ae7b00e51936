"""Comparison of GPU keypoints with the oracle's (test helper).

x, y, level, moments and R' must be bit-exact and in the same order; the angle (float32
atan2 on the GPU, double on the CPU) must agree within 1e-5 rad, wrapped."""
import numpy as np

ANGLE_TOL = 1e-5


def assert_same_keypoints(got, ref, what=""):
    assert len(got) == len(ref), f"{what}: {len(got)} keypoints vs oracle {len(ref)}"
    for k in ("x", "y", "level", "m10", "m01", "score"):
        g, r = got[k].astype(np.int64), ref[k].astype(np.int64)
        if not np.array_equal(g, r):
            i = int(np.nonzero(g != r)[0][0])
            raise AssertionError(f"{what}: field {k} differs first at {i}: "
                                 f"gpu {got[i]} oracle {ref[i]}")
    if len(got):
        d = np.abs(got["angle"].astype(np.float64) - ref["angle"])
        d = np.minimum(d, 2 * np.pi - d)
        assert d.max() <= ANGLE_TOL, f"{what}: angle off by {d.max()}"
