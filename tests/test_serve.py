"""Served form: continuous batching with HBM-budget admission (GPU).

Every frame's keypoints from the mix equal the same frame detected alone, and the
oracle's; the resident bytes never exceed the budget."""
import numpy as np
import pytest

import oracle
from parity import assert_same_keypoints
from synth import FrameSpec, make_frame, stream_schedule

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SIZES = [(320, 240), (400, 300), (512, 384), (640, 480)]
KW = dict(n_levels=4, fast_t=20, fast_t_min=7, cell=30, n_features=500)


def log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_07164_amd import ofhip, serve
    ofhip.lib()
    pool = {}
    for s in range(8):
        for k in range(2):
            w, h = SIZES[s % 4]
            img = make_frame(FrameSpec(w, h, 500 + 10 * s + k, 40, 1.0 + (s % 5)))
            pool[(s, k)] = (torch.from_numpy(img).pin_memory(), img)
    refs = {key: oracle.detect(img, oracle.params(**KW)) for key, (_, img) in pool.items()}
    return ofhip, serve, pool, refs


def _frame_of(pool):
    return lambda s, k: (pool[(s, k % 2)][0], (s, k % 2))


def _alone(ofhip, img):
    det = ofhip.Detector([img.shape], ofhip.params(**KW))
    det.detect_batch([torch.from_numpy(img).cuda()])
    return det.results()[0]


def test_mix_equals_alone_and_oracle(env):
    ofhip, serve, pool, refs = env
    log("case: serve 8 streams, mixed sizes, rate x4")
    server = serve.Server(ofhip.params(**KW), hbm_budget=1 << 30, max_batch=8, lanes=3)
    sched = stream_schedule(8, 1.0, 30.0, seed=77)
    res, wall = serve.run_schedule(server, sched, _frame_of(pool), rate_scale=4.0)
    assert len(res) == len(sched)
    assert sorted((r.request.stream, r.request.index) for r in res) == \
        sorted((s, k) for _, s, k in sched)
    assert max(r.batch_size for r in res) > 1, "no frames were batched together"
    alone = {key: _alone(ofhip, img) for key, (_, img) in pool.items()}
    for r in res:
        key = r.request.key
        assert_same_keypoints(r.keypoints, alone[key], f"mix vs alone {key}")
        assert_same_keypoints(r.keypoints, refs[key], f"mix vs oracle {key}")
    st = serve.summarize(res, wall, 8 * 30.0 * 4)
    log(f"  {st}")
    assert st["p99_ms"] > 0 and server.in_flight == 0
    assert 0 < server.resident <= server.budget  # pools stay resident between batches
    assert any(len(l.pools) for l in server.lanes)


def test_budget_admission(env):
    """A budget that fits about two large frames in flight: launches are held back,
    resident bytes stay within the budget, results stay exact."""
    ofhip, serve, pool, refs = env
    log("case: serve under a tight HBM budget")
    p = ofhip.params(**KW)
    server = serve.Server(p, hbm_budget=1, max_batch=8, lanes=3)
    one = server.min_bytes((480, 640))
    two = server.min_bytes((480, 640)) + server.batch_bytes([(480, 640)] * 2)
    server.budget = two + one // 2
    sched = stream_schedule(8, 0.5, 30.0, seed=78)
    res, _ = serve.run_schedule(server, sched, _frame_of(pool), rate_scale=20.0)
    assert len(res) == len(sched)
    assert server.peak_resident <= server.budget
    assert server.deferred > 0
    for r in res:
        assert_same_keypoints(r.keypoints, refs[r.request.key], f"budget {r.request.key}")


def test_frame_larger_than_budget_waits_not_spins(env):
    """A budget below a single frame's bytes can never admit it: launch() reports no
    progress and leaves the frame queued (the caller decides what to do)."""
    ofhip, serve, pool, _ = env
    import collections
    server = serve.Server(ofhip.params(**KW), hbm_budget=1024, max_batch=4, lanes=2)
    q = collections.deque([serve.Request(0, 0, 0.0, pool[(0, 0)][0])])
    assert not server.launch(q)
    assert len(q) == 1 and server.deferred == 1 and server.resident == 0


def test_run_schedule_rejects_frames_over_budget(env):
    """Driven through run_schedule: frames whose batch alone exceeds the budget complete
    at once with a "rejected" status (the loop ends), the others are detected exactly."""
    ofhip, serve, pool, refs = env
    log("case: serve with frames larger than the budget")
    server = serve.Server(ofhip.params(**KW), hbm_budget=1, max_batch=4, lanes=2)
    small = server.min_bytes((240, 320))
    assert server.min_bytes((300, 400)) > small * 13 // 10
    server.budget = small * 13 // 10  # only 320x240 frames (streams 0 and 4) fit
    sched = stream_schedule(8, 0.3, 30.0, seed=79)
    res, _ = serve.run_schedule(server, sched, _frame_of(pool), rate_scale=4.0)
    assert len(res) == len(sched)
    for r in res:
        if r.request.stream % 4 == 0:
            assert r.status == "ok"
            assert_same_keypoints(r.keypoints, refs[r.request.key], f"small {r.request.key}")
        else:
            assert r.status.startswith("rejected") and len(r.keypoints) == 0
    assert server.in_flight == 0 and server.peak_resident <= server.budget
