"""of_detect_batch_scratch, the entry point on the library's static workspace, against
of_detect_batch on a caller workspace: bit-exact keypoints and counts on two calls in a
row, the second with a smaller batch (GPU).  Also checked against the oracle."""
import numpy as np
import pytest

import oracle
from parity import assert_same_keypoints
from synth import FrameSpec, make_frame

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


def _scratch_call(hip, frames, p):
    n, N = len(frames), p.n_features
    out = torch.zeros((n * N, 32), dtype=torch.uint8, device="cuda")
    counts = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    offs = [i * N for i in range(n)]
    hip.of_detect_batch_scratch([hip.image_of(f) for f in frames], p, out.data_ptr(), offs, N,
                                counts.data_ptr(), None, hip.stream_ptr())
    torch.cuda.synchronize()
    c = counts.cpu().tolist()
    raw = out.cpu().numpy()
    return [np.ascontiguousarray(raw[o:o + k]).view(hip.KEYPOINT_DTYPE).reshape(-1)
            for o, k in zip(offs, c)]


def _workspace_call(hip, frames, p):
    det = hip.Detector([tuple(f.shape) for f in frames], p)
    det.detect_batch(frames)
    return det.results()


def test_scratch_matches_workspace_call_twice_smaller_second(hip):
    kw = dict(n_levels=4, fast_t=20, fast_t_min=7, cell=30, n_features=800)
    p = hip.params(**kw)
    specs = [FrameSpec(640, 480, 901, 40, 2.0), FrameSpec(512, 384, 902, 40, 3.0),
             FrameSpec(800, 600, 903, 60, 2.5)]
    imgs = [make_frame(s) for s in specs]
    frames = [torch.from_numpy(i).cuda() for i in imgs]
    for rep, sub in enumerate([[0, 1, 2], [1]]):
        log(f"case: static workspace call {rep}, frames {sub}")
        fs = [frames[i] for i in sub]
        got = _scratch_call(hip, fs, p)
        want = _workspace_call(hip, fs, p)
        for k, i in enumerate(sub):
            assert_same_keypoints(got[k], want[k], f"call {rep} frame {i} vs workspace call")
            assert_same_keypoints(got[k], oracle.detect(imgs[i], oracle.params(**kw)),
                                  f"call {rep} frame {i} vs oracle")


def test_scratch_rejects_batches_beyond_its_size(hip):
    kw = dict(n_levels=8, n_features=2000)
    p = hip.params(**kw)
    imgs = [hip.OfImage(0x1000, 1920, 1080, 1920)] * 16
    assert hip.of_workspace_size(imgs, p) > hip.OF_SCRATCH_BYTES
    frame = torch.zeros((1080, 1920), dtype=torch.uint8, device="cuda")
    out = torch.zeros((16 * 2000, 32), dtype=torch.uint8, device="cuda")
    counts = torch.zeros(16, dtype=torch.int32, device="cuda")
    with pytest.raises(hip.OfError) as err:
        hip.of_detect_batch_scratch([hip.image_of(frame)] * 16, p, out.data_ptr(),
                                    [i * 2000 for i in range(16)], 2000, counts.data_ptr(),
                                    None, hip.stream_ptr())
    assert err.value.status == hip.OF_ENOSPACE
