"""Served form: continuous batching of camera frames on one GPU.

Frames arrive from many camera streams in host memory (pinned), as a capture pipeline
delivers them.  The server keeps a FIFO of arrived frames and a few HIP streams
("lanes").  Whenever a lane is free it admits the oldest waiting frames into one batch,
as long as the batch holds at most ``max_batch`` frames and the device-resident bytes
of all batches in flight (frames, workspace with the level buffers, keypoints) stay
within ``hbm_budget``.  On its lane the batch is copied to the device, detected with
one ``of_detect_batch`` call and its keypoints copied back; batches on different lanes
overlap on the device.  A batch's frames complete, and its bytes return to the
budget, when its results are host-visible.  Frames that arrive while others are on
the device join the next batch as soon as a lane and budget free up: that is the
continuous part, there is no fixed batch window.

Latency is measured from a frame's arrival time to the moment its keypoints are
host-visible.  ``run_schedule`` replays Poisson camera schedules in real time and
reports p50/p99 latency and frames/s.

Run ``python -m paper_2506_07164_amd.serve`` for the 32-stream workload (720x540 to
1920x1080, 30 fps per stream) at the offered rate and at scaled rates.
"""
from __future__ import annotations

import argparse
import collections
import json
import time
from dataclasses import dataclass, field

import numpy as np

from . import ofhip


@dataclass
class Request:
    stream: int
    index: int
    t_arrival: float            # seconds on the server clock
    host: object                # pinned uint8 torch tensor (H, W)
    key: object = None          # caller's tag (e.g. which pre-generated frame)


@dataclass
class Result:
    request: Request
    keypoints: np.ndarray       # KEYPOINT_DTYPE, canonical order (empty unless status "ok")
    t_done: float
    batch_size: int
    status: str = "ok"          # "ok", "rejected: ..." (never admissible) or "error: ..."

    @property
    def latency(self) -> float:
        return self.t_done - self.request.t_arrival


@dataclass
class _Lane:
    stream: object
    out_host: object            # pinned (max_batch * N) keypoints, as uint8 bytes
    counts_host: object         # pinned int32 (max_batch)
    busy: bool = False
    batch: list = field(default_factory=list)
    event: object = None
    device: list = field(default_factory=list)   # tensors kept alive while in flight
    nbytes: int = 0


class Server:
    """Continuous-batching detector over a fixed set of HIP streams."""

    def __init__(self, params: ofhip.OfParams, hbm_budget: int = 4 << 30, max_batch: int = 16,
                 lanes: int = 3, tune: ofhip.OfTuning | None = None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the served form needs a GPU")
        if max_batch < 1 or max_batch > ofhip.OF_MAX_BATCH:
            raise ValueError("max_batch out of range")
        self.torch = torch
        self.p = params
        self.N = params.n_features
        self.budget = int(hbm_budget)
        self.max_batch = max_batch
        self.tune = tune
        self.resident = 0
        self.peak_resident = 0
        self.deferred = 0        # launches held back by the budget
        self.failed = 0          # frames whose detection call returned an error
        self.batches = 0
        kp = ofhip.KEYPOINT_DTYPE.itemsize
        self.lanes = []
        for _ in range(lanes):
            self.lanes.append(_Lane(
                stream=torch.cuda.Stream(),
                out_host=torch.empty(max_batch * self.N * kp, dtype=torch.uint8, pin_memory=True),
                counts_host=torch.empty(max_batch, dtype=torch.int32, pin_memory=True)))
        self._ws_cache = {}

    # -- sizing -------------------------------------------------------------------
    def _workspace_bytes(self, shapes):
        key = tuple(shapes)
        n = self._ws_cache.get(key)
        if n is None:
            imgs = [ofhip.OfImage(0x1000, w, h, w) for (h, w) in shapes]
            n = ofhip.of_workspace_size(imgs, self.p)
            self._ws_cache[key] = n
        return n

    def batch_bytes(self, shapes) -> int:
        """Device bytes of one batch: frames, workspace (plans, bitmaps, slots, levels),
        keypoints and counts."""
        frames = sum(h * w for (h, w) in shapes)
        out = len(shapes) * self.N * ofhip.KEYPOINT_DTYPE.itemsize + 4 * len(shapes)
        return frames + self._workspace_bytes(shapes) + out

    @property
    def in_flight(self) -> int:
        return sum(len(l.batch) for l in self.lanes if l.busy)

    # -- the loop -----------------------------------------------------------------
    def reject_oversized(self, queue: collections.deque, clock, done: list) -> int:
        """Frames whose batch alone exceeds the HBM budget can never be admitted: each
        leaves the queue at once with a "rejected" result instead of waiting forever."""
        keep, k = collections.deque(), 0
        while queue:
            r = queue.popleft()
            shp = tuple(r.host.shape)
            if self.batch_bytes([shp]) > self.budget:
                done.append(Result(r, np.empty(0, ofhip.KEYPOINT_DTYPE), clock(), 0,
                                   "rejected: one frame exceeds the HBM budget"))
                k += 1
            else:
                keep.append(r)
        queue.extend(keep)
        return k

    def launch(self, queue: collections.deque, clock=None, done: list | None = None) -> bool:
        """Admits the oldest waiting frames into a batch on a free lane, within the
        batch size and the HBM budget.  Returns True if a batch was launched.  If the
        detection call fails, the batch's frames complete with an "error" result (when
        ``done`` is given) or are put back at the head of the queue."""
        if not queue:
            return False
        lane = next((l for l in self.lanes if not l.busy), None)
        if lane is None:
            return False
        batch, shapes, nbytes = [], [], 0
        while queue and len(batch) < self.max_batch:
            shp = tuple(queue[0].host.shape)
            b = self.batch_bytes(shapes + [shp])
            if self.resident + b > self.budget:
                break
            batch.append(queue.popleft())
            shapes.append(shp)
            nbytes = b
        if not batch:
            self.deferred += 1
            return False
        torch = self.torch
        n = len(batch)
        kp = ofhip.KEYPOINT_DTYPE.itemsize
        try:
            with torch.cuda.stream(lane.stream):
                frames = [torch.empty(s, dtype=torch.uint8, device="cuda") for s in shapes]
                for f, r in zip(frames, batch):
                    f.copy_(r.host, non_blocking=True)
                ws = torch.empty(self._workspace_bytes(shapes), dtype=torch.uint8, device="cuda")
                out = torch.empty(n * self.N * kp, dtype=torch.uint8, device="cuda")
                counts = torch.empty(n, dtype=torch.int32, device="cuda")
                offs = [i * self.N for i in range(n)]
                ofhip.of_detect_batch([ofhip.image_of(f) for f in frames], self.p, ws.data_ptr(),
                                      ws.numel(), out.data_ptr(), offs, self.N, counts.data_ptr(),
                                      self.tune, lane.stream.cuda_stream)
                lane.out_host[: n * self.N * kp].copy_(out, non_blocking=True)
                lane.counts_host[:n].copy_(counts, non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(lane.stream)
        except ofhip.OfError as err:
            self.failed += n
            if done is None:
                queue.extendleft(reversed(batch))
            else:
                t = clock() if clock else 0.0
                for r in batch:
                    done.append(Result(r, np.empty(0, ofhip.KEYPOINT_DTYPE), t, n, f"error: {err}"))
            return False
        lane.busy, lane.batch, lane.event = True, batch, ev
        lane.device, lane.nbytes = [frames, ws, out, counts], nbytes
        self.resident += nbytes
        self.peak_resident = max(self.peak_resident, self.resident)
        self.batches += 1
        return True

    def poll(self, clock, done: list) -> int:
        """Completes every batch whose results are host-visible; returns how many frames."""
        k = 0
        for lane in self.lanes:
            if lane.busy and lane.event.query():
                t = clock()
                n = len(lane.batch)
                counts = lane.counts_host[:n].numpy().copy()
                raw = lane.out_host[: n * self.N * ofhip.KEYPOINT_DTYPE.itemsize].numpy()
                kps = raw.view(ofhip.KEYPOINT_DTYPE).reshape(n, self.N)
                for i, r in enumerate(lane.batch):
                    done.append(Result(r, kps[i, : counts[i]].copy(), t, n))
                k += n
                self.resident -= lane.nbytes
                lane.busy, lane.batch, lane.event, lane.device, lane.nbytes = False, [], None, [], 0
        return k

    def drain(self, clock, done: list) -> None:
        while any(l.busy for l in self.lanes):
            if not self.poll(clock, done):
                time.sleep(50e-6)


def run_schedule(server: Server, arrivals, frame_of, rate_scale: float = 1.0):
    """Replays ``arrivals`` = [(t, stream, index)] in real time (times divided by
    ``rate_scale``); ``frame_of(stream, index)`` returns (pinned host frame, key).
    Returns the results in completion order and the wall time."""
    queue = collections.deque()
    done = []
    t0 = time.perf_counter()

    def clock():
        return time.perf_counter() - t0

    i = 0
    while i < len(arrivals) or queue or server.in_flight:
        now = clock()
        while i < len(arrivals) and arrivals[i][0] / rate_scale <= now:
            t, s, k = arrivals[i]
            host, key = frame_of(s, k)
            queue.append(Request(s, k, t / rate_scale, host, key))
            i += 1
        progressed = server.poll(clock, done) > 0
        progressed = server.reject_oversized(queue, clock, done) > 0 or progressed
        while server.launch(queue, clock, done):
            progressed = True
        if not progressed:
            nxt = arrivals[i][0] / rate_scale - clock() if i < len(arrivals) else 0.0
            time.sleep(min(max(nxt, 0.0), 200e-6) if nxt > 0 else 20e-6)
    return done, clock()


def summarize(results, wall, offered_fps):
    lat = np.array([r.latency for r in results]) * 1e3
    bs = np.array([r.batch_size for r in results])
    return {"frames": len(results), "offered_fps": round(offered_fps, 1),
            "fps": round(len(results) / wall, 1),
            "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "max_ms": round(float(lat.max()), 3),
            "mean_batch": round(float(bs.mean()), 2)}


def camera_pool(n_streams: int, per_stream: int):
    """Pinned host frames for each stream (the stream's first ``per_stream`` frames;
    frame k of a stream reuses pool entry k mod per_stream, since generating frames is
    slower than real time)."""
    import torch
    from synth import make_frame, stream_frame_spec
    pool = {}
    for s in range(n_streams):
        for k in range(per_stream):
            img = make_frame(stream_frame_spec(s, k))
            pool[(s, k)] = (torch.from_numpy(img).pin_memory(), img)
    return pool


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--streams", type=int, default=32)
    ap.add_argument("--rate", type=float, default=30.0, help="frames/s per stream")
    ap.add_argument("--duration", type=float, default=2.0,
                    help="seconds of arrivals at the base rate (divided by each scale)")
    ap.add_argument("--scales", type=str, default="1,8,32", help="arrival-rate multipliers")
    ap.add_argument("--budget-mib", type=int, default=4096)
    ap.add_argument("--max-batch", type=int, default=16)
    ap.add_argument("--lanes", type=int, default=3)
    ap.add_argument("--pool", type=int, default=2)
    args = ap.parse_args()
    import torch
    from synth import CONFIGS, stream_schedule
    p = ofhip.params(**CONFIGS["c2"]["params"])
    pool = camera_pool(args.streams, args.pool)
    server = Server(p, hbm_budget=args.budget_mib << 20, max_batch=args.max_batch,
                    lanes=args.lanes)

    def frame_of(s, k):
        return pool[(s, k % args.pool)][0], (s, k % args.pool)

    warm = stream_schedule(args.streams, 0.2, args.rate)
    run_schedule(server, warm, frame_of, rate_scale=4.0)
    torch.cuda.synchronize()
    out = {"workload": f"{args.streams} streams x {args.rate:g} fps Poisson, 720x540..1920x1080, "
                       f"8 levels, N=2000", "budget_mib": args.budget_mib,
           "max_batch": args.max_batch, "lanes": args.lanes, "runs": []}
    for scale in (float(x) for x in args.scales.split(",")):
        sched = stream_schedule(args.streams, args.duration, args.rate)
        server.deferred = 0
        res, wall = run_schedule(server, sched, frame_of, rate_scale=scale)
        row = summarize(res, wall, args.streams * args.rate * scale)
        row.update(scale=scale, deferred=server.deferred)
        out["runs"].append(row)
        print(f"# scale {scale:g}: {row}", flush=True)
    out["peak_resident_mib"] = round(server.peak_resident / 2**20, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
