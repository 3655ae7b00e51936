"""Served form: continuous batching of camera frames on one GPU.

Frames arrive from many camera streams in host memory (pinned), as a capture pipeline
delivers them.  The server keeps a FIFO of arrived frames and a few HIP streams
("lanes").  Whenever a lane is free it admits the oldest waiting frame and, in arrival
order, up to ``max_batch - 1`` more frames of the same size into one batch.  Its device
buffers stay resident between batches: per lane and frame size a pool holds the frame
slots, the keypoint and count buffers, and per batch size (a power of two) a workspace
whose plan stays in it and a HIP graph of the detection call, captured on the pool's
first batch of that size and replayed afterwards.  A batch is one host-to-device copy
per frame into the pool's slots, one graph replay (its planning launch finds the plan in
place and only clears the counters) and one copy of the keypoints back; batches on different lanes overlap on the device.  The pools' bytes count against
``hbm_budget``: a new pool or workspace is allocated only within it, after freeing idle
pools of other sizes (least recently used first) if needed; otherwise the batch waits.
A batch's frames complete when its results are host-visible.  Frames that arrive while
others are on the device join the next batch as soon as a lane and budget free up: that
is the continuous part, there is no fixed batch window.

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
class _Pool:
    """Resident device buffers of one frame size on one lane."""
    shape: tuple
    frames: list                # max_batch device frames (H, W)
    out: object                 # device keypoints, max_batch * N records
    counts: object              # device int32, max_batch
    ws: dict = field(default_factory=dict)       # batch size -> workspace
    graphs: dict = field(default_factory=dict)   # batch size -> captured call
    nbytes: int = 0
    last_use: int = 0


@dataclass
class _Lane:
    stream: object
    out_host: object            # pinned (max_batch * N) keypoints, as uint8 bytes
    counts_host: object         # pinned int32 (max_batch)
    busy: bool = False
    batch: list = field(default_factory=list)
    event: object = None
    pools: dict = field(default_factory=dict)    # frame shape -> _Pool
    pool: object = None         # the pool of the batch in flight


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
        self._uses = 0

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
        """Device bytes of one batch in a pool of its own: frames, workspace (plans,
        bitmaps, slots, levels), keypoints and counts."""
        frames = sum(h * w for (h, w) in shapes)
        out = len(shapes) * self.N * ofhip.KEYPOINT_DTYPE.itemsize + 4 * len(shapes)
        return frames + self._workspace_bytes(shapes) + out

    def _pool_bytes(self) -> int:
        """Keypoints and counts of a pool (frame slots and workspaces come with the
        batch sizes it serves)."""
        return self.max_batch * (self.N * ofhip.KEYPOINT_DTYPE.itemsize + 4)

    def min_bytes(self, shape) -> int:
        """Bytes of a pool that serves single frames of this size."""
        return self._pool_bytes() + self.batch_bytes([shape])

    def _reserve(self, nbytes: int, keep) -> bool:
        """Makes room for nbytes within the budget, freeing idle pools (not `keep`, not
        on a busy lane) least recently used first.  True if it fits."""
        while self.resident + nbytes > self.budget:
            idle = [(pool.last_use, lane, shape) for lane in self.lanes if not lane.busy
                    for shape, pool in lane.pools.items() if pool is not keep]
            if not idle:
                return False
            _, lane, shape = min(idle, key=lambda x: x[0])
            self.resident -= lane.pools.pop(shape).nbytes
        return True

    def _alloc(self, lane: _Lane, pool: _Pool, n: int) -> bool:
        """Gives the pool a workspace for batches of n (and n frame slots) within the
        budget."""
        torch = self.torch
        h, w = pool.shape
        ws = self._workspace_bytes([pool.shape] * n)
        need = ws + max(0, n - len(pool.frames)) * h * w
        if not self._reserve(need, pool):
            return False
        with torch.cuda.stream(lane.stream):
            while len(pool.frames) < n:
                pool.frames.append(torch.empty((h, w), dtype=torch.uint8, device="cuda"))
            pool.ws[n] = torch.empty(ws, dtype=torch.uint8, device="cuda")
        pool.nbytes += need
        self.resident += need
        self.peak_resident = max(self.peak_resident, self.resident)
        return True

    def _fit(self, lane: _Lane, pool: _Pool, want: int) -> int:
        """The largest batch size n <= want (powers of two) that the pool holds a
        workspace for or can get one for within the budget; 0 if none.  When not even a
        single frame fits beside the pool's other workspaces, those are freed (with their
        captured calls and extra frame slots; the lane is idle), which always makes room
        once no other lane holds memory: a single-frame pool is min_bytes."""
        n = want
        while n >= 1:
            if n in pool.ws or self._alloc(lane, pool, n):
                return n
            n //= 2
        if pool.ws or len(pool.frames) > 1:
            h, w = pool.shape
            freed = sum(self._workspace_bytes([pool.shape] * k) for k in pool.ws)
            freed += max(0, len(pool.frames) - 1) * h * w
            pool.ws.clear()
            pool.graphs.clear()
            del pool.frames[1:]
            pool.nbytes -= freed
            self.resident -= freed
            if self._alloc(lane, pool, 1):
                return 1
        return 0

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
            if self.min_bytes(shp) > self.budget:
                done.append(Result(r, np.empty(0, ofhip.KEYPOINT_DTYPE), clock(), 0,
                                   "rejected: one frame exceeds the HBM budget"))
                k += 1
            else:
                keep.append(r)
        queue.extend(keep)
        return k

    def launch(self, queue: collections.deque, clock=None, done: list | None = None) -> bool:
        """Admits the oldest waiting frame and, in arrival order, up to max_batch - 1 more
        of its size into a batch on a free lane, within the HBM budget.  Returns True if
        a batch was launched.  If the detection call fails, the batch's frames complete
        with an "error" result (when ``done`` is given) or go back to the queue."""
        if not queue:
            return False
        lane = next((l for l in self.lanes if not l.busy), None)
        if lane is None:
            return False
        return self._launch_on(lane, queue, clock, done)

    def _launch_on(self, lane: _Lane, queue: collections.deque, clock, done,
                   exact: int = 0) -> bool:
        torch = self.torch
        shape = tuple(queue[0].host.shape)
        pool = lane.pools.get(shape)
        h, w = shape
        if pool is None:
            if self.min_bytes(shape) > self.budget:  # never admissible (see reject_oversized)
                self.deferred += 1
                return False
            need = self._pool_bytes()
            if not self._reserve(need, None):
                self.deferred += 1
                return False
            with torch.cuda.stream(lane.stream):
                pool = _Pool(shape=shape, frames=[],
                             out=torch.empty((self.max_batch * self.N, 32), dtype=torch.uint8,
                                             device="cuda"),
                             counts=torch.zeros(self.max_batch, dtype=torch.int32, device="cuda"),
                             nbytes=need)
            lane.pools[shape] = pool
            self.resident += need
            self.peak_resident = max(self.peak_resident, self.resident)
        # the batch: frames of this size in arrival order, as many as have (or get) room
        picked = [i for i, r in enumerate(queue) if tuple(r.host.shape) == shape]
        picked = picked[:self.max_batch]
        want = 1 << (len(picked).bit_length() - 1)  # batch sizes are powers of two: few graphs
        n = self._fit(lane, pool, exact or want)
        if n == 0 or (exact and n != exact):
            self.deferred += 0 if exact else 1
            return False
        take = set(picked[:n])
        batch = [r for i, r in enumerate(queue) if i in take]
        rest = [r for i, r in enumerate(queue) if i not in take]
        queue.clear()
        queue.extend(rest)
        kp = ofhip.KEYPOINT_DTYPE.itemsize
        try:
            with torch.cuda.stream(lane.stream):
                for f, r in zip(pool.frames, batch):
                    f.copy_(r.host, non_blocking=True)
                g = pool.graphs.get(n)
                if g is None:
                    # first batch of this size: an eager call plans the workspace, then the
                    # call is captured with its plan resident and replayed from now on
                    self._detect(pool, n, lane.stream)
                    g = torch.cuda.CUDAGraph()
                    with torch.cuda.graph(g, stream=lane.stream):
                        self._detect(pool, n, lane.stream)
                    pool.graphs[n] = g
                g.replay()
                lane.out_host[: n * self.N * kp].copy_(pool.out[: n * self.N].view(-1),
                                                       non_blocking=True)
                lane.counts_host[:n].copy_(pool.counts[:n], non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(lane.stream)
        except (ofhip.OfError, RuntimeError) as err:
            self.failed += n
            if done is None:
                queue.extendleft(reversed(batch))
            else:
                t = clock() if clock else 0.0
                for r in batch:
                    done.append(Result(r, np.empty(0, ofhip.KEYPOINT_DTYPE), t, n, f"error: {err}"))
            return False
        self._uses += 1
        pool.last_use = self._uses
        lane.busy, lane.batch, lane.event, lane.pool = True, batch, ev, pool
        self.batches += 1
        return True

    def warm(self, shapes) -> int:
        """Allocates the pools of these frame sizes on every lane and captures their
        calls for every batch size (powers of two up to max_batch), within the budget,
        so that no capture (it synchronises the device) falls in a measured run.
        Returns the number of calls captured."""
        torch = self.torch
        k = 0
        for lane in self.lanes:
            for shape in shapes:
                n = 1
                while n <= self.max_batch:
                    dummy = collections.deque(
                        Request(-1, i, 0.0, torch.zeros(shape, dtype=torch.uint8))
                        for i in range(n))
                    if not self._launch_on(lane, dummy, None, None, exact=n):
                        break
                    lane.event.synchronize()
                    lane.busy, lane.batch, lane.event, lane.pool = False, [], None, None
                    k += 1
                    n *= 2
        self.batches = 0
        return k

    def _detect(self, pool: _Pool, n: int, stream) -> None:
        # The call keeps its planning launch: it re-plans only when the workspace does not
        # hold this call's plan, so a workspace whose memory was reused is planned again
        # while an unchanged one costs the launch alone.
        ws = pool.ws[n]
        ofhip.of_detect_batch([ofhip.image_of(f) for f in pool.frames[:n]], self.p,
                              ws.data_ptr(), ws.numel(), pool.out.data_ptr(),
                              [i * self.N for i in range(n)], self.N, pool.counts.data_ptr(),
                              self.tune, stream.cuda_stream)

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
                lane.busy, lane.batch, lane.event, lane.pool = False, [], None, None
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

    server.warm(sorted({tuple(v[0].shape) for v in pool.values()}))
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
