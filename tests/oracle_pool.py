"""Run the CPU oracle on many synthetic frames in worker processes (test helper).

Workers are spawned (never forked from a process that may hold GPU state) and rebuild
each frame from its FrameSpec, so only small specs cross process boundaries."""
import multiprocessing as mp
import os

import oracle
from synth import make_frame


def _one(args):
    spec, kw = args
    return oracle.detect(make_frame(spec), oracle.params(**kw))


def detect_many(specs, kw, workers=None):
    if len(specs) == 1:
        return [_one((specs[0], kw))]
    workers = workers or min(len(specs), max(1, min(16, os.cpu_count() or 1)))
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        return pool.map(_one, [(s, kw) for s in specs])
