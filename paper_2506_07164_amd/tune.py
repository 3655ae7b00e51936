"""Autotuner for the batched path: tile shapes and persistent grid sizes.

For a batch shape (frame sizes + detector parameters) it times candidate launch shapes
of of_detect_batch on the device (with the plan resident in the workspace, as a detector
that owns its workspace runs) and keeps the fastest.  The search is coordinate
descent over (segment-test tile, Harris/NMS tile, grids) from the library defaults;
every candidate is timed with HIP events over a few calls after a warm-up.  Results are
cached in a JSON file keyed by GPU name, frame sizes and parameters.  Outputs do not
depend on the tuning (the parity tests check that), so tuning only moves time.
"""
from __future__ import annotations

import json
import os

from . import ofhip

CACHE = os.environ.get("OF_TUNE_CACHE", os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                      "tune_cache.json"))
# Results of this tuner shipped with the library for known devices and workloads,
# consulted after the local cache.
SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")

FIELDS = ("mark_words", "mark_rows", "det_cells_x", "det_cells_y", "det_w", "det_h",
          "mark_grid", "det_grid", "pyr_pass", "mark_order", "det_order")

# Searching is off unless OF_TUNE_SEARCH=1: a search (many launch shapes timed one after
# another on one resident workspace) has faulted the device once and the cause is not
# yet found.  Without it, a workload missing from the caches takes the library default
# for its frames and parameters (sweeps of the shipped workloads found the default
# within 10% of the best shape, and another workload's shape is no better a guess).
SEARCH = os.environ.get("OF_TUNE_SEARCH") == "1"


class SearchDisabled(RuntimeError):
    pass


def _key(shapes, p, device_name):
    return json.dumps({"dev": device_name, "shapes": [list(s) for s in shapes],
                       "params": [getattr(p, f) for f, _ in ofhip.OfParams._fields_]},
                      sort_keys=True)


def _as_tuning(d):
    return ofhip.tuning(**{k: int(v) for k, v in d.items()})


def time_tuning(det, frames, tune, calls=20, warmup=3):
    """Mean milliseconds per of_detect_batch call (HIP events on the current stream)."""
    import torch
    for _ in range(warmup):
        det.detect_batch(frames, tune=tune)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(calls):
        det.detect_batch(frames, tune=tune)
    e.record()
    e.synchronize()
    return s.elapsed_time(e) / calls


def candidates(p, n_cus):
    marks = [dict(mark_words=w, mark_rows=r) for w in (1, 2, 4)
             for r in (8, 16, 24, 32, 40, 48, 56, 64) if 16 <= w * r <= 128]
    if p.cell > 0:
        dets = [dict(det_cells_x=cx, det_cells_y=cy) for cx, cy in
                ((1, 1), (2, 1), (4, 1), (2, 2), (8, 1), (4, 2))
                if cx * p.cell <= 256 and cy * p.cell <= 128]
    else:
        dets = [dict(det_w=w, det_h=h) for w, h in ((64, 32), (128, 32), (128, 64), (256, 32))]
    grids = [dict(mark_grid=0, det_grid=0, pyr_pass=0, mark_order=0, det_order=0),
             dict(mark_grid=0, det_grid=0, pyr_pass=0, mark_order=1, det_order=0),
             dict(mark_grid=0, det_grid=0, pyr_pass=0, mark_order=1, det_order=1),
             dict(mark_grid=0, det_grid=0, pyr_pass=1, mark_order=1, det_order=1)]
    grids += [dict(mark_grid=m * n_cus, det_grid=d * n_cus) for m, d in ((2, 2), (4, 3))]
    return marks, dets, grids


def _descriptors(shapes):
    """Frame descriptors of these (H, W) shapes for the host-only calls (no pixels)."""
    return [ofhip.OfImage(None, w, h, w) for h, w in shapes]


def device_key():
    """Architecture and compute-unit count of device 0, e.g. 'gfx950/256'."""
    import torch
    prop = torch.cuda.get_device_properties(0)
    return f"{prop.gcnArchName.split(':')[0]}/{prop.multi_processor_count}"


def autotune(frames, p, calls=20, use_cache=True, verbose=False):
    """Best tuning (as a dict of of_tuning fields) for these frames and parameters:
    from the local cache, else from the shipped results, else searched when SEARCH is on
    (else the library default for these frames).  The result of a search is written to
    the local cache (also when use_cache is False)."""
    import torch
    name = device_key()
    shapes = [tuple(f.shape) for f in frames]
    key = _key(shapes, p, name)
    cache = {}
    if use_cache:
        for path in (CACHE, SHIPPED):
            try:
                with open(path) as fh:
                    found = json.load(fh)
            except (OSError, ValueError):
                continue
            if path == CACHE:
                cache = found
            if key in found:
                return found[key]["tuning"]
    if not SEARCH:
        if not use_cache:
            raise SearchDisabled("tuner search is off (set OF_TUNE_SEARCH=1 to search)")
        default = ofhip.of_tuning_default(_descriptors(shapes), p)
        return {f: getattr(default, f) for f in FIELDS}
    n_cus = torch.cuda.get_device_properties(0).multi_processor_count
    det = ofhip.Detector(shapes, p, resident=True)  # timed as bench.py runs it: plan resident
    best = {}
    default = ofhip.of_tuning_default(_descriptors(shapes), p)
    for f in FIELDS:
        best[f] = getattr(default, f)
    marks, dets, grids = candidates(p, n_cus)
    log = []

    def trial(upd):
        cand = dict(best, **upd)
        try:
            ms = time_tuning(det, frames, _as_tuning(cand), calls)
        except ofhip.OfError:
            return None
        log.append((cand, ms))
        if verbose:
            print(f"  {cand} -> {ms * 1e3:.1f} us", flush=True)
        return ms

    best_ms = trial({})
    for group in (grids, marks, dets, grids):
        for upd in group:
            ms = trial(upd)
            if ms is not None and ms < best_ms:
                best_ms = ms
                best.update(upd)
    result = {"tuning": best, "ms": best_ms, "trials": len(log)}
    if not use_cache:
        try:
            with open(CACHE) as fh:
                cache = json.load(fh)
        except (OSError, ValueError):
            cache = {}
    cache[key] = result
    tmp = CACHE + ".tmp%d" % os.getpid()
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1)
    os.replace(tmp, CACHE)
    return best
