"""The tuner's search is off unless OF_TUNE_SEARCH=1: an explicit re-search raises
before any GPU work, a shipped workload takes its shipped shape and a workload missing
from the caches takes the library default (host logic only, no GPU)."""
import json

import numpy as np
import pytest

from paper_2506_07164_amd import ofhip, tune


@pytest.fixture
def no_search(monkeypatch, tmp_path):
    monkeypatch.setattr(tune, "SEARCH", False)
    monkeypatch.setattr(tune, "CACHE", str(tmp_path / "cache.json"))
    monkeypatch.setattr(tune, "device_key", lambda: "gfx950/256")


def _params():
    return ofhip.params(n_levels=8, fast_t=20, fast_t_min=7, cell=30, n_features=2000)


def test_retune_raises_without_search(no_search):
    with pytest.raises(tune.SearchDisabled):
        tune.autotune([np.zeros((1080, 1920), np.uint8)], _params(), use_cache=False)


def test_missing_workload_takes_library_default(no_search):
    shapes = [(480, 640)]
    got = tune.autotune([np.zeros(sh, np.uint8) for sh in shapes], _params(), use_cache=True)
    d = ofhip.of_tuning_default([ofhip.OfImage(None, w, h, w) for h, w in shapes], _params())
    assert got == {f: getattr(d, f) for f in tune.FIELDS}


def test_shipped_workload_found(no_search):
    got = tune.autotune([np.zeros((1080, 1920), np.uint8)], _params(), use_cache=True)
    assert got["mark_words"] == 2 and got["mark_rows"] == 48


@pytest.mark.parametrize("name", ["c1", "c3", "c4"])
def test_shipped_config_workloads_found(no_search, name):
    """The benchmark's other workloads have shipped shapes of their own, with the sweep's
    per-call time recorded beside them."""
    from synth import CONFIGS
    cfg = CONFIGS[name]
    p = ofhip.params(**cfg["params"])
    shapes = [(s.height, s.width) for s in cfg["frames"]]
    with open(tune.SHIPPED) as fh:
        entry = json.load(fh)[tune._key(shapes, p, "gfx950/256")]
    assert entry["ms"] > 0 and entry["trials"] > 1
    got = tune.autotune([np.zeros(sh, np.uint8) for sh in shapes], p, use_cache=True)
    assert got == entry["tuning"]
