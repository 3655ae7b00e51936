"""The tuner's search is off unless OF_TUNE_SEARCH=1: an explicit re-search raises
before any GPU work, and a workload missing from the caches takes the device's shipped
tuning (host logic only, no GPU)."""
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


def test_missing_workload_takes_shipped_tuning(no_search):
    with open(tune.SHIPPED) as fh:
        shipped = json.load(fh)
    dev = [v["tuning"] for k, v in shipped.items() if json.loads(k)["dev"] == "gfx950/256"]
    assert dev, "no shipped tuning for gfx950/256"
    got = tune.autotune([np.zeros((480, 640), np.uint8)], _params(), use_cache=True)
    assert got == dev[0]


def test_shipped_workload_found(no_search):
    got = tune.autotune([np.zeros((1080, 1920), np.uint8)], _params(), use_cache=True)
    assert got["mark_words"] == 2 and got["mark_rows"] == 48
