"""Autotuner: selection, exactness guard and cache, with a fake timer on the
CPU; one real tuning run on the GPU."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2010_08695_amd import autotune
from paper_2010_08695_amd import graphgen as gg


def test_choose_fastest_and_tie_break():
    t = [{"tune": [32, 8192], "ms": 5.0}, {"tune": [64, 8192], "ms": 3.0}, {"tune": [128, 8192], "ms": 3.0}]
    assert autotune.choose(t)["tune"] == [64, 8192]
    with pytest.raises(ValueError):
        autotune.choose([])


def test_tune_graph_with_fake_timer():
    g = gg.complete_bipartite(3, 3)
    theta = np.arange(3)
    cost = {(512, 4096): 1.0}

    def timer(g, side, tune):
        return theta, cost.get(tuple(tune), 10.0 + tune[0] / 1000)

    r = autotune.tune_graph(g, 0, timer=timer)
    assert r["tune"] == [512, 4096] and r["ms"] == 1.0
    assert len(r["trials"]) == len(autotune.DEFAULT_GRID["dense_div"]) * len(autotune.DEFAULT_GRID["bitmap_max"])


def test_tune_graph_rejects_differing_results():
    g = gg.complete_bipartite(3, 3)
    calls = {"n": 0}

    def timer(g, side, tune):
        calls["n"] += 1
        return np.array([calls["n"]]), 1.0

    with pytest.raises(RuntimeError):
        autotune.tune_graph(g, 0, timer=timer)


def test_cache_roundtrip(tmp_path):
    g = gg.complete_bipartite(4, 5)
    path = str(tmp_path / "c.json")
    assert autotune.lookup(g, 0, path) is None
    autotune.store(g, 0, {"tune": [128, 32768], "ms": 2.0}, path)
    assert autotune.lookup(g, 0, path) == [128, 32768]
    assert autotune.lookup(g, 1, path) is None            # other side, other class
    assert autotune.size_class(1000, 200, 9000, 0) == autotune.size_class(1100, 190, 9500, 0)


@pytest.mark.gpu
def test_real_tuning_is_exact(gpu_lib, tmp_path):
    g = gg.chung_lu(5000, 1000, 50000, 2.2, 2.0, seed=23)
    grid = {"dense_div": [16, 256], "bitmap_max": [1024, 65536]}
    r = autotune.tune_graph(g, 0, grid=grid, reps=1)
    assert r["tune"] in ([16, 1024], [16, 65536], [256, 1024], [256, 65536])
    from paper_2010_08695_amd import tip
    np.testing.assert_array_equal(tip.decompose(g, 0, tune=r["tune"]), oracle.bup(g, 0)[0])
