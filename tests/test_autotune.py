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

    r = autotune.tune_graph(g, 0, timer=lambda g, s, t: timer(g, s, t[:2]))
    assert r["tune"][:2] == [512, 4096] and r["ms"] == 1.0
    n1 = len(autotune.STAGES[0]["dense_div"][1]) * len(autotune.STAGES[0]["bitmap_max"][1])
    n2 = len(autotune.STAGES[1]["help_chunk"][1]) * len(autotune.STAGES[1]["help_level_min"][1])
    assert len(r["trials"]) == n1 + n2
    # stage 2 keeps stage 1's winner and varies only the queue parameters
    assert all(t["tune"][:2] == [512, 4096] for t in r["trials"][n1:])
    assert {t["tune"][4] for t in r["trials"][n1:]} == set(autotune.STAGES[1]["help_chunk"][1])


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
    assert autotune.lookup(g, 0, path, table=None) is None
    autotune.store(g, 0, {"tune": [128, 32768], "ms": 2.0}, path)
    assert autotune.lookup(g, 0, path, table=None) == [128, 32768, 0, 0, 0, 0, 0, 0]
    assert autotune.lookup(g, 1, path, table=None) is None            # other side, other class
    assert autotune.size_class(1000, 200, 9000, 0) == autotune.size_class(1100, 190, 9500, 0)


def test_stored_tuning_reaches_tip_opts(tmp_path):
    """A tuning stored for a size class is what tip_decompose_batch receives
    in that graph's tip_opts.tune (per-graph options flag set); graphs of
    other classes get the library defaults (zeros)."""
    from paper_2010_08695_amd import tip
    table = str(tmp_path / "table.json")
    a, b = gg.chung_lu(2000, 400, 15000, 2.2, 2.1, seed=1), gg.complete_bipartite(4, 5)
    autotune.store(a, 0, {"tune": [512, 4096, 0, 0, 32, 128, 0, 0], "ms": 1.0}, table)
    tunes = autotune.batch_tunes([a, b], [0, 0], path=None, table=table)
    assert tunes == [[512, 4096, 0, 0, 32, 128, 0, 0], None]
    opts = tip.batch_opts(2, 150, 0, tunes)
    assert list(opts[0].tune) == [512, 4096, 0, 0, 32, 128, 0, 0] and opts[0].P == 150
    assert list(opts[1].tune) == [0] * 8
    assert all(o.flags & tip.TIP_FLAG_OPTS_PER_GRAPH for o in opts)


def test_package_table_is_well_formed():
    tab = autotune.load_cache(autotune.TABLE)
    for key, rec in tab.items():
        dev, cls = key.split("|")
        assert cls.startswith("side") and len(rec["tune"]) <= 8 and rec["ms"] > 0
        assert all(int(t) >= 0 for t in rec["tune"])


@pytest.mark.gpu
def test_real_tuning_is_exact(gpu_lib, tmp_path):
    g = gg.chung_lu(5000, 1000, 50000, 2.2, 2.0, seed=23)
    stages = [{"dense_div": (0, [16, 256]), "bitmap_max": (1, [1024, 65536])},
              {"help_chunk": (4, [4, 64]), "help_level_min": (5, [1, 256])}]
    r = autotune.tune_graph(g, 0, stages=stages, reps=1)
    assert r["tune"][0] in (16, 256) and r["tune"][1] in (1024, 65536) and r["tune"][4] in (4, 64)
    from paper_2010_08695_amd import tip
    np.testing.assert_array_equal(tip.decompose(g, 0, tune=r["tune"]), oracle.bup(g, 0)[0])
