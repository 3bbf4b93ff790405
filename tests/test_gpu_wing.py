"""GPU parity of the edge-peeling path and of k-tip extraction against the
CPU oracle (oracle/wing_oracle.cpp), bit-exact: per-edge butterfly counts,
wing numbers (level-synchronous edge peeling with the smallest-id rule for
butterflies that lose several edges in one round) and k-tips (Def. 1)."""
from __future__ import annotations

from math import comb

import numpy as np
import pytest

import oracle
from paper_2010_08695_amd import graphgen as gg
from paper_2010_08695_amd import tip

pytestmark = pytest.mark.gpu


def to_input(g, canon_vals):
    """Canonical-order values (edges sorted by (u, v)) at each input edge."""
    cu, cv = oracle.canonical_edges(g)
    key = cu.astype(np.int64) * max(g.n_v, 1) + cv
    idx = np.searchsorted(key, g.eu.astype(np.int64) * max(g.n_v, 1) + g.ev)
    return np.asarray(canon_vals)[idx]


def tiny_graphs(n, seed0, max_u=10, max_v=9):
    rng = np.random.default_rng(seed0)
    for i in range(n):
        yield gg.tiny_random(int(rng.integers(1, max_u + 1)), int(rng.integers(1, max_v + 1)),
                             float(rng.choice([0.2, 0.4, 0.6, 0.8, 1.0])), seed0 * 10000 + i)


def test_edge_counts_tiny_and_closed_forms(gpu_lib):
    for g in tiny_graphs(60, 31):
        c, tot = tip.count_edge_butterflies(g)
        np.testing.assert_array_equal(c, to_input(g, oracle.edge_count(g)), err_msg=g.name)
        assert tot == oracle.count(g)[2]
    for a, b in ((2, 2), (5, 3), (30, 20)):
        c, tot = tip.count_edge_butterflies(gg.complete_bipartite(a, b))
        assert (c == (a - 1) * (b - 1)).all() and tot == comb(a, 2) * comb(b, 2)


def test_edge_counts_medium_and_hubs(gpu_lib):
    """Chung-Lu graphs with hubs past the LDS table (per-workgroup arrays in
    HBM) and a duplicate-laden edge list."""
    for g in (gg.chung_lu(4000, 900, 40000, 2.3, 2.0, seed=91), gg.config_graph("plain-small"),
              gg.chung_lu(20000, 300, 120000, 2.5, 1.8, seed=92)):
        c, tot = tip.count_edge_butterflies(g)
        np.testing.assert_array_equal(c, to_input(g, oracle.edge_count(g)), err_msg=g.name)
        assert tot == oracle.count(g)[2]
    g = gg.tiny_random(12, 9, 0.6, 5)
    rep = gg.Graph(g.n_u, g.n_v, np.concatenate([g.eu, g.eu[::2]]), np.concatenate([g.ev, g.ev[::2]]))
    c, _ = tip.count_edge_butterflies(rep)
    np.testing.assert_array_equal(c, to_input(rep, oracle.edge_count(g)))


def test_wing_tiny_random(gpu_lib):
    for g in tiny_graphs(80, 33):
        np.testing.assert_array_equal(tip.wing_decompose(g), to_input(g, oracle.wing(g)[0]), err_msg=g.name)


def test_wing_closed_forms_and_degenerate(gpu_lib):
    for a, b in ((2, 2), (4, 7), (12, 9)):
        assert (tip.wing_decompose(gg.complete_bipartite(a, b)) == (a - 1) * (b - 1)).all()
    empty = gg.Graph(4, 3, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert tip.wing_decompose(empty).shape == (0,)
    for g in (gg.star(9, "u"), gg.star(5, "v"), gg.random_tree(20, 9, 4)):
        assert not tip.wing_decompose(g).any()
    g = gg.disjoint_union(gg.complete_bipartite(4, 3), gg.complete_bipartite(3, 5), gg.tiny_random(6, 6, 0.7, 2))
    np.testing.assert_array_equal(tip.wing_decompose(g), to_input(g, oracle.wing(g)[0]))


def test_wing_medium(gpu_lib):
    for g in (gg.config_graph("plain-small"), gg.chung_lu(3000, 700, 25000, 2.2, 2.0, seed=94),
              gg.chung_lu(8000, 200, 40000, 2.5, 1.8, seed=95)):
        psi, st = tip.wing_decompose(g, with_stats=True)
        np.testing.assert_array_equal(psi, to_input(g, oracle.wing(g)[0]), err_msg=g.name)
        assert st["rounds"] >= st["fd_levels"] >= 1


@pytest.mark.parametrize("side", [0, 1])
def test_ktips_tiny_random(gpu_lib, side):
    for g in tiny_graphs(40, 35 + side):
        th = oracle.bup(g, side)[0]
        for k in sorted(set(th.tolist()) | {0, 1}):
            np.testing.assert_array_equal(tip.ktips(g, side, th, k), oracle.ktip(g, side, th, k),
                                          err_msg=f"{g.name} k={k}")


@pytest.mark.parametrize("side", [0, 1])
def test_ktips_medium(gpu_lib, side):
    for g in (gg.config_graph("plain-small"), gg.chung_lu(4000, 900, 40000, 2.3, 2.0, seed=96)):
        th = tip.decompose(g, side)
        levels = np.unique(th)
        for k in [0, 1] + levels[np.linspace(0, len(levels) - 1, 6).astype(int)].tolist():
            np.testing.assert_array_equal(tip.ktips(g, side, th, k), oracle.ktip(g, side, th, k),
                                          err_msg=f"{g.name} side {side} k={k}")


def test_ktips_rejects_bad_arguments(gpu_lib):
    g = gg.complete_bipartite(3, 3)
    with pytest.raises(tip.TipError):
        tip.ktips(g, 2, np.zeros(3, np.int64), 1)
    with pytest.raises(tip.TipError):
        tip.ktips(g, 0, np.full(3, -1, np.int64), 1)


def test_wing_cl1m_against_oracle_digest(gpu_lib):
    """cl-1m (957,055 edges): per-edge counts and wing numbers equal the
    digests the oracle's sequential bottom-up edge peeling wrote
    (tests/golden/cl-1m-wing.json), in canonical edge order."""
    import hashlib
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "cl-1m-wing.json")) as f:
        rec = json.load(f)
    g = gg.config_graph("cl-1m")
    assert gg.graph_sha256(g) == rec["graph_sha256"]
    order = np.argsort(g.eu.astype(np.int64) * g.n_v + g.ev, kind="stable")

    def digest(a):
        return hashlib.sha256(np.ascontiguousarray(a[order], dtype="<i8").tobytes()).hexdigest()

    c, tot = tip.count_edge_butterflies(g)
    assert digest(c) == rec["edge_count"]["sha256"] and int(c.sum()) == rec["edge_count"]["sum"]
    psi, st = tip.wing_decompose(g, with_stats=True)
    assert digest(psi) == rec["wing"]["sha256"]
    assert int(psi.max()) == rec["wing"]["max"] and st["fd_levels"] == rec["wing"]["distinct"]
