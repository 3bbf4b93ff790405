"""Why no butterfly count can overflow int64 (the boundary accepts at most
2^31 - 1 edges), checked against the oracle's counts.

Section 2.1 defines the butterflies of x as the sum over same-side w != x of
C(c(x, w), 2), with c(x, w) the number of common neighbours.  Since
c(x, w) <= d_x, each term is at most c(x, w) * (d_x - 1) / 2, and the c(x, w)
summed over w are the sum over y in N_x of (d_y - 1).  Hence
    count_x <= (d_x - 1) / 2 * sum_{y in N_x} (d_y - 1),
and summing over one side,
    sum_x count_x <= 1/2 * sum over edges (x, y) of (d_x - 1)(d_y - 1)
                   <  1/2 * sum_x d_x * (sum_{y in N_x} d_y) <= m^2 / 2,
which is below 2^61 for m < 2^31.  Equality holds in the first two steps for
complete bipartite graphs.  These tests check each inequality on graphs the
oracle counts; a zero-butterfly graph with two huge hubs (the case a looser
bound once refused) has bound 0.
"""
from __future__ import annotations

from math import comb

import numpy as np

import oracle
from paper_2010_08695_amd import graphgen as gg


def _per_vertex_bound(g, side):
    du = np.bincount(g.eu, minlength=g.n_u).astype(np.int64)
    dv = np.bincount(g.ev, minlength=g.n_v).astype(np.int64)
    x, y, dx, dy, n = ((g.eu, g.ev, du, dv, g.n_u) if side == 0 else (g.ev, g.eu, dv, du, g.n_v))
    w = np.zeros(n, np.int64)
    np.add.at(w, x, dy[y] - 1)
    return np.maximum(dx - 1, 0) * w // 2, dx, dy, x, y


def _check(g):
    bu, bv, _ = oracle.count(g)
    for side, cnt in ((0, bu), (1, bv)):
        pv, dx, dy, x, y = _per_vertex_bound(g, side)
        assert (cnt <= pv).all(), g.name
        edge_sum = int(((dx[x] - 1) * (dy[y] - 1)).sum())
        assert 2 * int(cnt.sum()) <= edge_sum, g.name
        assert edge_sum < g.m * g.m or g.m == 0, g.name
    return bu, bv


def test_bound_holds_on_random_graphs():
    rng = np.random.default_rng(8)
    for i in range(60):
        g = gg.tiny_random(int(rng.integers(2, 12)), int(rng.integers(2, 10)),
                           float(rng.choice([0.3, 0.6, 0.9])), 700 + i)
        _check(g)
    for seed in range(3):
        _check(gg.chung_lu(400, 120, 3000, 2.2, 2.0, seed=50 + seed))


def test_bound_is_tight_on_complete_bipartite():
    for a in range(2, 8):
        for b in range(2, 8):
            g = gg.complete_bipartite(a, b)
            bu, bv = _check(g)
            assert int(bu.sum()) * 2 == a * b * (a - 1) * (b - 1)
            assert int(bu[0]) == (a - 1) * comb(b, 2)


def test_two_hub_stars_have_zero_bound():
    # a U hub and a V hub of degree k each, no butterfly: every edge has a
    # degree-1 end, so the bound is exactly 0 however large k is
    k = 50_000
    eu = np.concatenate([np.zeros(k, np.int32), np.arange(1, k + 1, dtype=np.int32)])
    ev = np.concatenate([np.arange(1, k + 1, dtype=np.int32), np.zeros(k, np.int32)])
    g = gg.Graph(k + 1, k + 1, eu, ev, "two-stars")
    for side in (0, 1):
        _pv, dx, dy, x, y = _per_vertex_bound(g, side)
        assert int(((dx[x] - 1) * (dy[y] - 1)).sum()) == 0


def test_largest_accepted_edge_count_cannot_overflow():
    m = 2**31 - 1
    assert m * m // 2 < 2**61 < 2**63 - 1
