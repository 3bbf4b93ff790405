"""Pins for the oracle's per-edge butterfly counts, wing numbers and k-tips
(oracle/wing_oracle.cpp) against facts fixed by the definitions:
* brute-force 4-tuple enumeration of the butterflies containing each edge;
* brute-force edge-subset max-min wing numbers (the k-wing analogue of Def. 1);
* Def. 1's k-tips read literally (maximal butterfly-connected vertex sets with
  k or more butterflies each) by subset enumeration;
* closed forms: in K_{a,b} every edge lies in (a-1)(b-1) butterflies and that
  is its wing number; trees and stars have none;
* invariants: the edge counts of one vertex sum to twice its butterfly count
  (each butterfly at u uses two edges at u), all edge counts sum to 4B;
  wing numbers never exceed edge counts and are non-decreasing along the
  peel order; disjoint unions decompose independently.
"""
from __future__ import annotations

from math import comb

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2010_08695_amd import graphgen as gg


def _tiny(n, seed0, max_u=7, max_v=6, ps=(0.35, 0.5, 0.7, 0.9)):
    rng = np.random.default_rng(seed0)
    for i in range(n):
        yield gg.tiny_random(int(rng.integers(2, max_u + 1)), int(rng.integers(2, max_v + 1)),
                             float(rng.choice(ps)), seed0 * 1000 + i)


def test_canonical_edges_are_sorted_and_distinct():
    g = gg.tiny_random(9, 7, 0.5, 3)
    rep = gg.Graph(g.n_u, g.n_v, np.concatenate([g.eu, g.eu[::3]]), np.concatenate([g.ev, g.ev[::3]]))
    cu, cv = oracle.canonical_edges(rep)
    bu, bv = brute.canonical(g)
    np.testing.assert_array_equal(cu, bu)
    np.testing.assert_array_equal(cv, bv)


def test_edge_count_matches_enumeration():
    for g in _tiny(120, 5, 9, 8):
        np.testing.assert_array_equal(oracle.edge_count(g), brute.edge_butterflies(g), err_msg=g.name)


def test_edge_counts_sum_to_vertex_counts():
    for seed in range(3):
        g = gg.chung_lu(300, 100, 2000, 2.2, 2.1, seed=60 + seed)
        cu, cv = oracle.canonical_edges(g)
        c = oracle.edge_count(g)
        bu, bv, tot = oracle.count(g)
        su = np.zeros(g.n_u, np.int64)
        np.add.at(su, cu, c)
        sv = np.zeros(g.n_v, np.int64)
        np.add.at(sv, cv, c)
        np.testing.assert_array_equal(su, 2 * bu)
        np.testing.assert_array_equal(sv, 2 * bv)
        assert int(c.sum()) == 4 * tot


def test_wing_matches_subset_brute_force():
    n = 0
    for g in _tiny(300, 7, 6, 5, ps=(0.5, 0.7, 0.9)):
        if brute.canonical(g)[0].shape[0] > 13:
            continue
        n += 1
        psi, order, _ = oracle.wing(g)
        np.testing.assert_array_equal(psi, brute.wing_numbers(g), err_msg=g.name)
    assert n >= 60


def test_wing_closed_forms_and_zero_families():
    for a in range(1, 7):
        for b in range(1, 7):
            g = gg.complete_bipartite(a, b)
            assert (oracle.edge_count(g) == (a - 1) * (b - 1)).all()
            assert (oracle.wing(g)[0] == (a - 1) * (b - 1)).all()
    for g in (gg.star(8, "u"), gg.star(6, "v"), gg.random_tree(10, 7, 2)):
        assert not oracle.edge_count(g).any() and not oracle.wing(g)[0].any()


def test_wing_invariants_medium():
    for seed in range(3):
        g = gg.chung_lu(250, 80, 1800, 2.2, 2.0, seed=70 + seed)
        c = oracle.edge_count(g)
        psi, order, _ = oracle.wing(g)
        assert (psi <= c).all() and ((psi == 0) == (c == 0)).all()
        assert (np.diff(psi[order]) >= 0).all()
        assert np.array_equal(np.sort(order), np.arange(c.shape[0]))


def test_wing_disjoint_union():
    parts = [gg.complete_bipartite(3, 4), gg.tiny_random(6, 5, 0.7, 8), gg.complete_minus_matching(4)]
    g = gg.disjoint_union(*parts)
    psi = oracle.wing(g)[0]
    off = 0
    for p in parts:
        q = oracle.wing(p)[0]
        np.testing.assert_array_equal(psi[off:off + q.shape[0]], q)
        off += q.shape[0]


@pytest.mark.parametrize("side", [0, 1])
def test_ktip_matches_definition(side):
    n = 0
    for g in _tiny(60, 9 + side, 8, 7, ps=(0.4, 0.6, 0.8)):
        th = oracle.bup(g, side)[0]
        for k in sorted(set(th.tolist()) | {0, 1}):
            got = oracle.ktip(g, side, th, k)
            np.testing.assert_array_equal(got, brute.ktips(g, side, k), err_msg=f"{g.name} k={k}")
            n += 1
    assert n > 100


def test_ktip_of_disjoint_bicliques():
    # two bicliques joined by one edge share no butterfly: two separate k-tips
    a, b = gg.complete_bipartite(4, 3), gg.complete_bipartite(3, 5)
    g = gg.disjoint_union(a, b)
    g = gg.Graph(g.n_u, g.n_v, np.append(g.eu, 0), np.append(g.ev, 6))
    th = oracle.bup(g, 0)[0]
    comp = oracle.ktip(g, 0, th, 1)
    assert (comp[:4] == 0).all() and (comp[4:] == 4).all()
    k = 3 * comb(3, 2)  # theta of the K_{4,3} vertices
    comp = oracle.ktip(g, 0, th, k)
    want = np.where(th >= k, np.where(np.arange(g.n_u) < 4, 0, 4), -1)
    np.testing.assert_array_equal(comp, want)
