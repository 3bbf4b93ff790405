"""Pins for the CPU oracle against facts fixed by the paper and mathematics.

The oracle (oracle/tip_oracle.cpp) is checked against:
* brute-force 4-tuple butterfly enumeration (Section 2.1 definition);
* brute-force subset max-min tip numbers (Def. 1);
* closed forms for K_{a,b} and K_{n,n} minus a perfect matching;
* zero-butterfly families (stars, trees) and disjoint unions;
* invariants: per-side sums = 2B, pair bound, certificate, level property,
  non-decreasing theta along the peel order, relabelling invariance,
  the wedge total of bottom-up peeling.
"""
from __future__ import annotations

import json
import os
from math import comb

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2010_08695_amd import graphgen as gg

import _props

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _tiny_cases(n_cases, max_u, max_v, seed0):
    rng = np.random.default_rng(seed0)
    for i in range(n_cases):
        nu = int(rng.integers(2, max_u + 1))
        nv = int(rng.integers(2, max_v + 1))
        p = float(rng.choice([0.25, 0.4, 0.55, 0.7, 0.85]))
        yield gg.tiny_random(nu, nv, p, seed0 * 1000 + i)


def test_count_matches_4tuple_enumeration():
    for g in _tiny_cases(150, 9, 8, 11):
        bu, bv, tot = oracle.count(g)
        eu_, ev_, et = brute.butterflies(g)
        assert tot == et, g.name
        np.testing.assert_array_equal(bu, eu_, err_msg=g.name)
        np.testing.assert_array_equal(bv, ev_, err_msg=g.name)


@pytest.mark.parametrize("side", [0, 1])
def test_bup_matches_subset_brute_force(side):
    for g in _tiny_cases(80, 9, 9, 21 + side):
        th, order, _ = oracle.bup(g, side)
        np.testing.assert_array_equal(th, brute.tip_numbers(g, side), err_msg=g.name)


@pytest.mark.parametrize("side", [0, 1])
def test_support_levels_matches_pair_brute_force(side):
    """f_x(S) for the three theta-defined sets against the butterflies each
    pair {x, w} shares, found by enumerating column pairs (Section 2.1);
    theta here is an arbitrary labelling with ties, not tip numbers."""
    rng = np.random.default_rng(17 + side)
    for g in _tiny_cases(40, 9, 8, 31 + side):
        a = brute.dense(g) if side == 0 else brute.dense(g).T
        pair = brute._pair_butterflies(a)
        n = a.shape[0]
        theta = rng.integers(0, 4, n)
        q = np.arange(n, dtype=np.int32)
        got = oracle.support_levels(g, side, theta, q)
        for x in range(n):
            want = (pair[x].sum(), pair[x][theta >= theta[x]].sum(), pair[x][theta > theta[x]].sum())
            assert tuple(got[x]) == want, (g.name, x, got[x], want)


def test_bup_matches_brute_force_on_denser_tiny_graphs():
    # 12-vertex sides with a biclique planted inside a sparse background, so
    # several distinct tip levels appear
    rng = np.random.default_rng(5)
    for i in range(12):
        g = gg.tiny_random(12, 7, 0.3, 500 + i)
        a = brute.dense(g)
        rows = rng.choice(12, size=5, replace=False)
        cols = rng.choice(7, size=4, replace=False)
        a[np.ix_(rows, cols)] = 1
        u, v = np.nonzero(a)
        g2 = gg.Graph(12, 7, u.astype(np.int32), v.astype(np.int32), f"planted-{i}")
        for side in (0, 1):
            th, _, _ = oracle.bup(g2, side)
            np.testing.assert_array_equal(th, brute.tip_numbers(g2, side), err_msg=g2.name)


def test_complete_bipartite_closed_form():
    for a in range(1, 9):
        for b in range(1, 9):
            g = gg.complete_bipartite(a, b)
            bu, bv, tot = oracle.count(g)
            assert tot == comb(a, 2) * comb(b, 2)
            assert (bu == (a - 1) * comb(b, 2)).all()
            assert (bv == (b - 1) * comb(a, 2)).all()
            assert (oracle.bup(g, 0)[0] == (a - 1) * comb(b, 2)).all()
            assert (oracle.bup(g, 1)[0] == (b - 1) * comb(a, 2)).all()


def test_k30_20_golden_fixture():
    with open(os.path.join(GOLDEN, "k30_20.json")) as f:
        fx = json.load(f)
    g = gg.complete_bipartite(fx["a"], fx["b"])
    bu, bv, tot = oracle.count(g)
    assert tot == fx["total"]
    assert (bu == fx["bfly_u"]).all() and (bv == fx["bfly_v"]).all()
    assert (oracle.bup(g, 0)[0] == fx["theta_u"]).all()
    assert (oracle.bup(g, 1)[0] == fx["theta_v"]).all()


def test_complete_minus_matching_closed_form():
    # u and w (u != w) share the n-2 columns other than u's and w's own, so
    # every vertex has (n-1) * C(n-2, 2) butterflies; the graph is
    # vertex-transitive, so the tip number is the same value.
    for n in range(2, 10):
        g = gg.complete_minus_matching(n)
        bu, bv, tot = oracle.count(g)
        want = (n - 1) * comb(n - 2, 2)
        assert (bu == want).all() and (bv == want).all()
        assert (oracle.bup(g, 0)[0] == want).all()
        assert (oracle.bup(g, 1)[0] == want).all()


def test_zero_butterfly_families():
    for g in [gg.star(7, "u"), gg.star(7, "v"), gg.random_tree(9, 6, 1),
              gg.random_tree(15, 4, 2), gg.random_tree(3, 12, 3)]:
        bu, bv, tot = oracle.count(g)
        assert tot == 0 and not bu.any() and not bv.any()
        assert not oracle.bup(g, 0)[0].any() and not oracle.bup(g, 1)[0].any()


def test_empty_and_isolated():
    g = gg.Graph(5, 3, np.zeros(0, np.int32), np.zeros(0, np.int32))
    bu, bv, tot = oracle.count(g)
    assert tot == 0 and bu.shape == (5,) and bv.shape == (3,)
    assert (oracle.bup(g, 0)[0] == 0).all()
    g = gg.Graph(0, 0, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert oracle.bup(g, 0)[0].shape == (0,)


def test_disjoint_union_is_independent():
    parts = [gg.complete_bipartite(4, 3), gg.tiny_random(7, 6, 0.6, 3),
             gg.complete_minus_matching(5), gg.tiny_random(6, 5, 0.7, 4)]
    g = gg.disjoint_union(*parts)
    bu, bv, tot = oracle.count(g)
    th_u = oracle.bup(g, 0)[0]
    th_v = oracle.bup(g, 1)[0]
    ou = ov = 0
    t_sum = 0
    for p in parts:
        pu, pv, pt = oracle.count(p)
        t_sum += pt
        np.testing.assert_array_equal(bu[ou:ou + p.n_u], pu)
        np.testing.assert_array_equal(bv[ov:ov + p.n_v], pv)
        np.testing.assert_array_equal(th_u[ou:ou + p.n_u], oracle.bup(p, 0)[0])
        np.testing.assert_array_equal(th_v[ov:ov + p.n_v], oracle.bup(p, 1)[0])
        ou += p.n_u
        ov += p.n_v
    assert tot == t_sum


def test_duplicate_edges_merged():
    g = gg.tiny_random(8, 6, 0.5, 9)
    rep = gg.Graph(g.n_u, g.n_v, np.concatenate([g.eu, g.eu[::2]]),
                   np.concatenate([g.ev, g.ev[::2]]))
    for a, b in zip(oracle.count(g)[:2], oracle.count(rep)[:2]):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(oracle.bup(g, 0)[0], oracle.bup(rep, 0)[0])


def test_invalid_input_rejected():
    g = gg.Graph(3, 3, np.array([0, 3], np.int32), np.array([0, 1], np.int32))
    with pytest.raises(ValueError):
        oracle.count(g)
    with pytest.raises(ValueError):
        oracle.bup(gg.complete_bipartite(2, 2), 2)


@pytest.mark.parametrize("name", ["plain-small"])
def test_invariants_plain_small(name):
    g = gg.config_graph(name)
    bu, bv, tot = oracle.count(g)
    _props.check_count_sums(bu, bv, tot)
    for side, cnt in ((0, bu), (1, bv)):
        th, order, wedges = oracle.bup(g, side)
        _props.check_bounds(g, side, th, cnt)
        _props.check_certificate(g, side, th, np.arange(th.shape[0]))
        _props.check_levels(g, side, th)
        # tip numbers are assigned in non-decreasing order along the peel
        assert (np.diff(th[order]) >= 0).all()
        # bottom-up peeling visits every (u, v, u') with u' != u once:
        # sum over the other side of d(d-1)
        d_other = np.bincount(g.ev if side == 0 else g.eu,
                              minlength=g.n_v if side == 0 else g.n_u).astype(np.int64)
        assert wedges == int((d_other * (d_other - 1)).sum())


def test_invariants_random_medium():
    for seed in range(4):
        g = gg.chung_lu(300, 120, 2500, 2.3, 2.1, seed=40 + seed)
        bu, bv, tot = oracle.count(g)
        _props.check_count_sums(bu, bv, tot)
        for side, cnt in ((0, bu), (1, bv)):
            th, order, _ = oracle.bup(g, side)
            _props.check_bounds(g, side, th, cnt)
            _props.check_certificate(g, side, th, np.arange(th.shape[0]))
            _props.check_levels(g, side, th)
            assert (np.diff(th[order]) >= 0).all()


def test_relabel_invariance():
    g = gg.chung_lu(200, 90, 1500, 2.2, 2.2, seed=77)
    gp, pu, pv = gg.permute_ids(g, 5)
    th = oracle.bup(g, 0)[0]
    thp = oracle.bup(gp, 0)[0]
    np.testing.assert_array_equal(thp[pu], th)
    th = oracle.bup(g, 1)[0]
    thp = oracle.bup(gp, 1)[0]
    np.testing.assert_array_equal(thp[pv], th)


def test_side_swap_is_transpose():
    g = gg.chung_lu(150, 60, 900, 2.2, 2.4, seed=8)
    gt = gg.transpose(g)
    np.testing.assert_array_equal(oracle.bup(g, 1)[0], oracle.bup(gt, 0)[0])


def test_two_core_pruning_keeps_theta():
    # vertices outside the 2-core lie on no 4-cycle: removing them (and
    # iterating) leaves every tip number unchanged and they have theta 0
    g = gg.chung_lu(400, 150, 2000, 2.3, 2.1, seed=91)
    th = oracle.bup(g, 0)[0]
    eu, ev = g.eu.astype(np.int64), g.ev.astype(np.int64)
    keep = np.ones(eu.shape[0], bool)
    while True:
        du = np.bincount(eu[keep], minlength=g.n_u)
        dv = np.bincount(ev[keep], minlength=g.n_v)
        drop = keep & ((du[eu] < 2) | (dv[ev] < 2))
        if not drop.any():
            break
        keep &= ~drop
    g2 = gg.Graph(g.n_u, g.n_v, g.eu[keep], g.ev[keep])
    th2 = oracle.bup(g2, 0)[0]
    np.testing.assert_array_equal(th, th2)
    du = np.bincount(eu[keep], minlength=g.n_u)
    assert (th[du == 0] == 0).all()


def test_plain_small_golden_matches_oracle():
    with open(os.path.join(GOLDEN, "plain-small.json")) as f:
        rec = json.load(f)
    g = gg.config_graph("plain-small")
    assert gg.graph_sha256(g) == rec["graph_sha256"]
    np.testing.assert_array_equal(oracle.bup(g, 0)[0], np.array(rec["theta_u"]["values"]))
