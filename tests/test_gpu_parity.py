"""GPU parity: libtip (HIP, gfx950) against the CPU oracle, bit-exact.

Counts and tip numbers are exact int64, so every comparison is equality.
Small graphs are compared element by element with the oracle run in the
test; the larger workloads are compared with SHA-256 digests the committed
golden script wrote from the oracle, plus sampled entries and invariants.
"""
from __future__ import annotations

import hashlib
import json
import os
from math import comb

import numpy as np
import pytest

import oracle
from paper_2010_08695_amd import graphgen as gg
from paper_2010_08695_amd import tip

import _props

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i8").tobytes()).hexdigest()


def tiny_graphs(n, seed0, max_u=12, max_v=10):
    rng = np.random.default_rng(seed0)
    for i in range(n):
        nu = int(rng.integers(1, max_u + 1))
        nv = int(rng.integers(1, max_v + 1))
        p = float(rng.choice([0.2, 0.4, 0.6, 0.8, 1.0]))
        yield gg.tiny_random(nu, nv, p, seed0 * 10000 + i)


def test_count_k30_20(gpu_lib):
    bu, bv, tot = tip.count_butterflies(gg.complete_bipartite(30, 20))
    assert tot == 82650 and (bu == 5510).all() and (bv == 8265).all()


def test_count_tiny_random(gpu_lib):
    for g in tiny_graphs(60, 3):
        bu, bv, tot = tip.count_butterflies(g)
        ou, ov, ot = oracle.count(g)
        assert tot == ot, g.name
        np.testing.assert_array_equal(bu, ou, err_msg=g.name)
        np.testing.assert_array_equal(bv, ov, err_msg=g.name)


def test_count_plain_small(gpu_lib):
    g = gg.config_graph("plain-small")
    bu, bv, tot = tip.count_butterflies(g)
    ou, ov, ot = oracle.count(g)
    assert tot == ot
    np.testing.assert_array_equal(bu, ou)
    np.testing.assert_array_equal(bv, ov)


def test_count_chung_lu_medium(gpu_lib):
    for seed in range(3):
        g = gg.chung_lu(3000, 800, 30000, 2.2, 2.0, seed=60 + seed)
        bu, bv, tot = tip.count_butterflies(g)
        ou, ov, ot = oracle.count(g)
        assert tot == ot
        np.testing.assert_array_equal(bu, ou)
        np.testing.assert_array_equal(bv, ov)


@pytest.mark.parametrize("side", [0, 1])
def test_decompose_tiny_random(gpu_lib, side):
    for g in tiny_graphs(40, 7 + side):
        th = tip.decompose(g, side)
        np.testing.assert_array_equal(th, oracle.bup(g, side)[0], err_msg=g.name)


def test_decompose_closed_forms(gpu_lib):
    for a, b in ((30, 20), (5, 7), (1, 9), (9, 1), (2, 2)):
        g = gg.complete_bipartite(a, b)
        assert (tip.decompose(g, 0) == (a - 1) * comb(b, 2)).all()
        assert (tip.decompose(g, 1) == (b - 1) * comb(a, 2)).all()
    for n in (3, 6, 11):
        g = gg.complete_minus_matching(n)
        assert (tip.decompose(g, 0) == (n - 1) * comb(n - 2, 2)).all()


def test_decompose_degenerate(gpu_lib):
    empty = gg.Graph(4, 3, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert (tip.decompose(empty, 0) == 0).all() and tip.decompose(empty, 0).shape == (4,)
    none = gg.Graph(0, 0, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert tip.decompose(none, 0).shape == (0,)
    for g in (gg.star(9, "u"), gg.random_tree(20, 9, 4)):
        assert not tip.decompose(g, 0).any() and not tip.decompose(g, 1).any()
    # duplicates merged
    g = gg.tiny_random(10, 8, 0.6, 3)
    rep = gg.Graph(g.n_u, g.n_v, np.concatenate([g.eu, g.eu]), np.concatenate([g.ev, g.ev]))
    np.testing.assert_array_equal(tip.decompose(rep, 0), oracle.bup(g, 0)[0])


@pytest.mark.parametrize("side", [0, 1])
def test_decompose_plain_small(gpu_lib, side):
    g = gg.config_graph("plain-small")
    th = tip.decompose(g, side)
    np.testing.assert_array_equal(th, oracle.bup(g, side)[0])


def test_decompose_chung_lu_medium(gpu_lib):
    for seed in range(3):
        g = gg.chung_lu(4000, 900, 40000, 2.3, 2.0, seed=80 + seed)
        for side in (0, 1):
            np.testing.assert_array_equal(tip.decompose(g, side), oracle.bup(g, side)[0])


@pytest.mark.parametrize("n_side", [8_500_000, 17_000_000])
def test_side_above_eight_million_keys(gpu_lib, n_side):
    """Sides of more than 2^23 keys make the list tiles 32K keys wide, so that
    one tile of 16-bit counters fills a dense workgroup's LDS; above 2^24 keys
    the tile-bound table has more than 512 tiles per list.  K_{300,3000}
    (theta = 299 * C(3000, 2) for every U vertex, closed form; degree 3000
    takes 16-bit counters) beside a Chung-Lu part checked by the oracle on its
    own, padded with isolated U vertices."""
    k = gg.complete_bipartite(300, 3000)
    r = gg.chung_lu(3000, 800, 30000, 2.2, 2.0, seed=91)
    n_pad = n_side - k.n_u - r.n_u
    pad = gg.Graph(n_pad, 1, np.zeros(0, np.int32), np.zeros(0, np.int32), "pad")
    g = gg.disjoint_union(k, r, pad)
    th = tip.decompose(g, 0)
    assert len(th) == n_side
    assert (th[:300] == 299 * comb(3000, 2)).all()
    np.testing.assert_array_equal(th[300:300 + r.n_u], oracle.bup(r, 0)[0])
    assert not th[300 + r.n_u:].any()


@pytest.mark.parametrize("P", [1, 2, 7, 150, 2001])
def test_decompose_any_P(gpu_lib, P):
    g = gg.chung_lu(2000, 500, 15000, 2.2, 2.1, seed=5)
    np.testing.assert_array_equal(tip.decompose(g, 0, P=P), oracle.bup(g, 0)[0])


def test_relabel_and_side_swap(gpu_lib):
    g = gg.chung_lu(1500, 400, 12000, 2.2, 2.1, seed=6)
    gp, pu, pv = gg.permute_ids(g, 9)
    th = tip.decompose(g, 0)
    np.testing.assert_array_equal(tip.decompose(gp, 0)[pu], th)
    np.testing.assert_array_equal(tip.decompose(gg.transpose(g), 1), th)


def test_cd_state_theorem1(gpu_lib):
    """Each vertex's tip number lies in its subset's range (Theorem 1), and
    its initial support equals its butterflies with the vertices of its own
    and all later subsets."""
    g = gg.chung_lu(2500, 600, 20000, 2.2, 2.1, seed=11)
    r = tip.decompose_ex(g, 0, P=20)
    th = oracle.bup(g, 0)[0]
    np.testing.assert_array_equal(r["theta"], th)
    b = r["bounds"]
    sub = r["subset"]
    assert r["n_subsets"] >= 1 and (np.diff(b) > 0).all()
    assert ((b[sub] <= th) & (th < b[sub + 1])).all()
    for i in range(r["n_subsets"]):
        member = (sub >= i).astype(np.uint8)
        q = np.nonzero(sub == i)[0].astype(np.int32)
        if q.size:
            np.testing.assert_array_equal(oracle.support_in(g, 0, member, q), r["init"][q])


def test_repeatable(gpu_lib):
    g = gg.chung_lu(3000, 700, 25000, 2.2, 2.1, seed=13)
    a, sa = tip.decompose(g, 0, with_stats=True)
    b, sb = tip.decompose(g, 0, with_stats=True)
    np.testing.assert_array_equal(a, b)
    for k in ("wedges_count", "wedges_cd", "wedges_fd", "pair_updates", "rounds", "subsets"):
        assert sa[k] == sb[k], k


@pytest.mark.parametrize("P", [3, 150])
def test_graph_rounds_match_eager(gpu_lib, P):
    """Coarse-grained rounds replayed from a captured HIP graph (several
    rounds per replay) give the same tip numbers, subsets and work as rounds
    launched one by one from the host."""
    g = gg.chung_lu(6000, 1200, 60000, 2.2, 2.0, seed=19)
    th = oracle.bup(g, 0)[0]
    runs = [tip.decompose(g, 0, P=P, with_stats=True, flags=f)
            for f in (0, tip.TIP_FLAG_NO_GRAPH, tip.TIP_FLAG_TIME_KERNELS)]
    for t, st in runs:
        np.testing.assert_array_equal(t, th)
        assert st["rounds"] > 0
    for k in ("wedges_cd", "wedges_fd", "pair_updates", "rounds", "subsets", "skipped"):
        assert runs[0][1][k] == runs[1][1][k] == runs[2][1][k], k
    ex_graph = tip.decompose_ex(g, 0, P=P)
    ex_eager = tip.decompose_ex(g, 0, P=P, flags=tip.TIP_FLAG_NO_GRAPH)
    np.testing.assert_array_equal(ex_graph["subset"], ex_eager["subset"])
    np.testing.assert_array_equal(ex_graph["bounds"], ex_eager["bounds"])


@pytest.mark.parametrize("permille", [0, 1, 500])
def test_list_compaction_changes_nothing_but_work(gpu_lib, permille):
    """Removing peeled vertices from the traversed lists (DGM) leaves the tip
    numbers, the range partition and the per-range supports unchanged and
    only lowers the coarse-grained wedge count; permille 1 compacts at
    almost every range start."""
    g = gg.chung_lu(8000, 1500, 90000, 2.2, 2.0, seed=29)
    th = oracle.bup(g, 0)[0]
    tune = [0, 0, permille]
    ref = tip.decompose_ex(g, 0, flags=tip.TIP_FLAG_NO_COMPACT)
    got = tip.decompose_ex(g, 0, tune=tune)
    np.testing.assert_array_equal(ref["theta"], th)
    np.testing.assert_array_equal(got["theta"], th)
    np.testing.assert_array_equal(got["subset"], ref["subset"])
    np.testing.assert_array_equal(got["init"], ref["init"])
    np.testing.assert_array_equal(got["bounds"], ref["bounds"])
    _, s0 = tip.decompose(g, 0, with_stats=True, flags=tip.TIP_FLAG_NO_COMPACT)
    _, s1 = tip.decompose(g, 0, with_stats=True, tune=tune)
    assert s1["wedges_cd"] < s0["wedges_cd"]
    # decrements of peeled vertices drop with their list entries
    assert s1["pair_updates"] <= s0["pair_updates"] and s1["rounds"] == s0["rounds"]
    for side in (0, 1):
        np.testing.assert_array_equal(tip.decompose(g, side, tune=tune, flags=tip.TIP_FLAG_NO_GRAPH),
                                      oracle.bup(g, side)[0])


def test_batch_matches_single(gpu_lib):
    gs = [gg.chung_lu(800 + 100 * k, 300, 5000 + 500 * k, 2.2, 2.3, seed=200 + k) for k in range(5)]
    sides = [0, 1, 0, 1, 0]
    out = tip.decompose_batch(gs, sides)
    for g, s, th in zip(gs, sides, out):
        np.testing.assert_array_equal(th, oracle.bup(g, s)[0])


def test_batch_forms_agree(gpu_lib):
    """The batched forms (the batch as one disjoint union; the graphs on
    concurrent streams with one fine-grained launch over all graphs' subsets)
    and the plain one-after-another form give the oracle's tip numbers; the
    streams form reports the same per-graph work as the plain one, and the
    union's totals (in entry 0) cover every graph's count wedges."""
    params = gg.batch_params(12, seed_base=3000, m_lo=2e3, m_hi=4e4)
    gs = [gg.batch_graph(p) for p in params]
    sides = [k % 2 for k in range(len(gs))]
    tu, su = tip.decompose_batch(gs, sides, with_stats=True)
    ts, ss = tip.decompose_batch(gs, sides, with_stats=True, flags=tip.TIP_FLAG_BATCH_STREAMS)
    tp, sp = tip.decompose_batch(gs, sides, with_stats=True, flags=tip.TIP_FLAG_BATCH_PLAIN)
    for g, s, a, b, c in zip(gs, sides, tu, ts, tp):
        th = oracle.bup(g, s)[0]
        np.testing.assert_array_equal(a, th)
        np.testing.assert_array_equal(b, th)
        np.testing.assert_array_equal(c, th)
    for x, y in zip(ss, sp):
        for k in ("wedges_count", "wedges_cd", "wedges_fd", "pair_updates", "subsets", "fd_levels"):
            assert x[k] == y[k], k
    assert su[0]["m_unique"] == sum(y["m_unique"] for y in sp)
    assert all(x["m_unique"] == 0 for x in su[1:])


def test_batch_with_empty_and_tiny_graphs(gpu_lib):
    gs = [gg.Graph(3, 2, np.zeros(0, np.int32), np.zeros(0, np.int32), "empty"),
          gg.complete_bipartite(4, 3), gg.star(5), gg.chung_lu(900, 300, 6000, 2.2, 2.3, seed=41)]
    out = tip.decompose_batch(gs, [0, 1, 0, 0])
    for g, s, th in zip(gs, [0, 1, 0, 0], out):
        np.testing.assert_array_equal(th, oracle.bup(g, s)[0])


def test_async_device_resident(gpu_lib):
    import torch
    g = gg.chung_lu(3000, 700, 25000, 2.2, 2.1, seed=17)
    dev = torch.device("cuda:0")
    d_eu = torch.from_numpy(g.eu).to(dev)
    d_ev = torch.from_numpy(g.ev).to(dev)
    for side in (0, 1):
        n = g.n_u if side == 0 else g.n_v
        ws = torch.empty(tip.workspace_size(g.n_u, g.n_v, g.m, side), dtype=torch.uint8, device=dev)
        d_theta = torch.empty(n, dtype=torch.int64, device=dev)
        tip.decompose_async(d_eu, d_ev, g.n_u, g.n_v, side, d_theta, ws)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(d_theta.cpu().numpy(), oracle.bup(g, side)[0])


def test_async_reports_bad_ids(gpu_lib):
    import torch
    dev = torch.device("cuda:0")
    d_eu = torch.tensor([0, 1, 5], dtype=torch.int32, device=dev)
    d_ev = torch.tensor([0, 1, 1], dtype=torch.int32, device=dev)
    ws = torch.empty(tip.workspace_size(3, 2, 3, 0), dtype=torch.uint8, device=dev)
    d_theta = torch.empty(3, dtype=torch.int64, device=dev)
    with pytest.raises(tip.TipError) as ei:
        tip.decompose_async(d_eu, d_ev, 3, 2, 0, d_theta, ws)
    assert ei.value.status == tip.TIP_EINVAL


def _golden(name):
    path = os.path.join(GOLDEN, f"{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"no golden file for {name}")
    with open(path) as f:
        return json.load(f)


@pytest.mark.parametrize("name", ["cl-1m", "cl-10m"])
def test_full_size_against_golden(gpu_lib, name):
    rec = _golden(name)
    g = gg.config_graph(name)
    assert gg.graph_sha256(g) == rec["graph_sha256"]
    bu, bv, tot = tip.count_butterflies(g)
    c = rec["count"]
    assert tot == c["total"]
    assert digest(bu) == c["sha256_u"] and digest(bv) == c["sha256_v"]
    for side, key in ((0, "theta_u"), (1, "theta_v")):
        if key not in rec:
            continue
        th = tip.decompose(g, side)
        s = rec[key]["sample"]
        np.testing.assert_array_equal(th[s["index"]], s["value"])
        assert int(th.max()) == rec[key]["max"] and int(th.sum()) == rec[key]["sum"]
        assert digest(th) == rec[key]["sha256"]


def test_batch_with_large_subsets_against_golden(gpu_lib):
    """A batch holding graphs whose first subsets are large enough for the
    fine-grained help board (4,096+ vertices): the single fine-grained launch
    then publishes levels of jobs taken from the job list.  Results equal the
    stored golden ones and the oracle."""
    rec = _golden("cl-1m")
    big = gg.config_graph("cl-1m")
    small = gg.chung_lu(2000, 500, 15000, 2.2, 2.1, seed=71)
    ex = tip.decompose_ex(big, 0)
    sizes = np.bincount(ex["subset"], minlength=ex["n_subsets"])
    assert sizes.max() >= 4096
    out = tip.decompose_batch([small, big, big], [0, 0, 1])
    np.testing.assert_array_equal(out[0], oracle.bup(small, 0)[0])
    assert digest(out[1]) == rec["theta_u"]["sha256"]
    assert digest(out[2]) == rec["theta_v"]["sha256"]


@pytest.mark.parametrize("P", [5, 150])
def test_huc_recount_changes_nothing(gpu_lib, P):
    """HUC (Section 4.1): with a threshold of 1% nearly every coarse-grained
    round re-counts the live supports (Alg. 1 on the live graph) instead of
    peeling; the subsets, their initial supports and the tip numbers are
    those of peeling, in graph replay and in host-launched rounds."""
    g = gg.chung_lu(6000, 1200, 60000, 2.2, 2.0, seed=43)
    th = oracle.bup(g, 0)[0]
    ref = tip.decompose_ex(g, 0, P=P)
    for flags in (0, tip.TIP_FLAG_NO_GRAPH):
        got = tip.decompose_ex(g, 0, P=P, flags=flags, tune=[0, 0, 0, 1])
        np.testing.assert_array_equal(got["theta"], th)
        np.testing.assert_array_equal(got["subset"], ref["subset"])
        np.testing.assert_array_equal(got["init"], ref["init"])
        np.testing.assert_array_equal(got["bounds"], ref["bounds"])
        assert got["stats"]["huc_rounds"] > 0
        assert got["stats"]["rounds"] == ref["stats"]["rounds"]
    assert ref["stats"]["huc_rounds"] == 0
    # side V and a degenerate graph
    np.testing.assert_array_equal(tip.decompose(g, 1, tune=[0, 0, 0, 1]), oracle.bup(g, 1)[0])
    k = gg.complete_bipartite(30, 20)
    np.testing.assert_array_equal(tip.decompose(k, 0, tune=[0, 0, 0, 1]), np.full(30, 29 * comb(20, 2)))


def test_hubs_above_sixteen_bit_counts(gpu_lib):
    """Vertices of degree above 65,535 share more than 65,535 neighbours with
    others, so the dense path counts them with 32-bit counters.  K_{2,70000}
    (theta = C(70000, 2) for both U vertices, closed form), and a Chung-Lu
    graph whose V side has three hubs of degree about 82K, peeled on V and
    checked against the oracle."""
    k = gg.complete_bipartite(2, 70000)
    np.testing.assert_array_equal(tip.decompose(k, 0), np.full(2, comb(70000, 2)))
    g = gg.chung_lu(200000, 300, 1_000_000, 2.5, 1.8, seed=61, cap_v=1.5e5)
    assert (np.bincount(g.ev, minlength=g.n_v) > 65535).sum() == 3
    np.testing.assert_array_equal(tip.decompose(g, 1), oracle.bup(g, 1)[0])


def test_two_hub_stars_are_not_refused(gpu_lib):
    """A U hub and a V hub of degree 2.7M each (m = 5.4M) hold no butterfly.
    Every count and tip number is 0 and every call returns TIP_OK: no count
    bound is applied that could refuse a valid graph."""
    k = 2_700_000
    eu = np.concatenate([np.zeros(k, np.int32), np.arange(1, k + 1, dtype=np.int32)])
    ev = np.concatenate([np.arange(1, k + 1, dtype=np.int32), np.zeros(k, np.int32)])
    g = gg.Graph(k + 1, k + 1, eu, ev, "two-stars")
    bu, bv, tot = tip.count_butterflies(g)
    assert tot == 0 and not bu.any() and not bv.any()
    for side in (0, 1):
        th = tip.decompose(g, side)
        assert th.shape == (k + 1,) and not th.any()


def test_help_board_tunables_change_nothing(gpu_lib):
    """The fine-grained help-board parameters (tune[4..6]) only change which
    workgroups apply a level's updates: with every subset opening a slot,
    every level published and one update per claim, cl-1m's tip numbers on
    both sides equal the oracle's stored digests, as with the defaults."""
    rec = _golden("cl-1m")
    g = gg.config_graph("cl-1m")
    for side, key in ((0, "theta_u"), (1, "theta_v")):
        for tune in ([0, 0, 0, 0, 1, 1, 1], [0, 0, 0, 0, 64, 4096, 100000]):
            assert digest(tip.decompose(g, side, tune=tune)) == rec[key]["sha256"], (side, tune)


def test_batch_with_per_graph_tunings(gpu_lib):
    """tip_decompose_batch with one tip_opts per graph (each graph its own
    tuning, as the autotuner stores them): batched and plain forms equal the
    oracle."""
    params = gg.batch_params(6, seed_base=3100, m_lo=3e3, m_hi=3e4)
    gs = [gg.batch_graph(p) for p in params]
    tunes = [None, [256, 1024, 0, 0, 8, 128, 0, 0], [2048, 8192, 0, 0, 64, 512, 0, 0],
             [512, 4096, 0, 0, 1, 1, 1, 0], None, [1024, 2048, 0, 0, 32, 256, 0, 0]]
    for flags in (0, tip.TIP_FLAG_BATCH_PLAIN):
        out = tip.decompose_batch(gs, [0] * len(gs), flags=flags, tunes=tunes)
        for g, th in zip(gs, out):
            np.testing.assert_array_equal(th, oracle.bup(g, 0)[0])


def test_fd_huc_recount_changes_nothing(gpu_lib):
    """HUC in the fine-grained step (Section 4.1, last paragraph): with a
    threshold of 1%, nearly every step of a subset kept in HBM re-counts its
    live supports (support at the range start minus the butterflies shared
    with the subset's peeled vertices) instead of applying its updates.  The
    subsets, initial supports, bounds and tip numbers are those of peeling;
    on cl-1m both sides keep the oracle's digests."""
    g = gg.chung_lu(20000, 3000, 150000, 2.2, 2.0, seed=47)
    th = oracle.bup(g, 0)[0]
    for P in (1, 3):
        ref = tip.decompose_ex(g, 0, P=P)
        got = tip.decompose_ex(g, 0, P=P, tune=[0, 0, 0, 0, 0, 0, 0, 1])
        assert got["stats"]["fd_huc_steps"] > 0 and ref["stats"]["fd_huc_steps"] == 0
        np.testing.assert_array_equal(got["theta"], th)
        np.testing.assert_array_equal(got["subset"], ref["subset"])
        np.testing.assert_array_equal(got["init"], ref["init"])
        np.testing.assert_array_equal(got["bounds"], ref["bounds"])
    rec = _golden("cl-1m")
    c1 = gg.config_graph("cl-1m")
    for side, key in ((0, "theta_u"), (1, "theta_v")):
        out, st = tip.decompose(c1, side, P=4, tune=[0, 0, 0, 0, 0, 0, 0, 1], with_stats=True)
        assert st["fd_huc_steps"] > 0
        assert digest(out) == rec[key]["sha256"], side


def test_fd_dgm_changes_nothing_but_work(gpu_lib):
    """DGM in the fine-grained step (Section 4.2, TIP_FLAG_FD_DGM): a subset
    kept in HBM drops its peeled vertices from G_i's neighbour runs each time
    its updates walked as many wedges as G_i has edges.  Subsets, initial
    supports, bounds and tip numbers are unchanged, and the fine-grained step
    walks no more wedges; cl-1m keeps the oracle's digests on both sides."""
    g = gg.chung_lu(20000, 3000, 150000, 2.2, 2.0, seed=47)
    th = oracle.bup(g, 0)[0]
    for P in (1, 3):
        ref = tip.decompose_ex(g, 0, P=P)
        got = tip.decompose_ex(g, 0, P=P, flags=tip.TIP_FLAG_FD_DGM)
        assert got["stats"]["compactions"] >> 32 > 0 and ref["stats"]["compactions"] >> 32 == 0
        assert got["stats"]["wedges_fd"] < ref["stats"]["wedges_fd"]
        np.testing.assert_array_equal(got["theta"], th)
        np.testing.assert_array_equal(got["subset"], ref["subset"])
        np.testing.assert_array_equal(got["init"], ref["init"])
        np.testing.assert_array_equal(got["bounds"], ref["bounds"])
    rec = _golden("cl-1m")
    c1 = gg.config_graph("cl-1m")
    for side, key in ((0, "theta_u"), (1, "theta_v")):
        out, st = tip.decompose(c1, side, P=4, flags=tip.TIP_FLAG_FD_DGM, with_stats=True)
        assert st["compactions"] >> 32 > 0
        assert digest(out) == rec[key]["sha256"], side
    # with HUC forced in the same subsets, compaction stays off (a re-count
    # needs the peeled vertices) and results stay exact
    got = tip.decompose_ex(g, 0, P=1, flags=tip.TIP_FLAG_FD_DGM, tune=[0, 0, 0, 0, 0, 0, 0, 1])
    assert got["stats"]["compactions"] >> 32 == 0 and got["stats"]["fd_huc_steps"] > 0
    np.testing.assert_array_equal(got["theta"], th)


def test_fd_pair_rows_change_nothing(gpu_lib, monkeypatch):
    """The fine-grained step's pair rows (each vertex's update inside its
    subset, listed before peeling; the default) against walking every
    update's wedges (TIP_FLAG_FD_WALK, Alg. 4 as written): the same subsets,
    initial supports, bounds, tip numbers, levels and support decrements,
    with subsets kept in LDS and in HBM.  With the rows' budget cut
    (TIP_FD_PAIR_LIMIT) some subsets read rows and the others walk, and the
    results stay the same."""
    g = gg.chung_lu(20000, 3000, 150000, 2.2, 2.0, seed=47)
    th = oracle.bup(g, 0)[0]
    keys = ("subset", "init", "bounds")
    for P in (1, 3, 40):
        ref = tip.decompose_ex(g, 0, P=P, flags=tip.TIP_FLAG_FD_WALK)
        got = tip.decompose_ex(g, 0, P=P)
        assert ref["stats"]["fd_pair_subsets"] == 0 and ref["stats"]["fd_pair_entries"] == 0
        np.testing.assert_array_equal(ref["theta"], th)
        np.testing.assert_array_equal(got["theta"], th)
        for k in keys:
            np.testing.assert_array_equal(got[k], ref[k])
        assert got["stats"]["fd_levels"] == ref["stats"]["fd_levels"], P
        assert got["stats"]["pair_updates"] == ref["stats"]["pair_updates"], P
    assert got["stats"]["fd_pair_subsets"] > 0 and got["stats"]["fd_pair_entries"] > 0
    mixed = False
    for lim in (1 << 12, 1 << 14, 1 << 16, 1 << 18):
        monkeypatch.setenv("TIP_FD_PAIR_LIMIT", str(lim))
        cut = tip.decompose_ex(g, 0, P=40)
        k = cut["stats"]["fd_pair_subsets"]
        mixed = mixed or 0 < k < cut["stats"]["subsets"]
        np.testing.assert_array_equal(cut["theta"], th)
        assert cut["stats"]["pair_updates"] == got["stats"]["pair_updates"]
    assert mixed
    # side V, and the graph-replayed path with the rows on
    th_v = oracle.bup(g, 1)[0]
    monkeypatch.delenv("TIP_FD_PAIR_LIMIT")
    out, st = tip.decompose(g, 1, P=20, with_stats=True)
    assert st["fd_pair_subsets"] > 0
    np.testing.assert_array_equal(out, th_v)


def test_cd_dgm_paper_trigger_changes_nothing(gpu_lib):
    """Section 4.2's own trigger for the coarse-grained lists
    (TIP_FLAG_DGM_PAPER: compact once the wedges walked since the last
    compaction reach the entries left): same subsets, supports, bounds and
    tip numbers as with the default trigger and with no compaction."""
    g = gg.chung_lu(6000, 1200, 60000, 2.2, 2.0, seed=43)
    th = oracle.bup(g, 0)[0]
    ref = tip.decompose_ex(g, 0, flags=tip.TIP_FLAG_NO_COMPACT)
    got = tip.decompose_ex(g, 0, flags=tip.TIP_FLAG_DGM_PAPER)
    assert got["stats"]["compactions"] & 0xffffffff > 0
    assert got["stats"]["wedges_cd"] <= ref["stats"]["wedges_cd"]
    np.testing.assert_array_equal(got["theta"], th)
    for k in ("subset", "init", "bounds"):
        np.testing.assert_array_equal(got[k], ref[k])
    rec = _golden("cl-1m")
    assert digest(tip.decompose(gg.config_graph("cl-1m"), 0, flags=tip.TIP_FLAG_DGM_PAPER)) == rec["theta_u"]["sha256"]
