"""The large skewed workload cl-100m-skew: |U| = 2e7, |V| = 2e6, about
9.1e7 edges, V hubs of degree about 4e5; both sides in turn, CD rounds
replayed from captured HIP graphs.

Side V is compared in full with the oracle: its per-vertex counts and tip
numbers equal the SHA-256 digests tests/golden/make_golden.py wrote from the
oracle's sequential bottom-up peel (Theorem 2: RECEIPT computes BUP's tip
numbers).  The total butterfly count, twice of which is the sum of either
side's counts, follows from the V counts and pins the sum of the U counts.

On side U the oracle's full peel is out of reach (it walks about 9e12
wedges, weeks of CPU time), so U's tip numbers are checked by properties
that hold at any size, on sampled vertices the oracle evaluates one by one
from the plain definition of f_x(S):
* per-vertex butterfly counts: f_x(whole side) equals the GPU count, and the
  per-side sums are twice the total;
* theta_x <= count_x, and theta_x == 0 exactly when count_x == 0;
* certificate: H = {w : theta_w >= theta_x} is a theta_x-tip holding x, so
  f_x(H) >= theta_x;
* peel bound: when bottom-up peeling removes x, every vertex with a larger
  tip number is still present and x's support is at most theta_x, so
  f_x({w : theta_w > theta_x}) <= theta_x.

The run takes about four minutes, two of them generating the graph on the
host.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np
import pytest

import oracle
from paper_2010_08695_amd import graphgen as gg
from paper_2010_08695_amd import tip

import _props

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "cl-100m-skew.json")


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i8").tobytes()).hexdigest()


def _sample(theta, count, seed):
    """Random vertices with theta > 0, random ones with theta == 0, and the
    vertices of the largest tip numbers and counts."""
    rng = np.random.default_rng(seed)
    pos = np.nonzero(theta > 0)[0]
    zero = np.nonzero(theta == 0)[0]
    parts = [rng.choice(pos, min(48, len(pos)), replace=False),
             rng.choice(zero, min(8, len(zero)), replace=False),
             np.argsort(theta, kind="stable")[-8:], np.argsort(count, kind="stable")[-8:]]
    return np.unique(np.concatenate(parts)).astype(np.int32)


def test_large_skewed_both_sides(gpu_lib, capsys):
    t0 = time.time()

    def log(msg):
        # progress goes past pytest's capture: the steps below run for
        # minutes without another test finishing
        with capsys.disabled():
            print(f"[{time.time() - t0:6.1f}s] {msg}", flush=True)

    with open(GOLDEN) as f:
        gold = json.load(f)
    log("generating cl-100m-skew")
    g = gg.config_graph("cl-100m-skew")
    assert gg.graph_sha256(g) == gold["graph_sha256"]
    du = np.bincount(g.eu, minlength=g.n_u).astype(np.int64)
    dv = np.bincount(g.ev, minlength=g.n_v).astype(np.int64)
    wedges = int((du * (du - 1) // 2).sum() + (dv * (dv - 1) // 2).sum())
    log(f"graph m={g.m} max d_u={du.max()} max d_v={dv.max()} wedge total={wedges}")
    bu, bv, tot = tip.count_butterflies(g)
    _props.check_count_sums(bu, bv, tot)
    log(f"butterflies {tot}")
    # V counts and the total against the oracle
    assert digest(bv) == gold["count"]["sha256_v"]
    assert tot == gold["count"]["total"] and int(bu.sum()) == gold["count"]["sum_v"]
    for side in (1, 0):
        count = bu if side == 0 else bv
        th, st = tip.decompose(g, side, with_stats=True)
        log(f"side {'UV'[side]}: {st['t_total_ms']:.1f} ms (count {st['t_count_ms']:.1f}, cd {st['t_cd_ms']:.1f}, "
            f"fd {st['t_fd_ms']:.1f}), {st['rounds']} rounds, {st['subsets']} subsets, "
            f"{st['wedges_count'] + st['wedges_cd'] + st['wedges_fd']:.4g} wedges, theta max {th.max()}")
        if side == 1:
            # full parity with the oracle's bottom-up peel
            assert digest(th) == gold["theta_v"]["sha256"]
            assert int(th.max()) == gold["theta_v"]["max"] and int(th.sum()) == gold["theta_v"]["sum"]
            log("side V: tip numbers equal the oracle's digest")
        assert (th <= count).all(), "theta exceeds the butterfly count"
        assert ((th == 0) == (count == 0)).all(), "theta == 0 iff count == 0 violated"
        q = _sample(th, count, 11 + side)
        lv = oracle.support_levels(g, side, th, q)
        log(f"side {'UV'[side]}: oracle checked {len(q)} sampled vertices")
        np.testing.assert_array_equal(lv[:, 0], count[q])
        bad = q[lv[:, 1] < th[q]]
        assert len(bad) == 0, ("certificate", bad[:8], th[bad[:8]])
        bad = q[lv[:, 2] > th[q]]
        assert len(bad) == 0, ("peel bound", bad[:8], th[bad[:8]])
