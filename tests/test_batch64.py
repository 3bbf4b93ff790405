"""The 64-graph batch workload (Chung-Lu graphs, m log-uniform in [1e4, 2e6],
|U|:|V| in [1, 8], exponents in [2.0, 2.8], U side, P = 150) decomposed in
one tip_decompose_batch call, batched and plain: every graph's tip numbers
equal the SHA-256 digest the oracle's sequential bottom-up peel gave
(tests/golden/batch-64.json; Theorem 2: RECEIPT computes BUP's tip numbers),
and the two forms agree on every graph's work counters."""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np
import pytest

from paper_2010_08695_amd import autotune
from paper_2010_08695_amd import graphgen as gg
from paper_2010_08695_amd import tip

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "batch-64.json")


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i8").tobytes()).hexdigest()


@pytest.fixture(scope="module")
def batch():
    with open(GOLDEN) as f:
        gold = json.load(f)
    params = gg.batch_params(64)
    graphs = [gg.batch_graph(p) for p in params]
    for g, rec in zip(graphs, gold["graphs"]):
        assert gg.graph_sha256(g) == rec["graph_sha256"], g.name
    return graphs, gold


def test_batch64_against_oracle_digests(gpu_lib, batch):
    """Union form (default), streams form and plain form: every graph's tip
    numbers equal the oracle's digest; the streams form's per-graph work
    equals the plain form's."""
    graphs, gold = batch
    sides = [0] * len(graphs)
    tu = tip.decompose_batch(graphs, sides, P=150)
    ts, ss = tip.decompose_batch(graphs, sides, P=150, with_stats=True, flags=tip.TIP_FLAG_BATCH_STREAMS)
    tp, sp = tip.decompose_batch(graphs, sides, P=150, with_stats=True, flags=tip.TIP_FLAG_BATCH_PLAIN)
    for form, out in (("union", tu), ("streams", ts), ("plain", tp)):
        bad = [g.name for g, th, rec in zip(graphs, out, gold["graphs"]) if digest(th) != rec["theta_u"]["sha256"]]
        assert not bad, (form, bad)
    for g, x, y in zip(graphs, ss, sp):
        for k in ("wedges_count", "wedges_cd", "wedges_fd", "pair_updates", "subsets", "fd_levels"):
            assert x[k] == y[k], (g.name, k)


def test_batch64_with_stored_tunings(gpu_lib, batch):
    """The batch with each graph's stored tuning (the package table) gives the
    same tip numbers."""
    graphs, gold = batch
    tunes = autotune.batch_tunes(graphs, [0] * len(graphs))
    out = tip.decompose_batch(graphs, [0] * len(graphs), P=150, tunes=tunes)
    bad = [g.name for g, th, rec in zip(graphs, out, gold["graphs"]) if digest(th) != rec["theta_u"]["sha256"]]
    assert not bad, bad
