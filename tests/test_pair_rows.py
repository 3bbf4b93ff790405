"""The facts the fine-grained pair rows rest on, checked on the CPU against
the oracle (no GPU).

Peeling u inside a subset U_i lowers every w of U_i by C(c(u, w), 2), with
c(u, w) the common neighbours over all of the other side (Alg. 4 on G_i;
the other side is never peeled, so c does not change while U_i is peeled).
The library lists that update once per vertex as its pair row: the w != u of
U_i with c(u, w) >= 2 and C(c, 2).  Checked here:

* a row has at most min(n_i - 1, fd_w / 2) entries, where fd_w is the sum
  over u's edges (u, v) of |N_v inside U_i| - 1 (the capacity the workspace
  reserves per row);
* with all of a side in one subset, a row's C(c, 2) sum is u's butterfly
  count (Section 2.1), equal to the oracle's;
* bottom-up peeling that applies rows level by level (all vertices at or
  below the level at once) gives the oracle's tip numbers.
"""
from __future__ import annotations

import numpy as np

import oracle
from paper_2010_08695_amd import graphgen as gg


def _codegree(g, side):
    """Dense co-degree matrix c(x, w) of one side and its degrees."""
    a = np.zeros((g.n_u, g.n_v), np.int64)
    a[g.eu, g.ev] = 1
    if side == 1:
        a = a.T
    return a @ a.T, a


def _graphs():
    for i in range(12):
        yield gg.tiny_random(4 + i % 9, 3 + (i * 5) % 8, 0.2 + 0.07 * (i % 10), 900 + i)
    yield gg.chung_lu(300, 90, 2500, 2.2, 2.0, seed=5)
    yield gg.complete_bipartite(7, 5)


def _choose2(c):
    return c * (c - 1) // 2


def test_row_length_within_the_reserved_capacity():
    rng = np.random.default_rng(3)
    for g in _graphs():
        for side in (0, 1):
            c, a = _codegree(g, side)
            n = c.shape[0]
            for n_sub in (1, 3, 7):
                label = rng.integers(0, n_sub, n)
                for u in range(n):
                    same = label == label[u]
                    same[u] = False
                    n_i = int(same.sum()) + 1
                    # fd_w from the lists: for every neighbour v of u, the
                    # other members of U_i in N_v
                    nbrs = np.nonzero(a[u])[0]
                    fd_w = int(sum(int(a[same, v].sum()) for v in nbrs))
                    assert fd_w == int(c[u, same].sum())
                    entries = int((c[u, same] >= 2).sum())
                    assert entries <= min(n_i - 1, fd_w // 2), (g.name, side, u)


def test_one_subset_rows_sum_to_the_butterfly_counts():
    for g in _graphs():
        bu, bv, _ = oracle.count(g)
        for side, cnt in ((0, bu), (1, bv)):
            c, _ = _codegree(g, side)
            np.fill_diagonal(c, 0)
            rows = _choose2(c).sum(axis=1)
            np.testing.assert_array_equal(rows, cnt, err_msg=f"{g.name} side {side}")


def _peel_with_rows(c, support):
    """Level-synchronous bottom-up peeling from the given supports, each
    peeled vertex applying its row to the vertices still live."""
    n = len(support)
    sup = support.astype(np.int64).copy()
    rows = _choose2(c)
    np.fill_diagonal(rows, 0)
    alive = np.ones(n, bool)
    theta = np.zeros(n, np.int64)
    level = 0
    while alive.any():
        level = max(level, int(sup[alive].min()))
        peel = alive & (sup <= level)
        theta[peel] = level
        alive &= ~peel
        sup[alive] -= rows[np.ix_(peel, alive)].sum(axis=0)
    return theta


def test_peeling_from_rows_gives_the_oracle_tip_numbers():
    for g in _graphs():
        bu, bv, _ = oracle.count(g)
        for side, cnt in ((0, bu), (1, bv)):
            c, _ = _codegree(g, side)
            np.testing.assert_array_equal(_peel_with_rows(c, cnt), oracle.bup(g, side)[0],
                                          err_msg=f"{g.name} side {side}")
