"""Properties that tip numbers and butterfly counts must satisfy at any size.

Each check takes the graph, a tip-number (or count) array, and optionally a
sample of vertices, and raises AssertionError with a message on failure.
They use only ``oracle.support_in`` (the plain f_x(S) definition) and numpy.

Why they hold (Def. 1 / generalized-core reading of tip numbers):
* pair bound:   u and w share C(c(u,w),2) butterflies, so S = {u, w} shows
                theta_u >= C(c(u,w),2) for every w; and theta_u <= count_u.
* certificate:  H = {x : theta_x >= theta_u} is a theta_u-tip containing u,
                so f_u(H) >= theta_u.
* level:        for each value k taken by theta, min over H_k of f(H_k) = k
                (otherwise all of H_k would have a larger tip number).
"""
from __future__ import annotations

import numpy as np

import oracle


def c2(c):
    c = np.asarray(c, dtype=np.int64)
    return c * (c - 1) // 2


def side_adjacency(g, side: int):
    """(n_a, rows of the side as python sets of other-side ids)."""
    if side == 0:
        n, a, b = g.n_u, g.eu, g.ev
    else:
        n, a, b = g.n_v, g.ev, g.eu
    rows = [[] for _ in range(n)]
    for x, y in zip(a.tolist(), b.tolist()):
        rows[x].append(y)
    return n, rows


def check_count_sums(bu, bv, total):
    assert int(bu.sum()) == 2 * total, (int(bu.sum()), total)
    assert int(bv.sum()) == 2 * total, (int(bv.sum()), total)


def check_bounds(g, side, theta, count, sample=None):
    """theta <= count; theta == 0 iff count == 0; max pair term <= theta."""
    assert (theta <= count).all(), "theta exceeds the butterfly count"
    assert ((theta == 0) == (count == 0)).all(), "theta == 0 iff count == 0 violated"
    n, rows = side_adjacency(g, side)
    other = 1 - side
    _, cols = side_adjacency(g, other)
    idx = range(n) if sample is None else sample
    for u in idx:
        cnt = {}
        for y in rows[u]:
            for w in cols[y]:
                if w != u:
                    cnt[w] = cnt.get(w, 0) + 1
        best = max((c * (c - 1) // 2 for c in cnt.values()), default=0)
        assert best <= theta[u], (u, best, theta[u])


def check_certificate(g, side, theta, sample):
    """f_u({x : theta_x >= theta_u}) >= theta_u for sampled u."""
    sample = np.asarray(sample, dtype=np.int32)
    by_level: dict[int, list[int]] = {}
    for u in sample.tolist():
        by_level.setdefault(int(theta[u]), []).append(u)
    for k, us in by_level.items():
        member = (theta >= k).astype(np.uint8)
        f = oracle.support_in(g, side, member, np.array(us, np.int32))
        assert (f >= k).all(), (k, us, f)


def check_levels(g, side, theta, levels=None):
    """For each chosen value k of theta: min over H_k of f(H_k) == k."""
    vals = np.unique(theta)
    if levels is not None:
        vals = np.asarray(levels)
    for k in vals.tolist():
        member = (theta >= k).astype(np.uint8)
        h = np.nonzero(member)[0].astype(np.int32)
        f = oracle.support_in(g, side, member, h)
        assert int(f.min()) == int(k), (k, int(f.min()))
