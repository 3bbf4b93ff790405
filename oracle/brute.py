"""Exponential brute force for tiny graphs (|U| <= 14, |V| <= 12).

TEST INFRASTRUCTURE ONLY.  These are the textbook definitions, written out
with no algorithmic shortcut, used to pin the oracle itself:

* ``butterflies(g)``: every butterfly is a 2x2 biclique {u1, u2} x {v1, v2}
  whose four edges are all present (Section 2.1); enumerate all such 4-tuples.
* ``tip_numbers(g, side)``: Def. 1 read as "theta_u is the largest k such that
  u lies in a vertex subset S of its side in which every member takes part in
  at least k butterflies of the subgraph induced on S and the whole other
  side"; enumerate all subsets S.
"""
from __future__ import annotations

import itertools

import numpy as np


def dense(g) -> np.ndarray:
    a = np.zeros((g.n_u, g.n_v), dtype=np.int64)
    a[g.eu.astype(np.int64), g.ev.astype(np.int64)] = 1
    return a


def butterflies(g):
    """Returns (per-U counts, per-V counts, total) by 4-tuple enumeration."""
    a = dense(g)
    bu = np.zeros(g.n_u, np.int64)
    bv = np.zeros(g.n_v, np.int64)
    total = 0
    for u1, u2 in itertools.combinations(range(g.n_u), 2):
        for v1, v2 in itertools.combinations(range(g.n_v), 2):
            if a[u1, v1] and a[u1, v2] and a[u2, v1] and a[u2, v2]:
                total += 1
                bu[u1] += 1
                bu[u2] += 1
                bv[v1] += 1
                bv[v2] += 1
    return bu, bv, total


def _pair_butterflies(a: np.ndarray) -> np.ndarray:
    """B[x, w] = butterflies containing both x and w (rows of ``a`` are one
    side), by enumerating every pair of columns both rows contain."""
    n, k = a.shape
    b = np.zeros((n, n), np.int64)
    for x in range(n):
        for w in range(n):
            if x == w:
                continue
            s = 0
            for y1, y2 in itertools.combinations(range(k), 2):
                if a[x, y1] and a[x, y2] and a[w, y1] and a[w, y2]:
                    s += 1
            b[x, w] = s
    return b


def tip_numbers(g, side: int = 0) -> np.ndarray:
    """theta_u = max over S containing u of min over x in S of f_x(S)."""
    a = dense(g)
    if side == 1:
        a = a.T.copy()
    n = a.shape[0]
    if n > 16:
        raise ValueError("brute force needs at most 16 vertices on the side")
    theta = np.zeros(n, np.int64)
    if n == 0:
        return theta
    b = _pair_butterflies(a)
    masks = np.arange(1, 1 << n, dtype=np.int64)
    member = ((masks[:, None] >> np.arange(n)[None, :]) & 1).astype(np.int64)
    f = member @ b                      # f[s, x] = sum_{w in S_s} B[x, w]
    big = np.iinfo(np.int64).max
    fmin = np.where(member == 1, f, big).min(axis=1)
    for x in range(n):
        theta[x] = fmin[member[:, x] == 1].max()
    return theta


# ---------------------------------------------------------------------------
# Edges and k-tips
# ---------------------------------------------------------------------------

def canonical(g):
    """Distinct edges sorted by (u, v), as two int arrays."""
    key = np.unique(g.eu.astype(np.int64) * max(g.n_v, 1) + g.ev.astype(np.int64))
    return (key // max(g.n_v, 1)).astype(np.int64), (key % max(g.n_v, 1)).astype(np.int64)


def _butterfly_list(g):
    """Every butterfly as the four canonical edge ids it consists of."""
    cu, cv = canonical(g)
    eid = {(int(u), int(v)): i for i, (u, v) in enumerate(zip(cu, cv))}
    out = []
    for u1, u2 in itertools.combinations(range(g.n_u), 2):
        for v1, v2 in itertools.combinations(range(g.n_v), 2):
            es = [eid.get((u1, v1)), eid.get((u1, v2)), eid.get((u2, v1)), eid.get((u2, v2))]
            if all(e is not None for e in es):
                out.append(es)
    return out, cu.shape[0]


def edge_butterflies(g) -> np.ndarray:
    """Butterflies containing each canonical edge, by 4-tuple enumeration."""
    bf, m = _butterfly_list(g)
    cnt = np.zeros(m, np.int64)
    for es in bf:
        for e in es:
            cnt[e] += 1
    return cnt


def wing_numbers(g) -> np.ndarray:
    """psi_e = max over edge sets S containing e of min over f in S of the
    butterflies of f inside S (the k-wing analogue of Def. 1), enumerating
    every edge subset (at most 16 edges)."""
    bf, m = _butterfly_list(g)
    if m > 16:
        raise ValueError("brute force needs at most 16 edges")
    psi = np.zeros(m, np.int64)
    if m == 0:
        return psi
    masks = np.arange(1, 1 << m, dtype=np.int64)
    member = ((masks[:, None] >> np.arange(m)[None, :]) & 1).astype(np.int64)
    f = np.zeros((masks.shape[0], m), np.int64)
    for es in bf:
        inside = member[:, es].all(axis=1).astype(np.int64)
        for e in es:
            f[:, e] += inside
    big = np.iinfo(np.int64).max
    fmin = np.where(member == 1, f, big).min(axis=1)
    for e in range(m):
        psi[e] = fmin[member[:, e] == 1].max()
    return psi


def ktips(g, side: int, k: int) -> np.ndarray:
    """Def. 1 read literally: the maximal vertex sets S of the side in which
    every member takes part in at least k butterflies of the subgraph on S
    and the whole other side, and every two members are joined by a chain of
    members that pairwise share a butterfly; enumerates every subset (at most
    12 vertices).  Returns each vertex's set labelled by its smallest member,
    -1 outside every such set."""
    a = dense(g)
    if side == 1:
        a = a.T.copy()
    n = a.shape[0]
    if n > 12:
        raise ValueError("brute force needs at most 12 vertices on the side")
    b = _pair_butterflies(a)
    valid = []
    for mask in range(1, 1 << n):
        s = [x for x in range(n) if mask >> x & 1]
        if min(sum(b[x, w] for w in s) for x in s) < k:
            continue
        seen, todo = {s[0]}, [s[0]]
        while todo:
            x = todo.pop()
            for w in s:
                if w not in seen and b[x, w] > 0:
                    seen.add(w)
                    todo.append(w)
        if len(seen) == len(s):
            valid.append(mask)
    maximal = [s for s in valid if not any(t != s and (s & t) == s for t in valid)]
    comp = np.full(n, -1, np.int64)
    for s in maximal:
        members = [x for x in range(n) if s >> x & 1]
        for x in members:
            assert comp[x] == -1, "maximal k-tips overlap"
            comp[x] = members[0]
    return comp
