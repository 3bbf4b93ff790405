"""Seeded synthetic bipartite graphs used as inputs everywhere.

This module only *draws* edge lists.  It holds none of the tip-decomposition
arithmetic (no counting, no peeling), so that both the HIP path and the CPU
oracle can be fed from it without sharing any of the method's code.

The paper evaluates on KONECT bipartite graphs that are not available here
(experiments, dataset table).  The Chung-Lu generator below stands in for
them: power-law expected degrees on both sides, with the skew the dataset
table shows (average degree 5-118, a few very large hubs), which produces the
long tail of tip numbers the paper reports for the trackers graph.

All generators return ``(n_u, n_v, eu, ev)`` with ``eu``/``ev`` int32 arrays
of 0-based ids and no duplicate edges.  Isolated vertices stay in the id
space.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Graph", "uniform_bipartite", "chung_lu", "complete_bipartite",
    "complete_minus_matching", "star", "random_tree", "tiny_random",
    "disjoint_union", "permute_ids", "transpose", "config_graph",
    "batch_params", "serving_trace", "graph_sha256",
]


@dataclass
class Graph:
    """A bipartite edge list: U ids in ``eu``, V ids in ``ev`` (int32)."""
    n_u: int
    n_v: int
    eu: np.ndarray
    ev: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.eu.shape[0])


def _finish(n_u: int, n_v: int, u: np.ndarray, v: np.ndarray, name: str,
            meta: dict | None = None) -> Graph:
    key = np.unique(u.astype(np.int64) * np.int64(max(n_v, 1)) + v.astype(np.int64))
    eu = (key // max(n_v, 1)).astype(np.int32)
    ev = (key % max(n_v, 1)).astype(np.int32)
    return Graph(int(n_u), int(n_v), eu, ev, name, dict(meta or {}))


def uniform_bipartite(n_u: int, n_v: int, m: int, seed: int) -> Graph:
    """Uniformly random simple bipartite graph with exactly ``m`` edges.

    Pairs (u, v) are drawn with replacement in batches from one PCG64 stream;
    the first ``m`` distinct pairs in draw order are kept.
    """
    if m > n_u * n_v:
        raise ValueError("more edges than vertex pairs")
    rng = np.random.default_rng(seed)
    seen: dict[int, None] = {}
    while len(seen) < m:
        k = max(1024, 2 * (m - len(seen)))
        us = rng.integers(0, n_u, size=k, dtype=np.int64)
        vs = rng.integers(0, n_v, size=k, dtype=np.int64)
        for key in (us * n_v + vs).tolist():
            if key not in seen:
                seen[key] = None
                if len(seen) == m:
                    break
    key = np.fromiter(seen.keys(), dtype=np.int64, count=m)
    return _finish(n_u, n_v, key // n_v, key % n_v, f"uniform-{n_u}x{n_v}-{m}",
                   {"seed": seed})


def _pareto_weights(rng: np.random.Generator, n: int, beta: float) -> np.ndarray:
    # inverse-CDF draw of a Pareto(beta) variate with x_min = 1
    x = rng.random(n)
    return (1.0 - x) ** (-1.0 / (beta - 1.0))


def _clip_rescale(r: np.ndarray, m_t: float, cap: float) -> np.ndarray:
    w = r * (m_t / r.sum())
    for _ in range(20):
        np.minimum(w, cap, out=w)
        w *= m_t / w.sum()
    np.minimum(w, cap, out=w)
    return w


def _draw_endpoints(rng: np.random.Generator, w: np.ndarray, k: int) -> np.ndarray:
    c = np.cumsum(w)
    idx = np.searchsorted(c, rng.random(k) * c[-1], side="right")
    np.minimum(idx, w.shape[0] - 1, out=idx)
    return idx.astype(np.int64)


def chung_lu(n_u: int, n_v: int, m_t: int, beta_u: float, beta_v: float,
             seed: int, cap_u: float | None = None, cap_v: float | None = None,
             name: str = "") -> Graph:
    """Chung-Lu bipartite graph with Pareto expected degrees on both sides.

    Recipe: Pareto weights (U first, then V) from one PCG64 stream, scaled to
    sum ``m_t`` with 20 rounds of clip-to-cap and rescale (cap defaults to the
    size of the other side), then ``m_t`` endpoint draws per side by inverse
    CDF (all U draws, then all V draws), then duplicate pairs dropped.
    """
    rng = np.random.default_rng(seed)
    ru = _pareto_weights(rng, n_u, beta_u)
    rv = _pareto_weights(rng, n_v, beta_v)
    wu = _clip_rescale(ru, float(m_t), float(n_v if cap_u is None else cap_u))
    wv = _clip_rescale(rv, float(m_t), float(n_u if cap_v is None else cap_v))
    u = _draw_endpoints(rng, wu, int(m_t))
    v = _draw_endpoints(rng, wv, int(m_t))
    meta = {"seed": seed, "m_t": int(m_t), "beta_u": beta_u, "beta_v": beta_v,
            "cap_u": cap_u, "cap_v": cap_v}
    return _finish(n_u, n_v, u, v, name or f"chung-lu-{n_u}x{n_v}-{m_t}", meta)


def complete_bipartite(a: int, b: int) -> Graph:
    u, v = np.meshgrid(np.arange(a), np.arange(b), indexing="ij")
    return _finish(a, b, u.ravel(), v.ravel(), f"K{a},{b}")


def complete_minus_matching(n: int) -> Graph:
    u, v = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    keep = u != v
    return _finish(n, n, u[keep], v[keep], f"K{n},{n}-M")


def star(k: int, center_side: str = "u") -> Graph:
    if center_side == "u":
        return _finish(1, k, np.zeros(k, np.int64), np.arange(k), f"star-u{k}")
    return _finish(k, 1, np.arange(k), np.zeros(k, np.int64), f"star-v{k}")


def random_tree(n_u: int, n_v: int, seed: int) -> Graph:
    """A random spanning tree on n_u + n_v vertices (needs n_u, n_v >= 1).

    u0 and v0 are joined first; every other vertex, in a random order, is
    joined to a random already placed vertex of the other side.  A tree has
    no cycle, so it has no butterfly.
    """
    rng = np.random.default_rng(seed)
    us, vs = [0], [0]
    placed_u, placed_v = [0], [0]
    rest = [("u", i) for i in range(1, n_u)] + [("v", j) for j in range(1, n_v)]
    for k in rng.permutation(len(rest)).tolist():
        side, x = rest[k]
        if side == "u":
            us.append(x); vs.append(placed_v[int(rng.integers(0, len(placed_v)))])
            placed_u.append(x)
        else:
            vs.append(x); us.append(placed_u[int(rng.integers(0, len(placed_u)))])
            placed_v.append(x)
    return _finish(n_u, n_v, np.array(us, np.int64), np.array(vs, np.int64),
                   f"tree-{n_u}x{n_v}")


def tiny_random(n_u: int, n_v: int, p: float, seed: int) -> Graph:
    """Erdos-Renyi bipartite graph G(n_u, n_v, p) for brute-force checks."""
    rng = np.random.default_rng(seed)
    mask = rng.random((n_u, n_v)) < p
    u, v = np.nonzero(mask)
    return _finish(n_u, n_v, u, v, f"tiny-{n_u}x{n_v}-{p}-{seed}")


def disjoint_union(*gs: Graph) -> Graph:
    us, vs = [], []
    ou = ov = 0
    for g in gs:
        us.append(g.eu.astype(np.int64) + ou)
        vs.append(g.ev.astype(np.int64) + ov)
        ou += g.n_u
        ov += g.n_v
    u = np.concatenate(us) if us else np.zeros(0, np.int64)
    v = np.concatenate(vs) if vs else np.zeros(0, np.int64)
    return _finish(ou, ov, u, v, "+".join(g.name for g in gs))


def permute_ids(g: Graph, seed: int) -> tuple[Graph, np.ndarray, np.ndarray]:
    """Relabel both sides by random permutations; returns (graph, pu, pv)
    with new_id = p[old_id].  Edge order is shuffled too."""
    rng = np.random.default_rng(seed)
    pu = rng.permutation(g.n_u).astype(np.int64)
    pv = rng.permutation(g.n_v).astype(np.int64)
    order = rng.permutation(g.m)
    eu = pu[g.eu.astype(np.int64)][order].astype(np.int32)
    ev = pv[g.ev.astype(np.int64)][order].astype(np.int32)
    return Graph(g.n_u, g.n_v, eu, ev, g.name + "-perm", dict(g.meta)), pu, pv


def transpose(g: Graph) -> Graph:
    return _finish(g.n_v, g.n_u, g.ev, g.eu, g.name + "-T")


def graph_sha256(g: Graph) -> str:
    h = hashlib.sha256()
    h.update(np.array([g.n_u, g.n_v, g.m], np.int64).tobytes())
    h.update(np.ascontiguousarray(g.eu, np.int32).tobytes())
    h.update(np.ascontiguousarray(g.ev, np.int32).tobytes())
    return h.hexdigest()


# --------------------------------------------------------------------------
# The evaluated workloads.
# --------------------------------------------------------------------------

def config_graph(name: str) -> Graph:
    """Named workloads.

    ``plain-small``  uniform 2,000 x 1,000 with 20,000 distinct edges (seed 1)
    ``k30_20``       the complete bipartite graph K_{30,20}
    ``cl-10m``       Chung-Lu |U|=1e6, |V|=2e5, 1e7 draws, beta_U=2.5,
                     beta_V=2.1 capped at 5e4 (seed 2)
    ``cl-100m-skew`` Chung-Lu |U|=2e7, |V|=2e6, 1e8 draws, beta_U=2.3,
                     beta_V=1.9 capped at 5e5 (seed 4)
    ``cl-1m``        a 1e6-draw Chung-Lu graph with the cl-10m shape scaled
                     down tenfold (seed 12), used for quick checks
    """
    if name == "plain-small":
        return uniform_bipartite(2000, 1000, 20000, seed=1)
    if name == "k30_20":
        return complete_bipartite(30, 20)
    if name == "cl-10m":
        return chung_lu(1_000_000, 200_000, 10_000_000, 2.5, 2.1, seed=2,
                        cap_v=5e4, name="cl-10m")
    if name == "cl-1m":
        return chung_lu(100_000, 20_000, 1_000_000, 2.5, 2.1, seed=12,
                        cap_v=5e3, name="cl-1m")
    if name == "cl-100m-skew":
        return chung_lu(20_000_000, 2_000_000, 100_000_000, 2.3, 1.9, seed=4,
                        cap_v=5e5, name="cl-100m-skew")
    raise KeyError(name)


def batch_params(count: int = 64, seed_base: int = 3000,
                 m_lo: float = 1e4, m_hi: float = 2e6) -> list[dict]:
    """Parameters of the batched workload: graph g draws its shape from
    PCG64(seed_base + g): m_t log-uniform in [m_lo, m_hi], |U|:|V| ratio
    uniform in [1, 8], |U| = m_t / 10, exponents uniform in [2.0, 2.8]."""
    out = []
    for g in range(count):
        rng = np.random.default_rng(seed_base + g)
        m_t = int(round(math.exp(rng.uniform(math.log(m_lo), math.log(m_hi)))))
        ratio = float(rng.uniform(1.0, 8.0))
        n_u = max(2, int(round(m_t / 10)))
        n_v = max(2, int(round(n_u / ratio)))
        bu = float(rng.uniform(2.0, 2.8))
        bv = float(rng.uniform(2.0, 2.8))
        out.append({"m_t": m_t, "n_u": n_u, "n_v": n_v, "beta_u": bu,
                    "beta_v": bv, "seed": seed_base + g})
    return out


def batch_graph(p: dict) -> Graph:
    return chung_lu(p["n_u"], p["n_v"], p["m_t"], p["beta_u"], p["beta_v"],
                    seed=p["seed"] + 100_000, name=f"batch-{p['seed']}")


def serving_trace(rate: float = 20.0, duration: float = 120.0, seed: int = 5,
                  m_lo: float = 1e4, m_hi: float = 5e6,
                  job_seed_base: int = 5_000_000) -> list[dict]:
    """Poisson arrivals (exponential gaps, PCG64(seed)) of decomposition
    jobs; job j draws its shape from PCG64(job_seed_base + j)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        j = len(jobs)
        jr = np.random.default_rng(job_seed_base + j)
        m_t = int(round(math.exp(jr.uniform(math.log(m_lo), math.log(m_hi)))))
        side = int(jr.integers(0, 2))
        ratio = float(jr.uniform(1.0, 8.0))
        n_u = max(2, int(round(m_t / 10)))
        n_v = max(2, int(round(n_u / ratio)))
        jobs.append({"id": j, "arrival": t, "m_t": m_t, "side": side,
                     "n_u": n_u, "n_v": n_v,
                     "beta_u": float(jr.uniform(2.0, 2.6)),
                     "beta_v": float(jr.uniform(2.0, 2.6)),
                     "seed": job_seed_base + j})
    return jobs


def job_graph(job: dict) -> Graph:
    return chung_lu(job["n_u"], job["n_v"], job["m_t"], job["beta_u"],
                    job["beta_v"], seed=job["seed"] + 7, name=f"job-{job['id']}")
