"""Writes the stored expected values under tests/golden/ from the CPU oracle.

Every value here comes from ``oracle`` (or a closed form in the paper's
notation) and nothing else.  Large outputs are stored as SHA-256 digests of
the little-endian int64 arrays plus a deterministic sample of entries, so that
the GPU tests can check full-size results exactly without re-running a
minutes-long oracle.

    python tests/golden/make_golden.py plain-small cl-1m cl-10m
    python tests/golden/make_golden.py batch-64 [--procs 6]
    python tests/golden/make_golden.py cl-100m-skew     # V side only
    python tests/golden/make_golden.py cl-1m-wing       # per-edge counts and wing numbers of cl-1m

``batch-64`` holds one record per graph of the 64-graph batch workload (U
side), computed in parallel, one oracle per process.  ``cl-100m-skew``
holds the V side only: the oracle's U side walks about 9e12 wedges there,
far beyond what the CPU can do.  Every timing is stored with the date, the
host's CPU model and the number of cores the oracle used (one).
"""
from __future__ import annotations

import argparse
import datetime
import hashlib
import json
import multiprocessing
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2010_08695_amd import graphgen  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i8").tobytes()).hexdigest()


def sample(a: np.ndarray, k: int = 64, seed: int = 0) -> dict:
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(a.shape[0], size=min(k, a.shape[0]), replace=False))
    return {"index": idx.tolist(), "value": a[idx].tolist()}


def host() -> dict:
    """Where and when the oracle ran: date, CPU model, cores it used."""
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"date": datetime.date.today().isoformat(), "cpu": cpu, "machine": platform.machine(),
            "nproc": os.cpu_count(), "cores_used": 1}


def make(name: str, sides=(0, 1), g=None) -> dict:
    g = g if g is not None else graphgen.config_graph(name)
    rec = {"config": name, "graph_sha256": graphgen.graph_sha256(g),
           "n_u": g.n_u, "n_v": g.n_v, "m": g.m, "source": "oracle/tip_oracle.cpp", "host": host()}
    t0 = time.time()
    if tuple(sides) == (0, 1):
        bu, bv, tot = oracle.count(g)
        rec["count"] = {"total": tot, "sum_u": int(bu.sum()), "sum_v": int(bv.sum()),
                        "sha256_u": digest(bu), "sha256_v": digest(bv),
                        "sample_u": sample(bu, seed=1), "sample_v": sample(bv, seed=2)}
    else:
        # one side only: its counts, and the total they imply
        rec["count"] = {}
        for side in sides:
            b = oracle.count_side(g, side)
            k = "uv"[side]
            rec["count"].update({f"sum_{k}": int(b.sum()), f"sha256_{k}": digest(b),
                                 f"sample_{k}": sample(b, seed=1 + side)})
            rec["count"]["total"] = int(b.sum()) // 2
    rec["count"]["seconds"] = round(time.time() - t0, 2)
    print(name, "count", rec["count"]["seconds"], "s", flush=True)
    for side in sides:
        t0 = time.time()
        th, _order, wedges = oracle.bup(g, side)
        key = "theta_u" if side == 0 else "theta_v"
        vals, cnts = np.unique(th, return_counts=True)
        rec[key] = {"sha256": digest(th), "max": int(th.max()) if th.size else 0,
                    "sum": int(th.sum()), "nonzero": int((th > 0).sum()),
                    "distinct": int(vals.shape[0]), "wedges": wedges,
                    "sample": sample(th, seed=3 + side),
                    "seconds": round(time.time() - t0, 2)}
        if g.n_u + g.n_v <= 5000:
            rec[key]["values"] = th.tolist()
        print(name, key, rec[key]["seconds"], "s", flush=True)
    return rec


def make_wing(name: str) -> dict:
    """Per-edge butterfly counts and wing numbers of a workload's edges, in
    canonical order (duplicates merged, sorted by (u, v))."""
    g = graphgen.config_graph(name)
    rec = {"config": f"{name}-wing", "graph_sha256": graphgen.graph_sha256(g), "n_u": g.n_u, "n_v": g.n_v,
           "m": g.m, "source": "oracle/wing_oracle.cpp", "host": host(), "order": "canonical (u, v)"}
    t0 = time.time()
    c = oracle.edge_count(g)
    rec["edge_count"] = {"sha256": digest(c), "sum": int(c.sum()), "max": int(c.max()) if c.size else 0,
                         "sample": sample(c, seed=5), "seconds": round(time.time() - t0, 2)}
    print(name, "edge counts", rec["edge_count"]["seconds"], "s", flush=True)
    t0 = time.time()
    psi, _order, pairs = oracle.wing(g)
    vals = np.unique(psi)
    rec["wing"] = {"sha256": digest(psi), "max": int(psi.max()) if psi.size else 0, "sum": int(psi.sum()),
                   "distinct": int(vals.shape[0]), "pairs": pairs, "sample": sample(psi, seed=6),
                   "seconds": round(time.time() - t0, 2)}
    print(name, "wing", rec["wing"]["seconds"], "s", flush=True)
    return rec


def _batch_one(p: dict) -> dict:
    g = graphgen.batch_graph(p)
    rec = make(g.name, sides=(0,), g=g)
    rec["params"] = p
    return rec


def make_batch(count: int, procs: int) -> dict:
    params = graphgen.batch_params(count)
    # largest graphs first, so the pool's tail is short
    order = sorted(range(count), key=lambda i: -params[i]["m_t"])
    with multiprocessing.Pool(procs) as pool:
        recs = pool.map(_batch_one, [params[i] for i in order], chunksize=1)
    graphs = [None] * count
    for i, r in zip(order, recs):
        graphs[i] = r
    return {"config": f"batch-{count}", "source": "oracle/tip_oracle.cpp", "host": host(),
            "graphs": graphs}


def main(argv):
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*", default=["plain-small", "cl-1m"])
    ap.add_argument("--procs", type=int, default=6)
    args = ap.parse_args(argv)
    for name in args.names:
        if name.startswith("batch-"):
            rec = make_batch(int(name.split("-")[1]), args.procs)
        elif name.endswith("-wing"):
            rec = make_wing(name[:-len("-wing")])
        elif name == "cl-100m-skew":
            rec = make(name, sides=(1,))
        else:
            rec = make(name)
        path = os.path.join(HERE, f"{name}.json")
        with open(path, "w") as f:
            json.dump(rec, f, indent=1)
        print("wrote", path, flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
