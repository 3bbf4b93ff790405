"""Writes the stored expected values under tests/golden/ from the CPU oracle.

Every value here comes from ``oracle`` (or a closed form in the paper's
notation) and nothing else.  Large outputs are stored as SHA-256 digests of
the little-endian int64 arrays plus a deterministic sample of entries, so that
the GPU tests can check full-size results exactly without re-running a
minutes-long oracle.

    python tests/golden/make_golden.py plain-small cl-1m cl-10m
"""
from __future__ import annotations

import hashlib
import json
import os
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


def make(name: str, sides=(0, 1)) -> dict:
    g = graphgen.config_graph(name)
    rec = {"config": name, "graph_sha256": graphgen.graph_sha256(g),
           "n_u": g.n_u, "n_v": g.n_v, "m": g.m, "source": "oracle/tip_oracle.cpp"}
    t0 = time.time()
    bu, bv, tot = oracle.count(g)
    rec["count"] = {"total": tot, "sum_u": int(bu.sum()), "sum_v": int(bv.sum()),
                    "sha256_u": digest(bu), "sha256_v": digest(bv),
                    "sample_u": sample(bu, seed=1), "sample_v": sample(bv, seed=2),
                    "seconds": round(time.time() - t0, 2)}
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


def main(argv):
    names = argv or ["plain-small", "cl-1m"]
    for name in names:
        rec = make(name)
        path = os.path.join(HERE, f"{name}.json")
        with open(path, "w") as f:
            json.dump(rec, f, indent=1)
        print("wrote", path, flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
