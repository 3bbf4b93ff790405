"""Autotuner for libtip's update-kernel selection thresholds.

The coarse-grained update kernels are chosen per vertex by two thresholds
(tip_opts.tune): tune[0] = D, the divisor of the dense-kernel threshold
(a vertex goes to the dense key-range kernel only when its wedges exceed
n_side * bits / D), and tune[1] = the largest wedge count handled by the
bitmap kernel.  Which setting is fastest depends on the degree distribution,
so the tuner times full decompositions of a representative graph over a
small grid of settings.  Every trial must give the same tip numbers (any
setting is exact; a mismatch is a library error and aborts the tuning).  The
winner is cached in a JSON file keyed by device name and graph size class.

    python -m paper_2010_08695_amd.autotune --workload cl-1m [--side 0]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import graphgen, tip

DEFAULT_GRID = {"dense_div": [256, 512, 1024, 2048], "bitmap_max": [1024, 2048, 4096, 8192]}
CACHE = os.path.join(os.path.expanduser("~"), ".cache", "libtip_autotune.json")


def size_class(n_u: int, n_v: int, m: int, side: int) -> str:
    """Graphs within a factor of ~2 in every size share a tuning."""
    def b(x):
        return int(round(math.log2(max(int(x), 1))))
    return f"side{side}-u{b(n_u)}-v{b(n_v)}-m{b(m)}"


def choose(trials: list[dict]) -> dict:
    """The fastest trial (median time); ties go to the earlier grid point."""
    if not trials:
        raise ValueError("no trials")
    best = min(range(len(trials)), key=lambda i: (trials[i]["ms"], i))
    return trials[best]


def tune_graph(g, side: int = 0, grid: dict | None = None, reps: int = 3, P: int = 0, timer=None) -> dict:
    """Times every grid point on graph g; returns {"tune": [D, bm], "ms": ...,
    "trials": [...]}.  timer(g, side, tune) -> (theta, ms) can replace the
    library call (tests)."""
    grid = grid or DEFAULT_GRID

    def lib_timer(g, side, tune):
        best, th = None, None
        for _ in range(reps):
            t0 = time.perf_counter()
            th = tip.decompose(g, side, P=P, tune=tune)
            dt = (time.perf_counter() - t0) * 1e3
            best = dt if best is None or dt < best else best
        return th, best

    timer = timer or lib_timer
    ref = None
    trials = []
    for d in grid["dense_div"]:
        for bm in grid["bitmap_max"]:
            th, ms = timer(g, side, [d, bm])
            if ref is None:
                ref = th
            elif not np.array_equal(ref, th):
                raise RuntimeError(f"tip numbers differ between tunings ({d}, {bm}): library error")
            trials.append({"tune": [d, bm], "ms": float(ms)})
    win = choose(trials)
    return {"tune": win["tune"], "ms": win["ms"], "trials": trials}


def device_name() -> str:
    try:
        import torch
        return torch.cuda.get_device_name(0)
    except Exception:  # noqa: BLE001 - any failure means "unknown device"
        return "unknown"


def load_cache(path: str = CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(g, side: int, path: str = CACHE):
    """Cached tune list for graphs of g's size class on this device, or None."""
    key = f"{device_name()}|{size_class(g.n_u, g.n_v, g.m, side)}"
    rec = load_cache(path).get(key)
    return rec["tune"] if rec else None


def store(g, side: int, result: dict, path: str = CACHE) -> None:
    cache = load_cache(path)
    cache[f"{device_name()}|{size_class(g.n_u, g.n_v, g.m, side)}"] = {"tune": result["tune"], "ms": result["ms"]}
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--workload", default="cl-1m")
    ap.add_argument("--side", type=int, default=0)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--cache", default=CACHE)
    args = ap.parse_args(argv)
    g = graphgen.config_graph(args.workload)
    res = tune_graph(g, args.side, reps=args.reps)
    store(g, args.side, res, args.cache)
    print(json.dumps({"workload": args.workload, "side": args.side, "device": device_name(), **res}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
