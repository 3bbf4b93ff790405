"""Autotuner for libtip's run-time tunables (tip_opts.tune).

Which setting is fastest depends on the graph's size and degree
distribution, so the tuner times full decompositions of a representative
graph and keeps the fastest.  The search is staged (coordinate descent):

1. the coarse-grained update-kernel selection: tune[0] = D, the divisor of
   the dense-kernel threshold (a vertex goes to the dense key-range kernel
   with its LDS counter table only when its wedges exceed n_side * bits / D),
   and tune[1], the largest wedge count handled by the bitmap kernel with its
   LDS bitmap and repeat table;
2. the fine-grained step's work queue (its help board, with stage 1's winner
   fixed): tune[4] updates taken per claim of a queue slot and tune[5] the
   fewest per-wave updates of a level worth publishing.

Every trial must give the same tip numbers (any setting is exact; a mismatch
is a library error and aborts the tuning).  Winners are stored per device
name and graph size class.  Lookups read the user's cache first, then the
table that ships with the package (``tuning.json``, written on an MI355X by
``--batch``).

    python -m paper_2010_08695_amd.autotune --workload cl-1m [--side 0]
    python -m paper_2010_08695_amd.autotune --batch 64 --out tuning.json
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

STAGES = [
    {"dense_div": (0, [256, 512, 1024, 2048]), "bitmap_max": (1, [1024, 2048, 4096, 8192])},
    {"help_chunk": (4, [8, 16, 32, 64]), "help_level_min": (5, [128, 256, 512])},
]
N_TUNE = 8
CACHE = os.path.join(os.path.expanduser("~"), ".cache", "libtip_autotune.json")
TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


def size_class(n_u: int, n_v: int, m: int, side: int) -> str:
    """Graphs within a factor of ~2 in every size share a tuning."""
    def b(x):
        return int(round(math.log2(max(int(x), 1))))
    return f"side{side}-u{b(n_u)}-v{b(n_v)}-m{b(m)}"


def choose(trials: list[dict]) -> dict:
    """The fastest trial (best time); ties go to the earlier grid point."""
    if not trials:
        raise ValueError("no trials")
    best = min(range(len(trials)), key=lambda i: (trials[i]["ms"], i))
    return trials[best]


def _grid(stage: dict, base: list[int]) -> list[list[int]]:
    points = [list(base)]
    for _name, (idx, values) in stage.items():
        nxt = []
        for p in points:
            for v in values:
                q = list(p)
                q[idx] = v
                nxt.append(q)
        points = nxt
    return points


def tune_graph(g, side: int = 0, stages: list | None = None, reps: int = 3, P: int = 0, timer=None) -> dict:
    """Times the staged grid on graph g; returns {"tune": [...8 ints], "ms":
    ..., "trials": [...]}.  timer(g, side, tune) -> (theta, ms) can replace
    the library call (tests)."""
    stages = STAGES if stages is None else stages

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
    base = [0] * N_TUNE
    win = None
    for stage in stages:
        stage_trials = []
        for point in _grid(stage, base):
            th, ms = timer(g, side, point)
            if ref is None:
                ref = th
            elif not np.array_equal(ref, th):
                raise RuntimeError(f"tip numbers differ between tunings ({point}): library error")
            stage_trials.append({"tune": point, "ms": float(ms)})
        win = choose(stage_trials)
        base = list(win["tune"])
        trials += stage_trials
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


def _key(g, side: int, device: str | None = None) -> str:
    return f"{device or device_name()}|{size_class(g.n_u, g.n_v, g.m, side)}"


def lookup(g, side: int, path: str | None = CACHE, table: str | None = TABLE, device: str | None = None):
    """Stored tune list for graphs of g's size class on this device (the
    user's cache first, then the package table), or None."""
    key = _key(g, side, device)
    for p in (path, table):
        if p is None:
            continue
        rec = load_cache(p).get(key)
        if rec:
            t = list(rec["tune"]) + [0] * N_TUNE
            return t[:N_TUNE]
    return None


def batch_tunes(graphs, sides, path: str | None = CACHE, table: str | None = TABLE):
    """Per-graph tune lists (None where nothing is stored) for
    tip.decompose_batch(..., tunes=...)."""
    dev = device_name()
    return [lookup(g, s, path, table, dev) for g, s in zip(graphs, sides)]


def store(g, side: int, result: dict, path: str = CACHE, device: str | None = None) -> None:
    cache = load_cache(path)
    cache[_key(g, side, device)] = {"tune": list(result["tune"]), "ms": result["ms"]}
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--workload", default="cl-1m")
    ap.add_argument("--side", type=int, default=0)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--batch", type=int, default=0, help="tune one graph per size class of the N-graph batch")
    ap.add_argument("--out", default=CACHE)
    args = ap.parse_args(argv)
    if args.batch:
        graphs = [graphgen.batch_graph(p) for p in graphgen.batch_params(args.batch)]
        seen = {}
        for g in graphs:
            seen.setdefault(size_class(g.n_u, g.n_v, g.m, 0), g)
        for cls, g in sorted(seen.items()):
            res = tune_graph(g, 0, reps=args.reps)
            store(g, 0, res, args.out)
            dflt = [t["ms"] for t in res["trials"] if t["tune"][:2] == [1024, 2048] and not any(t["tune"][2:])]
            print(json.dumps({"class": cls, "graph": g.name, "tune": res["tune"], "ms": res["ms"],
                              "default_ms": dflt[0] if dflt else None}), flush=True)
        return 0
    g = graphgen.config_graph(args.workload)
    res = tune_graph(g, args.side, reps=args.reps)
    store(g, args.side, res, args.out)
    print(json.dumps({"workload": args.workload, "side": args.side, "device": device_name(), **res}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
