"""Full serving-trace check (not collected by pytest; run on an MI355X):

    python tests/serve_trace_check.py [--duration 120] [--oracle-sample 24]

Replays the seeded serving trace (Poisson, 20 jobs/s, Chung-Lu graphs with
m log-uniform in [1e4, 5e6], random side) with continuous batching and with
a FIFO one-job-at-a-time loop, and checks that every job's tip numbers are
identical in both loops (tolerance 0) and, for a seeded sample of jobs,
equal to the CPU oracle's sequential bottom-up peel.  Prints one JSON line
with p50/p99 latency and throughput of both loops.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2010_08695_amd import serve  # noqa: E402


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--duration", type=float, default=120.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--oracle-sample", type=int, default=24)
    args = ap.parse_args(argv)
    t0 = time.time()

    def log(msg):
        print(f"[{time.time() - t0:7.1f}s] {msg}", file=sys.stderr, flush=True)

    out, jobs, mixed = serve.run_trace(args.rate, args.duration, 5e6, args.slots, 64.0, True, None, log=log)
    # a seeded sample: the smaller half of a random pick, so the CPU oracle
    # finishes in minutes
    rng = np.random.default_rng(11)
    pick = rng.choice(len(jobs), size=min(len(jobs), 2 * args.oracle_sample), replace=False)
    pick = sorted(pick, key=lambda i: jobs[i].graph.m)[:args.oracle_sample]
    equal = 0
    for n, i in enumerate(pick):
        j = jobs[i]
        equal += int(mixed[j.id] is not None and np.array_equal(oracle.bup(j.graph, j.side)[0], mixed[j.id]))
        log(f"oracle {n + 1}/{len(pick)}: job {j.id} m={j.graph.m}")
    out["oracle_sample"] = {"jobs": len(pick), "equal": equal, "largest_m": int(max(jobs[i].graph.m for i in pick))}
    print(json.dumps(out))
    return 0 if out.get("same_results") and equal == len(pick) else 1


if __name__ == "__main__":
    sys.exit(main())
