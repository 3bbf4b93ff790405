#!/usr/bin/env python3
"""Benchmark of the tip-decomposition hot path on one MI355X.

One step = one full tip decomposition (ingest, per-vertex counting,
coarse-grained range peeling, fine-grained subset peeling, output scatter)
of the U side of the cl-10m workload (Chung-Lu |U| = 1e6, |V| = 2e5,
~9.76e6 distinct edges, V exponent 2.1 capped at 5e4, U exponent 2.5, P =
150), with the edge list already resident in HBM.  Reported value: wedges
traversed per second (counting + coarse + fine wedges / step time).

After the timed steps, one more step runs with kernel timing on: HIP events
on the launch stream around every launch of the dominant kernel give the
roofline figures (the timed steps themselves run uninstrumented, with the
coarse-grained rounds replayed from a HIP graph).

After the headline, two records are measured once each (skip them with
--no-extras): "large", the cl-100m-skew workload (|U| = 2e7, |V| = 2e6, ~9.1e7
edges), both sides, one warm-up and one timed run each; and "batch", the
64-graph batch decomposed in the batched form and as 64 plain decompositions,
checked against the oracle's stored digests.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
    python bench.py --steps 0          # only the instrumented step (counter runs)
    python bench.py --batch            # only the 64-graph batch record

Prints one JSON line.  Only one GPU is used; --gpus above 1 exits with a
message.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per unit of work of the peeling kernel: the int32 id of
# every 2-hop vertex read, the int32 id of every first-hop vertex read, and
# one int64 read-modify-write per support decrement.
BYTES_PER_WEDGE = 4
BYTES_PER_EDGE = 4
BYTES_PER_PAIR = 16
DOMINANT_KERNEL = "k_peel_dense"
KERNEL_SOURCES = ["paper_2010_08695_amd/csrc/peel.hip", "paper_2010_08695_amd/csrc/agg.h",
                  "paper_2010_08695_amd/csrc/tip_common.h"]


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(workload: str):
    """HBM traffic of the dominant kernel from committed rocprofv3 counter
    runs, or None when there are none for the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{DOMINANT_KERNEL}.{workload}.traffic.txt")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.loads(f.read().split("\n---\n")[0])
    except (ValueError, OSError):
        return None
    if rec.get("kernel_sha") != kernel_source_sha():
        return None
    return rec.get("bytes_per_launch")


def host_cpu_model() -> str:
    """The host CPU's model name from /proc/cpuinfo ("unknown" elsewhere)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(g, seconds: float) -> dict:
    """The oracle's 2-hop aggregation (the update step of bottom-up peeling)
    on random U vertices of the same graph, sized to ~`seconds` of CPU work."""
    import numpy as np

    import oracle
    oracle.build()
    dv = np.bincount(g.ev, minlength=g.n_v).astype(np.int64)
    per_u = np.zeros(g.n_u, np.int64)
    np.add.at(per_u, g.eu, dv[g.ev] - 1)
    order = np.random.default_rng(0).permutation(g.n_u).astype(np.int32)
    member = np.ones(g.n_u, np.uint8)
    t0 = time.perf_counter()
    oracle.support_in(g, 0, member, order[:0])
    t_build = time.perf_counter() - t0
    k = 64
    while True:
        t0 = time.perf_counter()
        oracle.support_in(g, 0, member, order[:k])
        dt = time.perf_counter() - t0 - t_build
        if dt > 0.5 or k >= g.n_u:
            break
        k = min(g.n_u, k * 4)
    rate = max(dt, 1e-9) / k
    k = int(min(g.n_u, max(k, seconds / rate)))
    t0 = time.perf_counter()
    oracle.support_in(g, 0, member, order[:k])
    dt = time.perf_counter() - t0 - t_build
    wedges = int(per_u[order[:k]].sum())
    return {"value": wedges / dt, "unit": "wedges/s", "cores": 1, "kind": "oracle",
            "host": {"cpu": host_cpu_model(), "nproc": os.cpu_count()},
            "sample": (f"oracle 2-hop aggregation (the update step of sequential bottom-up peeling) for {k} "
                       f"random U vertices of {g.name}: {wedges} wedges in {dt:.1f} s on one host core; "
                       f"adjacency build ({t_build:.1f} s) excluded; heap upkeep of the full oracle not "
                       f"included, so this overstates the full oracle's rate")}


def digest(a) -> str:
    import numpy as np
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i8").tobytes()).hexdigest()


def load_golden(name: str):
    path = os.path.join(ROOT, "tests", "golden", f"{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def full_oracle_record(workload: str, side: int):
    """The full oracle's run on the workload, as stored with its expected
    values (date, host CPU and cores used), or None."""
    rec = load_golden(workload)
    key = "theta_u" if side == 0 else "theta_v"
    if not rec or key not in rec or "seconds" not in rec[key]:
        return None
    host = rec.get("host", {})
    return {"seconds": rec[key]["seconds"], "peel_wedges": rec[key]["wedges"],
            "count_seconds": rec["count"].get("seconds"), "date": host.get("date"), "cpu": host.get("cpu"),
            "cores": host.get("cores_used", 1),
            "what": ("sequential bottom-up peeling of the whole side (initial count included) by the oracle, "
                     "timed when its expected values were written; not re-run by the benchmark")}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def batch_record(P: int, count: int = 64, steps: int = 1) -> dict:
    """64 Chung-Lu graphs (m log-uniform in [1e4, 2e6], |U|:|V| in [1, 8],
    exponents in [2.0, 2.8], U side): the batched forms against the plain
    form (one full decomposition after another), same API call, each once
    after a warm-up; checked against the oracle's stored per-graph digests."""
    import numpy as np

    from paper_2010_08695_amd import autotune, graphgen, tip
    params = graphgen.batch_params(count)
    graphs = [graphgen.batch_graph(p) for p in params]
    sides = [0] * len(graphs)
    tunes = autotune.batch_tunes(graphs, sides)
    res = {}
    # union: the batch as one disjoint-union decomposition (the default
    # batched form); streams: graphs on concurrent streams with their stored
    # tunings and one fine-grained launch; plain: one after another
    forms = (("union", 0, None), ("streams", tip.TIP_FLAG_BATCH_STREAMS, tunes),
             ("plain", tip.TIP_FLAG_BATCH_PLAIN, None))
    for name, flags, tn in forms:
        tip.decompose_batch(graphs, sides, P=P, flags=flags, tunes=tn)  # warm-up
        best, out, sts = None, None, None
        for _ in range(max(1, steps)):
            t0 = time.perf_counter()
            out, sts = tip.decompose_batch(graphs, sides, P=P, with_stats=True, flags=flags, tunes=tn)
            dt = time.perf_counter() - t0
            best = dt if best is None or dt < best else best
        res[name] = (best, out, sts)
        log(f"batch {name}: {best:.3f} s")
    same = all(np.array_equal(a, b) and np.array_equal(a, c)
               for a, b, c in zip(res["union"][1], res["streams"][1], res["plain"][1]))
    gold = load_golden(f"batch-{count}")
    golden_match = None
    if gold is not None and P == 150:
        golden_match = all(gr["graph_sha256"] == graphgen.graph_sha256(g) and
                           digest(th) == gr["theta_u"]["sha256"]
                           for gr, g, th in zip(gold["graphs"], graphs, res["union"][1]))
    sts = res["union"][2]
    wedges = sum(s["wedges_count"] + s["wedges_cd"] + s["wedges_fd"] for s in sts)
    return {"workload": f"batch-{len(graphs)}: Chung-Lu graphs, m log-uniform in [1e4, 2e6], "
                        f"sum m = {sum(g.m for g in graphs)}, side U, P={P}",
            "wedges_per_s": wedges / res["union"][0], "wedges": wedges,
            "batched_s": res["union"][0], "streams_s": res["streams"][0], "plain_s": res["plain"][0],
            "speedup_vs_plain": res["plain"][0] / res["union"][0],
            "same_results": same, "oracle_digests_match": golden_match,
            "streams_tuned_graphs": sum(1 for t in tunes if t is not None),
            "note": "host edge lists in, host tip numbers out (H2D/D2H and allocation included in both forms)"}


def bench_batch(args) -> int:
    rec = batch_record(args.P, args.batch_graphs, args.steps)
    out = {"metric": "wedges/s (batch of tip decompositions, bit-exact)", "value": rec["wedges_per_s"],
           "unit": "wedges/s", "n_gpus": 1, "steps": args.steps, "higher_is_better": True, "dtype": "int64",
           "data": "synthetic", "config": {"workload": rec["workload"]}, **rec}
    print(json.dumps(out))
    return 0


def large_record(P: int) -> dict:
    """cl-100m-skew, side V then side U, edges resident in HBM: one warm-up
    and one timed decomposition per side, with phase times, wedges and the
    wedge total of the graph; V's tip numbers checked against the oracle's
    stored digest (the oracle cannot finish U at this size)."""
    import numpy as np
    import torch

    from paper_2010_08695_amd import graphgen, tip
    t0 = time.perf_counter()
    g = graphgen.config_graph("cl-100m-skew")
    t_gen = time.perf_counter() - t0
    log(f"large graph generated in {t_gen:.1f} s (m = {g.m})")
    du = np.bincount(g.eu, minlength=g.n_u).astype(np.int64)
    dv = np.bincount(g.ev, minlength=g.n_v).astype(np.int64)
    wedge_total = int((du * (du - 1) // 2).sum() + (dv * (dv - 1) // 2).sum())
    dev = torch.device("cuda:0")
    d_eu = torch.from_numpy(g.eu).to(dev)
    d_ev = torch.from_numpy(g.ev).to(dev)
    gold = load_golden("cl-100m-skew")
    sides = {}
    for side in (1, 0):
        n_side = g.n_u if side == 0 else g.n_v
        ws = torch.empty(tip.workspace_size(g.n_u, g.n_v, g.m, side, P), dtype=torch.uint8, device=dev)
        d_theta = torch.empty(n_side, dtype=torch.int64, device=dev)
        stream = torch.cuda.current_stream()
        tip.decompose_async(d_eu, d_ev, g.n_u, g.n_v, side, d_theta, ws, stream, P=P)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = tip.decompose_async(d_eu, d_ev, g.n_u, g.n_v, side, d_theta, ws, stream, P=P)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        theta = d_theta.cpu().numpy()
        wedges = st["wedges_count"] + st["wedges_cd"] + st["wedges_fd"]
        key = "theta_u" if side == 0 else "theta_v"
        rec = {"seconds": dt, "wedges": wedges, "wedges_per_s": wedges / dt,
               "phase_ms": {k: st[k] for k in ("t_ingest_ms", "t_count_ms", "t_cd_ms", "t_fd_ms", "t_total_ms")},
               "rounds": st["rounds"], "subsets": st["subsets"], "theta_max": int(theta.max()),
               "bit_exact": (digest(theta) == gold[key]["sha256"]) if gold and key in gold else None}
        if rec["bit_exact"] is None:
            rec["parity"] = "unpinned at this size: the oracle's bottom-up peel of this side walks ~9e12 wedges"
        sides["UV"[side]] = rec
        log(f"large side {'UV'[side]}: {dt:.2f} s, bit_exact={rec['bit_exact']}")
        del ws, d_theta
        torch.cuda.empty_cache()
    return {"workload": f"cl-100m-skew: Chung-Lu |U|={g.n_u} |V|={g.n_v} m={g.m} P={P}",
            "wedge_total": wedge_total, "generate_s": t_gen, "sides": sides,
            "note": "edges resident in HBM; one warm-up, then one timed decomposition per side"}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cl-10m")
    ap.add_argument("--side", type=int, default=0)
    ap.add_argument("--P", type=int, default=150)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", action="store_true", help="only the 64-graph batch record")
    ap.add_argument("--batch-graphs", type=int, default=64)
    ap.add_argument("--no-extras", action="store_true", help="skip the large-graph and batch records")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); this build has no multi-GPU path",
              file=sys.stderr)
        return 2
    if args.batch:
        return bench_batch(args)

    import numpy as np
    import torch

    from paper_2010_08695_amd import graphgen, tip

    g = graphgen.config_graph(args.workload)
    dev = torch.device("cuda:0")
    d_eu = torch.from_numpy(g.eu).to(dev)
    d_ev = torch.from_numpy(g.ev).to(dev)
    n_side = g.n_u if args.side == 0 else g.n_v
    ws = torch.empty(tip.workspace_size(g.n_u, g.n_v, g.m, args.side, args.P), dtype=torch.uint8, device=dev)
    d_theta = torch.empty(n_side, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    def step(flags=0):
        return tip.decompose_async(d_eu, d_ev, g.n_u, g.n_v, args.side, d_theta, ws, stream, P=args.P,
                                   flags=flags)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    st = None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sec_per_step = elapsed / args.steps if args.steps > 0 else None
    # the last timed (graph-replayed) step's tip numbers, before the
    # instrumented step overwrites them
    theta_timed = d_theta.cpu().numpy() if args.steps > 0 else None
    log(f"{args.steps} timed steps: {elapsed:.3f} s")

    # one instrumented step: the dominant kernel's launches timed with HIP
    # events on the launch stream, its algorithmic bytes counted on the device
    ist = step(tip.TIP_FLAG_TIME_KERNELS)
    torch.cuda.synchronize()
    if st is None:
        st = ist
    wedges = st["wedges_count"] + st["wedges_cd"] + st["wedges_fd"]
    launches = ist["peel_launches"]
    peel_ms = ist["peel_ms"]
    alg_bytes = (BYTES_PER_WEDGE * ist["peel_wedges"] + BYTES_PER_EDGE * ist["peel_edges"] +
                 BYTES_PER_PAIR * ist["peel_pairs"])
    achieved = (alg_bytes / (peel_ms / 1e3)) / 1e9 if peel_ms > 0 else None
    traffic = load_traffic(args.workload)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
                "kernel": DOMINANT_KERNEL, "launches_per_step": launches,
                "mean_launch_ms": peel_ms / max(launches, 1),
                "alg_bytes_per_launch": alg_bytes / max(launches, 1),
                "kernel_share_of_step": (peel_ms / 1e3) / sec_per_step if sec_per_step else None}

    # bit-exactness of the timed step and of the instrumented one against
    # the oracle's stored digest
    theta_inst = d_theta.cpu().numpy()
    bit_exact = bit_exact_inst = None
    rec = load_golden(args.workload)
    key = "theta_u" if args.side == 0 else "theta_v"
    if rec and key in rec:
        if theta_timed is not None:
            bit_exact = digest(theta_timed) == rec[key]["sha256"]
        bit_exact_inst = digest(theta_inst) == rec[key]["sha256"]

    out = {
        "metric": "wedges/s (full tip decomposition, bit-exact)",
        "value": wedges / sec_per_step if sec_per_step else None,
        "unit": "wedges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec_per_step * 1e3 if sec_per_step else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: Chung-Lu |U|={g.n_u} |V|={g.n_v} m={g.m} "
                               f"side={'U' if args.side == 0 else 'V'} P={args.P}",
                   "n_u": g.n_u, "n_v": g.n_v, "m": g.m, "side": args.side, "P": args.P},
        "bit_exact": bit_exact,
        "bit_exact_instrumented_step": bit_exact_inst,
        "wedges": {"count": st["wedges_count"], "cd": st["wedges_cd"], "fd": st["wedges_fd"]},
        "phase_ms": {k: st[k] for k in ("t_ingest_ms", "t_count_ms", "t_cd_ms", "t_fd_ms", "t_total_ms")},
        "rounds": st["rounds"], "subsets": st["subsets"], "pair_updates": st["pair_updates"],
        "spills": st["spills"],
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, args.cpu_seconds)
        full = full_oracle_record(args.workload, args.side)
        if full:
            full["gpu_speedup"] = full["seconds"] / sec_per_step if sec_per_step else None
            out["cpu_baseline"]["full_oracle"] = full
        log("cpu baseline done")
    if not args.no_extras:
        del ws
        torch.cuda.empty_cache()
        out["large"] = large_record(args.P)
        out["batch"] = batch_record(args.P)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
