"""Helpers for rocprofv3 measurements of libtip kernels.

    # plain copy of a known size, the calibration for FETCH_SIZE / WRITE_SIZE
    python -m paper_2010_08695_amd.profiling calib [--mib 1024]
    # short text summary of a --kernel-trace --stats run
    python -m paper_2010_08695_amd.profiling stats <dir> --cmd "<command>" --out profiles/x.txt
    # per-launch HBM traffic of one kernel from two counter runs + calibration
    python -m paper_2010_08695_amd.profiling traffic --fetch <dir> --write <dir> \\
        --calib-fetch <dir> --calib-write <dir> --kernel k_peel_big --workload cl-10m --cmd "..."
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ["paper_2010_08695_amd/csrc/peel.hip", "paper_2010_08695_amd/csrc/agg.h",
                  "paper_2010_08695_amd/csrc/tip_common.h"]


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def find_csv(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[-1]


def short_name(name: str) -> str:
    # demangled names look like "tip::(anonymous namespace)::k_peel_big(...)"
    base = name.replace("(anonymous namespace)", "anon").split("(")[0]
    return base.split("::")[-1] if "::" in base else base


def kernel_stats(d: str) -> list[dict]:
    rows = []
    with open(find_csv(d, "kernel_stats.csv")) as f:
        for r in csv.DictReader(f):
            rows.append({"name": short_name(r["Name"]), "calls": int(r["Calls"]),
                         "total_ns": float(r["TotalDurationNs"]), "avg_ns": float(r["AverageNs"]),
                         "pct": float(r["Percentage"]), "min_ns": float(r["MinNs"]),
                         "max_ns": float(r["MaxNs"])})
    rows.sort(key=lambda r: -r["total_ns"])
    return rows


def counter_per_dispatch(d: str, counter: str) -> dict[str, list[float]]:
    """{kernel short name: [counter value per dispatch]} (values summed over
    the per-XCD/per-instance rows of one dispatch)."""
    per: dict[tuple, float] = {}
    names: dict[tuple, str] = {}
    with open(find_csv(d, "counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if r.get("Counter_Name") != counter:
                continue
            key = (r.get("Dispatch_Id") or r.get("Correlation_Id"), r.get("Kernel_Name"))
            per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
            names[key] = short_name(r.get("Kernel_Name", ""))
    out: dict[str, list[float]] = {}
    for k, v in per.items():
        out.setdefault(names[k], []).append(v)
    return out


def cmd_calib(args) -> int:
    import torch
    n = args.mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {args.mib} MiB", flush=True)
    return 0


def cmd_stats(args) -> int:
    rows = kernel_stats(args.dir)
    lines = [f"# rocprofv3 kernel statistics", f"command: {args.cmd}", "",
             f"{'kernel':<28}{'calls':>8}{'total ms':>12}{'avg us':>12}{'min us':>10}{'max us':>10}{'%':>7}"]
    for r in rows[: args.top]:
        lines.append(f"{r['name']:<28}{r['calls']:>8}{r['total_ns'] / 1e6:>12.3f}{r['avg_ns'] / 1e3:>12.2f}"
                     f"{r['min_ns'] / 1e3:>10.2f}{r['max_ns'] / 1e3:>10.2f}{r['pct']:>7.2f}")
    text = "\n".join(lines) + "\n"
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    print(text)
    return 0


def cmd_traffic(args) -> int:
    fetch = counter_per_dispatch(args.fetch, "FETCH_SIZE")
    write = counter_per_dispatch(args.write, "WRITE_SIZE")
    cf = counter_per_dispatch(args.calib_fetch, "FETCH_SIZE")
    cw = counter_per_dispatch(args.calib_write, "WRITE_SIZE")
    copy_bytes = args.calib_mib * (1 << 20)
    # the calibration copy is the dispatch with the largest reading
    cf_kib = max(v for vs in cf.values() for v in vs)
    cw_kib = max(v for vs in cw.values() for v in vs)
    f_scale = copy_bytes / (cf_kib * 1024.0)
    w_scale = copy_bytes / (cw_kib * 1024.0)
    kf = fetch.get(args.kernel, [])
    kw = write.get(args.kernel, [])
    if not kf or not kw:
        raise SystemExit(f"kernel {args.kernel} not found in the counter runs")
    mean_f = sum(kf) / len(kf)
    mean_w = sum(kw) / len(kw)
    per_launch = mean_f * 1024.0 * f_scale + mean_w * 1024.0 * w_scale
    rec = {"kernel": args.kernel, "workload": args.workload, "kernel_sha": kernel_source_sha(),
           "dispatches": len(kf), "fetch_kib_per_dispatch": mean_f, "write_kib_per_dispatch": mean_w,
           "fetch_scale": f_scale, "write_scale": w_scale, "bytes_per_launch": per_launch}
    text = (json.dumps(rec) + "\n---\n"
            f"HBM traffic of {args.kernel} on {args.workload} (rocprofv3 --pmc, one counter per run)\n"
            f"command: {args.cmd}\n"
            f"calibration: plain copy of {args.calib_mib} MiB read FETCH_SIZE {cf_kib:.0f} KiB and WRITE_SIZE "
            f"{cw_kib:.0f} KiB -> scale {f_scale:.4f} / {w_scale:.4f}\n"
            f"{args.kernel}: {len(kf)} dispatches, mean FETCH_SIZE {mean_f:.1f} KiB, mean WRITE_SIZE "
            f"{mean_w:.1f} KiB -> {per_launch / 1e6:.3f} MB per launch after scaling\n")
    out = args.out or os.path.join(ROOT, "profiles", f"{args.kernel}.{args.workload}.traffic.txt")
    with open(out, "w") as f:
        f.write(text)
    print(text)
    return 0


LDS_PEAK_TBS = 128 * 256 * 2.4e9 / 1e12   # 128 B per clock per CU, 256 CUs, 2.4 GHz
LDS_CONFLICT_COUNTERS = ["SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE", "SQ_INSTS_LDS", "SQ_ACTIVE_INST_LDS",
                         "SQ_WAVE_CYCLES", "SQ_BUSY_CU_CYCLES", "GRBM_GUI_ACTIVE"]
LDS_BYTE_COUNTERS = ["SQ_INSTS_LDS_LOAD_BANDWIDTH", "SQ_INSTS_LDS_STORE_BANDWIDTH", "SQ_INSTS_LDS_ATOMIC_BANDWIDTH",
                     "SQ_INSTS_LDS_ATOMIC"]


def cmd_lds(args) -> int:
    """LDS bank conflicts and LDS bytes of the top kernels from two counter
    runs of the same program, with kernel times from a trace of it."""
    va = {c: counter_per_dispatch(args.conflicts, c) for c in LDS_CONFLICT_COUNTERS}
    vb = {c: counter_per_dispatch(args.bytes, c) for c in LDS_BYTE_COUNTERS}
    times = {r["name"]: r["total_ns"] for r in kernel_stats(args.trace)}
    lines = [f"# LDS bank conflicts and LDS traffic per kernel ({args.workload})",
             f"command: {args.cmd}", "",
             "conflict rate = SQ_LDS_BANK_CONFLICT / (SQ_LDS_IDX_ACTIVE - SQ_LDS_BANK_CONFLICT) (stall cycles per",
             "conflict-free LDS cycle); LDS share of wave time = SQ_ACTIVE_INST_LDS / SQ_WAVE_CYCLES; LDS bytes =",
             "64 x (SQ_INSTS_LDS_LOAD_BANDWIDTH + _STORE_ + _ATOMIC_) over the kernel's time in the trace;",
             f"LDS peak {LDS_PEAK_TBS:.1f} TB/s (128 B per clock per CU, 256 CUs, 2.4 GHz)", "",
             f"{'kernel':<18}{'disp':>6}{'LDS instr':>12}{'conflict rate':>15}{'LDS share':>11}"
             f"{'LDS GB':>9}{'ms':>9}{'LDS TB/s':>10}{'of peak':>9}"]
    for k in args.kernels.split(","):
        tot = {c: sum(va[c].get(k, [])) for c in LDS_CONFLICT_COUNTERS}
        tb = {c: sum(vb[c].get(k, [])) for c in LDS_BYTE_COUNTERS}
        n = len(va["SQ_LDS_IDX_ACTIVE"].get(k, []))
        if n == 0:
            continue
        bc, idx = tot["SQ_LDS_BANK_CONFLICT"], tot["SQ_LDS_IDX_ACTIVE"]
        rate = bc / (idx - bc) if idx > bc else float("nan")
        share = tot["SQ_ACTIVE_INST_LDS"] / tot["SQ_WAVE_CYCLES"] if tot["SQ_WAVE_CYCLES"] else float("nan")
        lds_bytes = 64.0 * (tb["SQ_INSTS_LDS_LOAD_BANDWIDTH"] + tb["SQ_INSTS_LDS_STORE_BANDWIDTH"] +
                            tb["SQ_INSTS_LDS_ATOMIC_BANDWIDTH"])
        ms = times.get(k, 0.0) / 1e6
        tbs = lds_bytes / (ms / 1e3) / 1e12 if ms > 0 else float("nan")
        lines.append(f"{k:<18}{n:>6}{tot['SQ_INSTS_LDS']:>12.4g}{rate:>15.3f}{share:>11.3f}"
                     f"{lds_bytes / 1e9:>9.2f}{ms:>9.2f}{tbs:>10.2f}{tbs / LDS_PEAK_TBS:>9.1%}")
    text = "\n".join(lines) + "\n"
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    print(text)
    return 0


WAVE_COUNTERS = ["SQ_WAVE_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_ANY", "SQ_ACTIVE_INST_VALU",
                 "SQ_ACTIVE_INST_LDS", "SQ_WAVES", "SQ_BUSY_CYCLES"]


def cmd_waves(args) -> int:
    """Where the waves of the top kernels spend their resident cycles, from
    one counter run: waiting on memory or a barrier (SQ_WAIT_ANY), ready but
    not issued (SQ_WAIT_INST_ANY), issuing (SQ_ACTIVE_INST_ANY, of which VALU
    and LDS)."""
    v = {c: counter_per_dispatch(args.dir, c) for c in WAVE_COUNTERS}
    lines = [f"# wave states per kernel ({args.workload})", f"command: {args.cmd}", "",
             "shares of the waves' resident cycles (SQ_WAVE_CYCLES): waiting for memory, LDS or a barrier",
             "(SQ_WAIT_ANY), ready but not selected to issue (SQ_WAIT_INST_ANY), issuing any instruction",
             "(SQ_ACTIVE_INST_ANY), of which VALU and LDS instructions", "",
             f"{'kernel':<18}{'disp':>6}{'waves':>10}{'wait mem/bar':>14}{'wait issue':>12}{'issuing':>9}"
             f"{'VALU':>7}{'LDS':>7}"]
    for k in args.kernels.split(","):
        tot = {c: sum(v[c].get(k, [])) for c in WAVE_COUNTERS}
        n = len(v["SQ_WAVE_CYCLES"].get(k, []))
        wc = tot["SQ_WAVE_CYCLES"]
        if n == 0 or wc <= 0:
            continue
        lines.append(f"{k:<18}{n:>6}{tot['SQ_WAVES']:>10.3g}{tot['SQ_WAIT_ANY'] / wc:>14.3f}"
                     f"{tot['SQ_WAIT_INST_ANY'] / wc:>12.3f}{tot['SQ_ACTIVE_INST_ANY'] / wc:>9.3f}"
                     f"{tot['SQ_ACTIVE_INST_VALU'] / wc:>7.3f}{tot['SQ_ACTIVE_INST_LDS'] / wc:>7.3f}")
    text = "\n".join(lines) + "\n"
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    print(text)
    return 0


def cmd_launch(args) -> int:
    """rocprofv3's average launch time of one kernel next to the figure the
    bench line reports for it (HIP events on the launch stream)."""
    st = {r["name"]: r for r in kernel_stats(args.dir)}.get(args.kernel)
    if st is None:
        raise SystemExit(f"kernel {args.kernel} not in {args.dir}")
    bench = None
    with open(args.bench_log) as f:
        for line in f:
            line = line.strip()
            if line.startswith("{") and '"roofline"' in line:
                bench = json.loads(line)
    if bench is None:
        raise SystemExit(f"no bench line in {args.bench_log}")
    rf = bench["roofline"]
    mean_us = round(rf["mean_launch_ms"] * 1e3, 1) if rf.get("mean_launch_ms") else None
    lines = [f"# {args.kernel} on {args.workload}: rocprofv3 average launch time vs the bench's HIP-event figure",
             f"command: {args.cmd}", "",
             f"rocprofv3: {args.kernel} {st['calls']} dispatches, total {st['total_ns'] / 1e6:.2f} ms, average "
             f"{st['avg_ns'] / 1e3:.1f} us (min {st['min_ns'] / 1e3:.1f}, max {st['max_ns'] / 1e3:.1f})",
             f"bench.py (HIP events on the launch stream, same run): mean {mean_us} us per launch" if mean_us
             else "bench.py: no per-launch time in its line",
             f"bench roofline: achieved {rf['achieved']:.1f} {rf['unit']} of {rf['peak']} -> frac {rf['frac']:.4f}"]
    if rf.get("alg_bytes_per_launch"):
        ab = rf["alg_bytes_per_launch"]
        ach = ab / (st["avg_ns"] / 1e9) / 1e9
        lines.append(f"algorithmic bytes per launch {ab / 1e6:.1f} MB / rocprofv3 average {st['avg_ns'] / 1e3:.1f} us "
                     f"-> {ach:.1f} GB/s = {ach / 8000.0:.1%} of 8 TB/s")
        tf = os.path.join(ROOT, "profiles", f"{args.kernel}.{args.workload}.traffic.txt")
        if os.path.exists(tf):
            with open(tf) as f:
                tr = json.loads(f.readline())
            lines.append(f"HBM traffic ({os.path.basename(tf)}): {tr['bytes_per_launch'] / 1e6:.1f} MB per launch, "
                         f"{tr['bytes_per_launch'] / ab:.2f}x the algorithmic bytes")
    text = "\n".join(lines) + "\n"
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    print(text)
    return 0


def cmd_fdtrace(args) -> int:
    """Critical path of one fine-grained launch from the tip-fd-task lines a
    TIP_TRACE_FD=1 run prints (kernel timing on): the tasks that end last,
    with their levels and time per level."""
    import re
    pat = re.compile(r"tip-fd-task task=(\d+) n=(\d+) levels=(\d+) start_us=([\d.]+) end_us=([\d.]+)")
    runs, cur = [], []
    with open(args.log) as f:
        for line in f:
            m = pat.search(line)
            if m:
                t = int(m.group(1))
                if t == 0 and cur:
                    runs.append(cur)
                    cur = []
                cur.append((t, int(m.group(2)), int(m.group(3)), float(m.group(4)), float(m.group(5))))
    if cur:
        runs.append(cur)
    if not runs:
        raise SystemExit(f"no tip-fd-task lines in {args.log}")
    tasks = runs[-1]
    span = max(e for *_, e in tasks)
    lines = [f"# fine-grained launch ({args.workload}): per-task times and the critical path", f"command: {args.cmd}", "",
             f"{len(tasks)} tasks (subsets); launch span {span / 1e3:.2f} ms (first task start to last task end)",
             f"levels: {sum(t[2] for t in tasks)} in all, at most {max(t[2] for t in tasks)} in one subset", "",
             "tasks ending last (subset size, levels, start, end, time per level):"]
    for t, n, lv, s0, e in sorted(tasks, key=lambda x: -x[4])[: args.top]:
        lines.append(f"  task {t:4d}  n_i {n:7d}  levels {lv:5d}  start {s0 / 1e3:7.3f} ms  end {e / 1e3:7.3f} ms  "
                     f"{(e - s0) / max(lv, 1):7.1f} us/level")
    text = "\n".join(lines) + "\n"
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    print(text)
    return 0


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    p = sub.add_parser("calib")
    p.add_argument("--mib", type=int, default=1024)
    p.set_defaults(fn=cmd_calib)
    p = sub.add_parser("stats")
    p.add_argument("dir")
    p.add_argument("--cmd", default="")
    p.add_argument("--out", default="")
    p.add_argument("--top", type=int, default=25)
    p.set_defaults(fn=cmd_stats)
    p = sub.add_parser("traffic")
    for k in ("fetch", "write", "calib_fetch", "calib_write"):
        p.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    p.add_argument("--calib-mib", type=int, default=1024)
    p.add_argument("--kernel", default="k_peel_big")
    p.add_argument("--workload", default="cl-10m")
    p.add_argument("--cmd", default="")
    p.add_argument("--out", default="")
    p.set_defaults(fn=cmd_traffic)
    p = sub.add_parser("lds")
    p.add_argument("--conflicts", required=True, help="counter run of LDS_CONFLICT_COUNTERS")
    p.add_argument("--bytes", required=True, help="counter run of LDS_BYTE_COUNTERS")
    p.add_argument("--trace", required=True, help="kernel-trace run of the same program")
    p.add_argument("--kernels", default="k_peel_dense,k_fd_peel,k_count_big,k_peel_bitmap,k_count_small,k_peel_wave")
    p.add_argument("--workload", default="cl-10m")
    p.add_argument("--cmd", default="")
    p.add_argument("--out", default="")
    p.set_defaults(fn=cmd_lds)
    p = sub.add_parser("waves")
    p.add_argument("dir")
    p.add_argument("--kernels", default="k_peel_dense,k_fd_peel,k_count_big,k_frontier_scan,k_peel_bitmap")
    p.add_argument("--workload", default="cl-10m")
    p.add_argument("--cmd", default="")
    p.add_argument("--out", default="")
    p.set_defaults(fn=cmd_waves)
    p = sub.add_parser("launch")
    p.add_argument("dir")
    p.add_argument("--bench-log", required=True)
    p.add_argument("--kernel", default="k_peel_dense")
    p.add_argument("--workload", default="cl-10m")
    p.add_argument("--cmd", default="")
    p.add_argument("--out", default="")
    p.set_defaults(fn=cmd_launch)
    p = sub.add_parser("fdtrace")
    p.add_argument("log")
    p.add_argument("--workload", default="cl-10m")
    p.add_argument("--top", type=int, default=12)
    p.add_argument("--cmd", default="")
    p.add_argument("--out", default="")
    p.set_defaults(fn=cmd_fdtrace)
    args = ap.parse_args(argv)
    return args.fn(args)


if __name__ == "__main__":
    sys.exit(main())
