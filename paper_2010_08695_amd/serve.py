"""Serving loop: continuous batching of tip-decomposition jobs on one GPU.

Jobs arrive over time (a seeded Poisson trace of Chung-Lu graphs).  A job
is admitted, in arrival order, as soon as an execution slot is free and its
device footprint (libtip workspace + edge list + theta, from
``tip_workspace_size``) fits under the HBM budget next to the jobs already
running.  Every admitted job runs ``tip_decompose_async`` on a stream of its
own, so the kernels of different jobs overlap on the device, and all of a
job's state (CSR/CSC, counts, supports) stays resident in its workspace from
ingest to the final tip numbers.  The comparison is a FIFO loop that runs
one job at a time on the same trace.

    python -m paper_2010_08695_amd.serve [--duration 20] [--rate 20] [--slots 4]

prints one JSON line with p50/p99 latency (completion - arrival) and
throughput for both loops.
"""
from __future__ import annotations

import argparse
import collections
import json
import sys
import threading
import time
from concurrent.futures import FIRST_COMPLETED, ThreadPoolExecutor, wait
from dataclasses import dataclass, field

import numpy as np

from . import graphgen, tip

GIB = 1 << 30


@dataclass
class Job:
    id: int
    arrival: float          # seconds after the start of the trace
    graph: graphgen.Graph
    side: int
    footprint: int = 0      # device bytes while running
    t_admit: float = -1.0
    t_done: float = -1.0
    theta: np.ndarray | None = None
    wedges: int = 0
    P: int = 0              # coarse-grained ranges (0 = the library default)
    status: str = "pending"  # "ok", "failed" (the executor raised) or "rejected" (waited too long)
    error: str = ""

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


class Admission:
    """Slots and an HBM budget.  Jobs are taken strictly in arrival order: a
    job that does not fit waits for running jobs to finish, and the jobs
    behind it wait too (no starvation of large jobs)."""

    def __init__(self, budget_bytes: int, slots: int):
        if slots < 1:
            raise ValueError("slots must be >= 1")
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.used = 0
        self.running = 0

    def fits(self, job: Job) -> bool:
        if job.footprint > self.budget:
            raise ValueError(f"job {job.id} needs {job.footprint} bytes, more than the whole budget")
        return self.running < self.slots and self.used + job.footprint <= self.budget

    def admit(self, job: Job) -> None:
        assert self.fits(job)
        self.used += job.footprint
        self.running += 1

    def release(self, job: Job) -> None:
        self.used -= job.footprint
        self.running -= 1
        assert self.used >= 0 and self.running >= 0


# Ranges of the coarse-grained step per job, by the job's wedge work
# W = sum over the other side of d(d - 1): below 5e7 wedges, 16 ranges;
# below 5e9, 40; else the paper's 150.  Results do not depend on P (any P
# gives the same tip numbers); small graphs pay mostly per-range host
# round trips, large ones need fine ranges to keep the fine-grained subsets
# short (measured on MI355X over the first 40 jobs of the serving trace:
# 1.95 s of device time at P = 150 for all, 1.50 s at P = 40 for all).
P_RULE = ((5e7, 16), (5e9, 40))
P_LARGE = 150


def wedge_work(g: graphgen.Graph, side: int) -> int:
    """sum over the other side of d(d - 1): the wedges bottom-up peeling of
    `side` would walk."""
    other = g.ev if side == tip.SIDE_U else g.eu
    d = np.bincount(other, minlength=g.n_v if side == tip.SIDE_U else g.n_u).astype(np.int64)
    return int((d * (d - 1)).sum())


def choose_P(g: graphgen.Graph, side: int) -> int:
    w = wedge_work(g, side)
    for limit, P in P_RULE:
        if w < limit:
            return P
    return P_LARGE


def footprint(g: graphgen.Graph, side: int, P: int = 0) -> int:
    """Device bytes of one job: libtip workspace + both edge arrays + theta."""
    n_side = g.n_u if side == tip.SIDE_U else g.n_v
    return tip.workspace_size(g.n_u, g.n_v, g.m, side, P) + 8 * g.m + 8 * n_side + 4096


def make_jobs(trace: list[dict], P: int | None = None, workers: int = 8) -> list[Job]:
    """Generates every job's graph (host side, seeded) before the replay.
    P: ranges for every job, or None to choose them per job (choose_P)."""
    def build(rec):
        g = graphgen.job_graph(rec)
        j = Job(rec["id"], rec["arrival"], g, rec["side"])
        j.P = choose_P(g, j.side) if P is None else P
        j.footprint = footprint(g, j.side, j.P)
        return j
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(build, trace))


class Executor:
    """Runs one job on a given stream: H2D edges, tip_decompose_async, D2H
    theta.  Device memory comes from torch's allocator on that stream."""

    def __init__(self, device: str = "cuda:0"):
        import torch
        self.torch = torch
        self.dev = torch.device(device)

    def __call__(self, job: Job, stream) -> None:
        torch = self.torch
        g = job.graph
        with torch.cuda.stream(stream):
            d_eu = torch.from_numpy(np.ascontiguousarray(g.eu, np.int32)).to(self.dev)
            d_ev = torch.from_numpy(np.ascontiguousarray(g.ev, np.int32)).to(self.dev)
            n_side = g.n_u if job.side == tip.SIDE_U else g.n_v
            d_theta = torch.empty(max(n_side, 1), dtype=torch.int64, device=self.dev)
            ws = torch.empty(tip.workspace_size(g.n_u, g.n_v, g.m, job.side, job.P), dtype=torch.uint8,
                             device=self.dev)
            st = tip.decompose_async(d_eu, d_ev, g.n_u, g.n_v, job.side, d_theta, ws, stream, P=job.P)
            job.theta = d_theta[:n_side].cpu().numpy()
            job.wedges = st["wedges_count"] + st["wedges_cd"] + st["wedges_fd"]
            del d_eu, d_ev, d_theta, ws
        stream.synchronize()


def replay(jobs: list[Job], run_job, slots: int, budget_bytes: int, streams=None,
           max_wait_s: float | None = None, progress=None) -> dict:
    """Replays the trace in real time.  run_job(job, stream) executes one job
    (blocking); up to `slots` run at once.  A job whose executor raises is
    recorded as failed (its error kept on the job) and its slot, memory and
    stream are released; the replay goes on.  With `max_wait_s`, a job still
    waiting for admission that long after its arrival is rejected without
    running.  Returns the summary."""
    for j in jobs:
        j.t_admit = j.t_done = -1.0
        j.status, j.error = "pending", ""
    adm = Admission(budget_bytes, slots)
    pending = collections.deque(sorted(jobs, key=lambda j: (j.arrival, j.id)))
    waiting: collections.deque[Job] = collections.deque()
    free_streams = list(streams) if streams is not None else [None] * slots
    running = {}
    lock = threading.Lock()
    t0 = time.perf_counter()

    def now() -> float:
        return time.perf_counter() - t0

    def task(job, stream):
        try:
            run_job(job, stream)
            job.status = "ok"
        except Exception as e:  # noqa: BLE001 - a job's failure is recorded, not fatal to the loop
            job.status, job.error = "failed", f"{type(e).__name__}: {e}"
        finally:
            with lock:
                job.t_done = now()

    next_report = 10.0
    with ThreadPoolExecutor(slots) as pool:
        while pending or waiting or running:
            t = now()
            if progress is not None and t >= next_report:
                next_report += 10.0
                progress(t, sum(1 for j in jobs if j.status != "pending"))
            while pending and pending[0].arrival <= t:
                waiting.append(pending.popleft())
            if max_wait_s is not None:
                while waiting and t - waiting[0].arrival > max_wait_s:
                    job = waiting.popleft()
                    job.status, job.t_done = "rejected", t
            while waiting and adm.fits(waiting[0]):
                job = waiting.popleft()
                adm.admit(job)
                job.t_admit = now()
                stream = free_streams.pop()
                running[pool.submit(task, job, stream)] = (job, stream)
            timeout = None
            if pending:
                timeout = max(0.0, pending[0].arrival - now())
            if progress is not None:
                timeout = min(timeout, 5.0) if timeout is not None else 5.0
            if running:
                done, _ = wait(list(running), timeout=timeout, return_when=FIRST_COMPLETED)
                for f in done:
                    job, stream = running.pop(f)
                    adm.release(job)
                    free_streams.append(stream)
            elif timeout:
                time.sleep(timeout)
    return summarize(jobs)


def summarize(jobs: list[Job]) -> dict:
    """Latency percentiles and throughput over the jobs that completed;
    failed and rejected jobs are counted, with the first errors."""
    ok = [j for j in jobs if j.status == "ok"]
    failed = [j for j in jobs if j.status == "failed"]
    rejected = [j for j in jobs if j.status == "rejected"]
    out = {"jobs": len(jobs), "completed": len(ok), "failed": len(failed), "rejected": len(rejected),
           "errors": [f"job {j.id}: {j.error}" for j in failed[:5]]}
    if not ok:
        return out
    lat = np.array([j.latency for j in ok])
    end = max(j.t_done for j in jobs)
    start = min(j.arrival for j in jobs)
    wedges = sum(j.wedges for j in ok)
    out.update({"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                "mean_s": float(lat.mean()), "makespan_s": end - start, "jobs_per_s": len(ok) / (end - start),
                "wedges_per_s": wedges / (end - start), "edges": int(sum(j.graph.m for j in ok))})
    return out


def run_trace(rate: float = 20.0, duration: float = 20.0, m_hi: float = 5e6, slots: int = 4,
              budget_gib: float = 64.0, fifo: bool = True, P: int | None = None, log=None):
    """Replays a seeded Poisson trace with continuous batching and, unless
    fifo is False, again one job at a time.  Returns (summary, jobs,
    tip numbers of every job in the continuous replay)."""
    import torch

    def say(msg):
        if log is not None:
            log(msg)

    trace = graphgen.serving_trace(rate=rate, duration=duration, m_hi=m_hi)
    say(f"generating {len(trace)} jobs")
    t_gen = time.perf_counter()
    jobs = make_jobs(trace, P=P, workers=16)
    say(f"generated in {time.perf_counter() - t_gen:.1f} s")
    ex = Executor()
    warm = graphgen.job_graph(trace[0])
    ex(Job(-1, 0.0, warm, 0, P=choose_P(warm, 0)), torch.cuda.Stream())
    budget = int(budget_gib * GIB)
    streams = [torch.cuda.Stream() for _ in range(slots)]
    prog = (lambda t, n: say(f"  {t:6.1f} s: {n} jobs finished")) if log is not None else None
    say("continuous batching replay")
    cont = replay(jobs, ex, slots, budget, streams, progress=prog)
    thetas = {j.id: j.theta for j in jobs}
    out = {"trace": {"rate": rate, "duration": duration, "jobs": len(jobs), "m_hi": m_hi,
                     "edges": int(sum(j.graph.m for j in jobs))},
           "slots": slots, "budget_gib": budget_gib,
           "P": "per job (serve.choose_P)" if P is None else P, "continuous": cont}
    if fifo:
        say("FIFO one-at-a-time replay")
        f = replay(jobs, ex, 1, budget, streams[:1], progress=prog)
        out["fifo"] = f
        out["same_results"] = all(thetas[j.id] is not None and np.array_equal(thetas[j.id], j.theta) for j in jobs)
        if "p99_s" in f and "p99_s" in cont:
            out["p99_speedup_vs_fifo"] = f["p99_s"] / cont["p99_s"]
            out["throughput_vs_fifo"] = cont["jobs_per_s"] / f["jobs_per_s"]
    return out, jobs, thetas


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--duration", type=float, default=20.0)
    ap.add_argument("--m-hi", type=float, default=5e6)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--budget-gib", type=float, default=64.0)
    ap.add_argument("--no-fifo", action="store_true")
    ap.add_argument("--P", type=int, default=None, help="ranges for every job (default: chosen per job)")
    args = ap.parse_args(argv)
    out, _jobs, _thetas = run_trace(args.rate, args.duration, args.m_hi, args.slots, args.budget_gib,
                                    not args.no_fifo, args.P,
                                    log=lambda m: print(m, file=sys.stderr, flush=True))
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
