"""Serving loop: admission and replay logic on the CPU; results alone vs in the
mix on the GPU."""
from __future__ import annotations

import threading
import time

import numpy as np
import pytest

import oracle
from paper_2010_08695_amd import graphgen as gg
from paper_2010_08695_amd import serve


def _job(i, arrival, fp, m=10):
    g = gg.Graph(2, 2, np.zeros(m, np.int32), np.zeros(m, np.int32), f"j{i}")
    return serve.Job(i, arrival, g, 0, footprint=fp)


def test_admission_budget_and_slots():
    a = serve.Admission(100, 2)
    j1, j2, j3 = _job(1, 0, 60), _job(2, 0, 30), _job(3, 0, 20)
    assert a.fits(j1)
    a.admit(j1)
    assert a.fits(j2)
    a.admit(j2)
    assert not a.fits(j3)          # both slots busy
    a.release(j2)
    assert a.fits(j3)
    big = _job(4, 0, 50)
    assert not a.fits(big)         # 60 + 50 > 100
    a.release(j1)
    assert a.fits(big)
    with pytest.raises(ValueError):
        a.fits(_job(5, 0, 101))    # can never fit


def test_replay_respects_slots_budget_and_order():
    """Fake executor: records concurrency and memory in use; every job must
    start no earlier than it arrives, in arrival order."""
    jobs = [_job(i, 0.01 * i, fp) for i, fp in enumerate([40, 40, 40, 10, 70, 10, 10, 30])]
    state = {"run": 0, "mem": 0, "max_run": 0, "max_mem": 0, "starts": []}
    lock = threading.Lock()

    def run(job, stream):
        with lock:
            state["run"] += 1
            state["mem"] += job.footprint
            state["max_run"] = max(state["max_run"], state["run"])
            state["max_mem"] = max(state["max_mem"], state["mem"])
            state["starts"].append(job.id)
        time.sleep(0.03)
        job.wedges = 1
        with lock:
            state["run"] -= 1
            state["mem"] -= job.footprint

    s = serve.replay(jobs, run, slots=3, budget_bytes=100)
    assert state["max_run"] <= 3 and state["max_mem"] <= 100
    admits = [j.t_admit for j in sorted(jobs, key=lambda j: j.arrival)]
    assert admits == sorted(admits)                       # admitted in arrival order
    for j in jobs:
        assert j.t_admit >= j.arrival - 1e-3 and j.t_done >= j.t_admit
    assert s["jobs"] == len(jobs) and s["p99_s"] >= s["p50_s"] > 0


def test_fifo_is_one_at_a_time():
    jobs = [_job(i, 0.0, 1) for i in range(5)]
    seen = {"run": 0, "max": 0}
    lock = threading.Lock()

    def run(job, stream):
        with lock:
            seen["run"] += 1
            seen["max"] = max(seen["max"], seen["run"])
        time.sleep(0.01)
        with lock:
            seen["run"] -= 1

    serve.replay(jobs, run, slots=1, budget_bytes=10)
    assert seen["max"] == 1


@pytest.mark.gpu
def test_results_alone_equal_results_in_the_mix(gpu_lib):
    """Every job's tip numbers are the same when it runs alone and when it
    overlaps other jobs on the device (tolerance 0), and equal the oracle's."""
    import torch
    trace = gg.serving_trace(rate=40.0, duration=0.5, m_lo=2e3, m_hi=3e4)
    jobs = serve.make_jobs(trace)
    ex = serve.Executor()
    streams = [torch.cuda.Stream() for _ in range(4)]
    serve.replay(jobs, ex, 4, 8 << 30, streams)
    mixed = {j.id: j.theta.copy() for j in jobs}
    serve.replay(jobs, ex, 1, 8 << 30, streams[:1])
    for j in jobs:
        np.testing.assert_array_equal(mixed[j.id], j.theta)
        np.testing.assert_array_equal(j.theta, oracle.bup(j.graph, j.side)[0])


def test_failed_job_releases_its_slot_and_the_loop_goes_on():
    """A job whose executor raises is recorded as failed; its slot, memory and
    stream are released, and the jobs behind it are still admitted and
    finish."""
    jobs = [_job(i, 0.005 * i, 60) for i in range(6)]
    streams = ["s0", "s1"]
    used = []

    def run(job, stream):
        used.append(stream)
        time.sleep(0.01)
        if job.id in (1, 4):
            raise RuntimeError(f"device error in job {job.id}")
        job.wedges = 5

    s = serve.replay(jobs, run, slots=2, budget_bytes=100, streams=streams)
    assert [j.status for j in jobs] == ["ok", "failed", "ok", "ok", "failed", "ok"]
    assert "device error in job 1" in jobs[1].error
    assert s["completed"] == 4 and s["failed"] == 2 and s["rejected"] == 0
    assert len(s["errors"]) == 2 and s["jobs_per_s"] > 0
    assert set(used) <= set(streams) and len(used) == 6
    # a 60-byte job at a time under a 100-byte budget: never two at once,
    # so the failed jobs must have released their memory for later ones
    assert all(j.t_done >= j.t_admit >= 0 for j in jobs)


def test_jobs_waiting_too_long_are_rejected():
    jobs = [_job(i, 0.0, 10) for i in range(4)]

    def run(job, stream):
        time.sleep(0.05)
        job.wedges = 1

    s = serve.replay(jobs, run, slots=1, budget_bytes=100, max_wait_s=0.07)
    assert s["completed"] >= 2 and s["rejected"] >= 1
    assert s["completed"] + s["rejected"] == 4
    assert all(j.status in ("ok", "rejected") for j in jobs)
