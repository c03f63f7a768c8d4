"""Serving policy on the CPU: a fake executor and a fake clock.

The fake device runs each job's chunks one after another (chunk time
proportional to cells x steps) while different jobs overlap freely, which is
what the per-job streams give on the GPU.
"""

import numpy as np
import pytest

from paper_2205_02774_amd.abi import E_UNSTABLE, StglbmError
from paper_2205_02774_amd.serve import Server, summarize, JobResult


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def advance(self, dt=1e-3):
        self.t += dt


class FakeExecutor:
    def __init__(self, clock, rate=1e9, fail_ids=()):
        self.clock = clock
        self.rate = rate
        self.fail_ids = set(fail_ids)
        self.started = []
        self.live = 0
        self.max_live = 0

    def footprint(self, job):
        return job["bytes"]

    def start(self, job):
        self.started.append(job["id"])
        self.live += 1
        self.max_live = max(self.max_live, self.live)
        return {"job": job, "busy_until": self.clock(), "steps": 0}

    def submit(self, h, n):
        if h["job"]["id"] in self.fail_ids and h["steps"] > 0:
            raise StglbmError(E_UNSTABLE, "forced instability")
        start = max(self.clock(), h["busy_until"])
        h["busy_until"] = start + h["job"]["cfg"]["cells"] * n / self.rate
        h["steps"] += n
        return h["busy_until"]

    def done(self, token):
        return self.clock() >= token

    def finish(self, h):
        self.live -= 1
        return "ok", np.full((2, 2, 9), float(h["steps"])), h["steps"], ""


def _jobs(n, rng, cells=(1_000_000, 4_000_000), steps=(100, 2000), nbytes=(1, 5)):
    out = []
    t = 0.0
    for i in range(n):
        out.append({"id": i, "arrival_s": t, "steps": int(rng.integers(*steps)),
                    "bytes": int(rng.integers(*nbytes)) * 2 ** 30,
                    "cfg": {"cells": int(rng.integers(*cells))}})
        t += float(rng.exponential(0.5))
    return out


def _serve(jobs, budget, max_active=4, chunk=100, fail_ids=()):
    clock = FakeClock()
    ex = FakeExecutor(clock, fail_ids=fail_ids)
    srv = Server(budget, max_active=max_active, chunk_steps=chunk, executor=ex, clock=clock, idle=clock.advance)
    res, summ = srv.run(jobs)
    return srv, ex, res, summ


def test_admission_respects_budget_and_slots():
    rng = np.random.default_rng(0)
    jobs = _jobs(40, rng)
    srv, ex, res, summ = _serve(jobs, budget=8 * 2 ** 30, max_active=3)
    assert srv.peak_bytes <= 8 * 2 ** 30
    assert ex.max_live <= 3 and srv.peak_active <= 3
    assert summ["jobs"] == 40 and summ["ok"] == 40
    # first come, first served
    assert ex.started == [j["id"] for j in sorted(jobs, key=lambda j: j["arrival_s"])]
    for r in res:
        assert r.n_samples == r.steps
        assert r.arrival_s <= r.admitted_s <= r.finished_s


def test_jobs_overlap_and_latency_percentiles():
    rng = np.random.default_rng(1)
    jobs = _jobs(30, rng)
    _, ex, res, summ = _serve(jobs, budget=64 * 2 ** 30, max_active=8)
    assert ex.max_live > 1               # concurrent jobs
    lat = np.array([r.latency_s for r in res])
    assert summ["p50_latency_s"] == pytest.approx(np.percentile(lat, 50))
    assert summ["p99_latency_s"] == pytest.approx(np.percentile(lat, 99))
    work = sum(r.cells * r.steps for r in res)
    assert summ["aggregate_mlups"] == pytest.approx(work / summ["makespan_s"] / 1e6)


def test_waiting_jobs_admitted_as_memory_frees():
    # a big job holds most of the budget; small ones queue until it finishes
    jobs = [{"id": 0, "arrival_s": 0.0, "steps": 1000, "bytes": 7 * 2 ** 30, "cfg": {"cells": 10_000_000}}]
    jobs += [{"id": i, "arrival_s": 0.01 * i, "steps": 100, "bytes": 2 * 2 ** 30, "cfg": {"cells": 1_000_000}}
             for i in range(1, 5)]
    srv, ex, res, summ = _serve(jobs, budget=8 * 2 ** 30, max_active=4)
    big = res[0]
    for r in res[1:]:
        assert r.admitted_s >= big.finished_s - 1e-9
    assert srv.peak_bytes <= 8 * 2 ** 30


def test_unstable_job_is_reported_and_released():
    rng = np.random.default_rng(2)
    jobs = _jobs(10, rng)
    _, ex, res, summ = _serve(jobs, budget=16 * 2 ** 30, fail_ids=(3,))
    assert res[3].status == "unstable" and "forced instability" in res[3].message
    assert summ["unstable"] == 1 and summ["ok"] == 9
    assert ex.live == 0


def test_oversized_job_rejected():
    jobs = [{"id": 0, "arrival_s": 0.0, "steps": 10, "bytes": 9 * 2 ** 30, "cfg": {"cells": 10}}]
    with pytest.raises(ValueError):
        _serve(jobs, budget=8 * 2 ** 30)


def test_summary_arithmetic():
    res = [JobResult(i, 0.0, 0.0, float(i + 1), 1000, 10, "ok") for i in range(100)]
    s = summarize(res, 100.0)
    assert s["p50_latency_s"] == pytest.approx(50.5)
    assert s["p99_latency_s"] == pytest.approx(99.01)
    assert s["aggregate_mlups"] == pytest.approx(100 * 1000 * 10 / 100.0 / 1e6)
