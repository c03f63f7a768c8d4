"""Continuous batching of STG-LBM jobs on one device.

Jobs (channel configurations with a step budget) arrive over time.  A job is
admitted, first come first served, when a slot is free and its exact device
footprint (`stglbm_footprint`) fits in the remaining memory budget; it then
keeps its lattice resident in its own workspace and runs on its own HIP
stream.  The loop hands every active job its next chunk of steps as soon as
one of its two enqueued chunks has drained, so the kernels of different jobs
overlap on the device, and it admits waiting jobs as soon as a finishing job
returns its memory.  Each finished job yields its FP64 statistics; the loop
reports completion latencies and aggregate MLUPS.

A job's numerical result does not depend on the mix: its kernels touch only
its own workspace and the statistics reductions have a fixed order.

The policy (`Server`) is separate from the execution (`DeviceExecutor`) so
the scheduling can be exercised with a fake executor and clock.
"""

import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class JobResult:
    job_id: int
    arrival_s: float
    admitted_s: float
    finished_s: float
    cells: int
    steps: int
    status: str                   # "ok" or "unstable"
    stats: object = None          # (NX, NY, 9) FP64 sums over the job's steps
    n_samples: int = 0
    message: str = ""

    @property
    def latency_s(self):
        return self.finished_s - self.arrival_s


@dataclass
class _Active:
    job: dict
    handle: object
    remaining: int
    admitted_s: float
    inflight: list = field(default_factory=list)
    failed: str = ""


class DeviceExecutor:
    """Runs jobs through libstglbm: one workspace and one HIP stream per job."""

    def __init__(self, device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)

    def footprint(self, job):
        from .lattice import derive_units, footprint, make_desc
        cfg = job["cfg"]
        rans = cfg["rans"]
        _, _, nu_lb = derive_units(cfg["delta"], cfg["ny"], cfg["u_b_lb"], rans["U_b"], cfg["nu_phys"])
        d = make_desc(cfg["nx"], cfg["ny"], cfg["nz"], nu_lb=nu_lb, store=cfg["store"],
                      sponge_cells=cfg["sponge_cells"], max_modes=cfg["n_modes"], max_rans=len(rans["y"]))
        return footprint(d)

    def start(self, job):
        from .lattice import channel_from_config
        torch = self.torch
        stream = torch.cuda.Stream(device=self.device)
        with torch.cuda.stream(stream):
            lat = channel_from_config(job["cfg"], device=self.device, stream=stream)
            lat.stats_reset()
        return (lat, stream)

    def submit(self, handle, n):
        """Enqueue n steps; returns a completion token, or raises StglbmError."""
        lat, stream = handle
        lat.step(n)
        ev = self.torch.cuda.Event()
        ev.record(stream)
        return ev

    def done(self, token):
        return token.query()

    def finish(self, handle):
        """(status, stats, n_samples, message) after the stream drains; frees the job."""
        from . import abi
        lat, stream = handle
        try:
            stats, ns = lat.get_stats()
            out = ("ok", stats, ns, "")
        except abi.StglbmError as e:
            out = ("unstable", None, 0, str(e))
        lat.close()
        return out


class Server:
    """Admission by footprint, per-job streams, chunked round-robin stepping."""

    def __init__(self, budget_bytes, max_active=16, chunk_steps=500, executor=None, clock=None, idle=None,
                 inflight_per_job=2):
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.chunk = int(chunk_steps)
        self.executor = executor if executor is not None else DeviceExecutor()
        self.clock = clock or time.perf_counter
        self.idle = idle or (lambda: time.sleep(2e-4))
        self.depth = int(inflight_per_job)

    def run(self, jobs):
        """Serve jobs (dicts with 'id', 'arrival_s', 'steps', 'cfg'); returns (results, summary)."""
        from .abi import StglbmError
        ex = self.executor
        pending = sorted(jobs, key=lambda j: (j["arrival_s"], j["id"]))
        need = {}
        for j in pending:
            need[j["id"]] = ex.footprint(j)
            if need[j["id"]] > self.budget:
                raise ValueError(f"job {j['id']} needs {need[j['id']]} B, more than the budget {self.budget}")
        waiting, active, results = [], [], []
        used = 0
        self.peak_bytes = 0
        self.peak_active = 0
        t0 = self.clock()
        while pending or waiting or active:
            now = self.clock() - t0
            while pending and pending[0]["arrival_s"] <= now:
                waiting.append(pending.pop(0))
            while waiting and len(active) < self.max_active and used + need[waiting[0]["id"]] <= self.budget:
                job = waiting.pop(0)
                used += need[job["id"]]
                active.append(_Active(job=job, handle=ex.start(job), remaining=int(job["steps"]),
                                      admitted_s=self.clock() - t0))
            self.peak_bytes = max(self.peak_bytes, used)
            self.peak_active = max(self.peak_active, len(active))
            progressed = False
            for a in list(active):
                a.inflight = [t for t in a.inflight if not ex.done(t)]
                while a.remaining > 0 and len(a.inflight) < self.depth and not a.failed:
                    n = min(self.chunk, a.remaining)
                    try:
                        a.inflight.append(ex.submit(a.handle, n))
                    except StglbmError as e:
                        a.failed = str(e)
                        break
                    a.remaining -= n
                    progressed = True
                if (a.remaining == 0 or a.failed) and not a.inflight:
                    status, stats, ns, msg = ex.finish(a.handle)
                    if a.failed:
                        status, msg = "unstable", a.failed
                    job = a.job
                    results.append(JobResult(job_id=job["id"], arrival_s=job["arrival_s"], admitted_s=a.admitted_s,
                                             finished_s=self.clock() - t0, cells=job["cfg"]["cells"],
                                             steps=int(job["steps"]), status=status, stats=stats,
                                             n_samples=ns, message=msg))
                    used -= need[job["id"]]
                    active.remove(a)
                    progressed = True
            if not progressed:
                self.idle()
        makespan = self.clock() - t0
        results.sort(key=lambda r: r.job_id)
        return results, summarize(results, makespan)


def summarize(results, makespan_s):
    lat = np.array([r.latency_s for r in results]) if results else np.zeros(1)
    work = sum(r.cells * r.steps for r in results if r.status == "ok")
    return {
        "jobs": len(results),
        "ok": sum(r.status == "ok" for r in results),
        "unstable": sum(r.status != "ok" for r in results),
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "mean_queue_s": float(np.mean([r.admitted_s - r.arrival_s for r in results])) if results else 0.0,
        "makespan_s": float(makespan_s),
        "aggregate_mlups": work / makespan_s / 1e6 if makespan_s > 0 else 0.0,
    }
