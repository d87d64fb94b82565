"""Continuous-batching walk server on one GPU.

Jobs (a graph, a walk, an initial state and a step count) arrive over time.
Host-side plan building (validation, reverse arcs, Taylor order) runs in a
thread pool; the admission controller admits jobs first-come-first-served
when a batch slot is free and the job's device footprint (graph tables +
workspace + state) fits the HBM budget.  Admitted jobs join the running
batch between chunks of launches, their states stay resident until they
finish, and every chunk advances every active job, so jobs that arrive while
others are on the GPU overlap with them.  Finished jobs are read out (FP64
probabilities) and their memory and slot are released.

A walk's arithmetic in a batch does not depend on the other slots, so each
result is the same alone and in the mix.
"""
from __future__ import annotations

import math
import threading
import time
from collections import deque
from concurrent.futures import Future, ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np


@dataclass
class Job:
    """One walk request.  kind: "coined" or "ctqw"; params go to Plan."""

    job_id: int
    graph: object
    kind: str
    params: dict
    psi0: np.ndarray
    steps: int
    arrival: float = 0.0          # seconds after the server's start
    # filled in by the server
    footprint: int = 0
    slot: int = -1
    admitted_at: float = math.nan
    finished_at: float = math.nan
    result: Optional[dict] = None
    status: str = "new"           # new, building, queued, running, done, rejected, cancelled

    @property
    def arcs(self) -> int:
        return int(self.graph.n_arcs)

    @property
    def latency(self) -> float:
        return self.finished_at - self.arrival


class AdmissionController:
    """FCFS admission by free slot and device-memory budget (host logic only)."""

    def __init__(self, capacity: int, budget_bytes: int):
        self.capacity = capacity
        self.budget = int(budget_bytes)
        self.used = 0
        self.free_slots = list(range(capacity - 1, -1, -1))
        self.queue: deque[Job] = deque()
        self.running: dict[int, Job] = {}

    def offer(self, job: Job) -> bool:
        """Queue a job whose footprint is known; reject it if it can never fit."""
        if job.footprint > self.budget:
            job.status = "rejected"
            return False
        job.status = "queued"
        self.queue.append(job)
        return True

    def admit(self) -> list[Job]:
        """Pop queued jobs in arrival order while a slot and the budget allow."""
        out = []
        while self.queue and self.free_slots and self.queue[0].footprint <= self.budget - self.used:
            job = self.queue.popleft()
            job.slot = self.free_slots.pop()
            job.status = "running"
            self.used += job.footprint
            self.running[job.slot] = job
            out.append(job)
        return out

    def release(self, job: Job) -> None:
        if self.running.get(job.slot) is not job:
            raise ValueError("job is not running")
        del self.running[job.slot]
        self.used -= job.footprint
        self.free_slots.append(job.slot)
        job.slot = -1

    def cancel(self, job: Job) -> bool:
        """Drop a queued job; running jobs are cancelled by the server."""
        try:
            self.queue.remove(job)
        except ValueError:
            return False
        job.status = "cancelled"
        return True


class WalkServer:
    """Serve walk jobs with continuous batching on one GPU (complex64 by default)."""

    def __init__(self, capacity: int = 64, budget_bytes: int | None = None, chunk: int = 64,
                 dtype: str = "c64", max_tiles: int = 1 << 18, workers: int = 4, device=None,
                 keep_states: bool = False):
        import torch

        from .walk import Batch
        self.torch = torch
        self.device = torch.device(device) if device is not None else torch.device("cuda", 0)
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            budget_bytes = int(0.5 * free)
        self.dtype = dtype
        self.chunk = chunk
        self.keep_states = keep_states
        self.batch = Batch(capacity, max_tiles, dtype, device=self.device)
        self.adm = AdmissionController(capacity, budget_bytes)
        self.pool = ThreadPoolExecutor(max_workers=workers)
        self.building: list[tuple[Job, Future]] = []
        self.live: dict[int, tuple] = {}
        self.done: list[Job] = []
        self.t0 = time.perf_counter()
        self.cycles = 0
        self._cancel: set[int] = set()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    # -- intake ------------------------------------------------------------
    def submit(self, job: Job) -> None:
        """Accept a job now: its host-side plan is built in the background."""
        from .walk import Plan
        job.status = "building"

        # coined jobs on cycles, grids and hypercubes take the index-free slot-major path;
        # everything else the CSR path (both run inside the batch)
        layout = "structured" if job.kind == "coined" else "csr"

        def build():
            return Plan(job.graph, job.kind, dtype=self.dtype, layout=layout, device=self.device,
                        upload=False, **job.params)

        self.building.append((job, self.pool.submit(build)))

    def cancel(self, job: Job) -> None:
        if not self.adm.cancel(job) and job.status == "running":
            self._cancel.add(job.job_id)

    def _collect_built(self) -> None:
        still = []
        for job, fut in self.building:
            if fut.done():
                plan = fut.result()
                job.footprint = plan.device_bytes
                if self.adm.offer(job):
                    self.live[job.job_id] = (plan, None)
                else:
                    plan.close()
                    job.finished_at = self.now()
                    self.done.append(job)
            else:
                still.append((job, fut))
        self.building = still

    # -- one scheduling cycle -------------------------------------------------
    def cycle(self) -> int:
        """Admit, run one chunk, reap.  Returns the number of launches run."""
        self._collect_built()
        changed = False
        for job in list(self.adm.running.values()):
            if job.job_id in self._cancel:
                self._cancel.discard(job.job_id)
                self._finish(job, cancelled=True)
                changed = True
        for job in self.adm.admit():
            plan, _ = self.live[job.job_id]
            plan.upload()
            psi = plan.state(job.psi0)
            self.batch.set_slot(job.slot, plan, psi, job.steps)
            self.live[job.job_id] = (plan, psi)
            job.admitted_at = self.now()
            changed = True
        if changed:
            self.batch.commit()
        active = list(self.adm.running.values())
        if not active:
            return 0
        rem = [self.batch.remaining(j.slot) for j in active]
        pending = [r for r in rem if r > 0]
        n = min(self.chunk, min(pending)) if pending else 0
        if n:
            self.batch.run(n)
        self.torch.cuda.synchronize(self.device)
        self.cycles += 1
        for job in active:
            if self.batch.remaining(job.slot) == 0:
                self._finish(job)
        return n

    def _finish(self, job: Job, cancelled: bool = False) -> None:
        plan, psi = self.live.pop(job.job_id)
        if not cancelled:
            p, norm, pm = self.batch.readout(job.slot)
            job.result = {"norm": float(norm), "p_marked": float(pm),
                          "p": p.cpu().numpy() if self.keep_states else None,
                          "psi": psi.cpu().numpy() if self.keep_states else None}
            job.status = "done"
        else:
            job.status = "cancelled"
        job.finished_at = self.now()
        self.batch.clear_slot(job.slot)
        self.adm.release(job)
        plan.release_device()
        plan.close()
        self.done.append(job)

    def busy(self) -> bool:
        return bool(self.building or self.adm.queue or self.adm.running)

    def close(self) -> None:
        self.pool.shutdown(wait=True)
        self.batch.close()


def serve_stream(server: WalkServer, jobs: list[Job], time_limit: float = 600.0) -> list[Job]:
    """Release jobs at their arrival times (seconds after start) and serve until all finish."""
    pending = deque(sorted(jobs, key=lambda j: j.arrival))
    server.t0 = time.perf_counter()
    while pending or server.busy():
        t = server.now()
        if t > time_limit:
            raise TimeoutError("serving stream exceeded its time limit")
        while pending and pending[0].arrival <= t:
            server.submit(pending.popleft())
        if server.cycle() == 0 and not server.adm.running:
            time.sleep(0.0005)
    return server.done


def serve_sequential(jobs: list[Job], dtype: str = "c64", device=None, time_limit: float = 600.0):
    """The plain form: one job at a time, in arrival order, on the single-walk path."""
    import torch

    from .walk import Plan
    dev = torch.device(device) if device is not None else torch.device("cuda", 0)
    t0 = time.perf_counter()
    for job in sorted(jobs, key=lambda j: j.arrival):
        while time.perf_counter() - t0 < job.arrival:
            time.sleep(0.0005)
        plan = Plan(job.graph, job.kind, dtype=dtype, layout="csr", device=dev, **job.params)
        psi = plan.state(job.psi0)
        p, norm, pm = plan.evolve(psi, job.steps, readout=True)
        torch.cuda.synchronize(dev)
        job.result = {"norm": float(norm), "p_marked": float(pm)}
        job.status = "done"
        job.finished_at = time.perf_counter() - t0
        plan.close()
        if job.finished_at > time_limit:
            raise TimeoutError("sequential stream exceeded its time limit")
    return jobs


def latency_stats(jobs: list[Job]) -> dict:
    lat = np.array([j.latency for j in jobs if j.status == "done"])
    if lat.size == 0:
        return {"p50_s": None, "p99_s": None, "mean_s": None}
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean())}


# ---- the mixed job stream ------------------------------------------------------

def make_job(job_id: int, rng: np.random.Generator, arc_range=(1e3, 4e6), steps_range=(100, 5000),
             ctqw_tol: float = 1e-8) -> Job:
    """One job of the mixed stream.

    Half coined Grover walks (periodic grid of side round(sqrt(A/4)), or the
    hypercube whose n 2^n is closest to A, n in 7..18) with one -I marked
    vertex from the uniform arc state; half CTQW searches on G(N, p) with mean
    degree d ~ U[4, 16], N = round(A/d), gamma = 1/d, one marked vertex, from
    the uniform vertex state, dt = 1/||H|| and the Taylor order from the
    truncation rule.  A is log-uniform in arc_range; steps uniform in
    steps_range.
    """
    from . import inputs as I
    A = math.exp(rng.uniform(math.log(arc_range[0]), math.log(arc_range[1])))
    steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
    seed = int(rng.integers(2**31))
    if rng.random() < 0.5:
        if rng.random() < 0.5:
            side = max(3, int(round(math.sqrt(A / 4))))
            g = I.torus(side, side)
        else:
            n = min(range(7, 19), key=lambda k: abs(k * 2**k - A))
            g = I.hypercube(n)
        mk = int(rng.integers(g.n))
        psi0 = I.uniform(g.n_arcs)
        return Job(job_id, g, "coined", {"coin": "grover", "marked": [mk]}, psi0, steps)
    dbar = float(rng.uniform(4, 16))
    n = max(32, int(round(A / dbar)))
    g = I.erdos_renyi(n, dbar / (n - 1), seed)
    mk = int(rng.integers(n))
    hb = 1.0 / dbar * int(np.diff(g.row_ptr).max()) + 1.0
    params = {"gamma": 1.0 / dbar, "dt": 1.0 / hb, "taylor_order": 0, "trunc_tol": ctqw_tol,
              "horizon_steps": steps, "marked": [mk]}
    return Job(job_id, g, "ctqw", params, I.uniform(n), steps)


def poisson_arrivals(n_jobs: int, rate: float, rng: np.random.Generator) -> np.ndarray:
    return np.cumsum(rng.exponential(1.0 / rate, size=n_jobs))
