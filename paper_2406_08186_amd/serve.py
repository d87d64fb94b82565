"""Continuous-batching walk server on one GPU.

Jobs (a graph, a walk, an initial state and a step count) arrive over time.
Host-side plan building (validation, reverse arcs, Taylor order) runs in a
thread pool; the admission controller admits jobs first-come-first-served
while the job's device footprint (graph tables + workspace + state) fits the
HBM budget.  Three lanes share the GPU on their own streams:

* the small lane runs jobs whose graphs fit one workgroup's LDS whole: a
  group of them goes out in one launch (qw_small_many), one workgroup per
  job, every step of every job inside that launch;
* the batch lane holds the mid-size jobs in one continuous batch: admitted
  jobs join between chunks of launches, their states stay resident until they
  finish, and every chunk advances every job in the batch; a cap on the arcs
  in the batch bounds the time of a launch;
* the solo lanes run, each on its own stream and in arrival order, jobs
  large enough to fill the GPU on their own and jobs that need many launches
  (steps x Taylor order for a CTQW): in the batch such a job would pay the
  whole batch's launch time for every one of its launches.  A solo job runs
  in chunks of steps on the single-walk path.

The lanes are polled independently, so a small job never waits for a large
job's launches, and a large job does not slow every launch of the batch.
Finished jobs are read out (FP64 probabilities) and their memory and slot
are released.  A walk's arithmetic does not depend on the other jobs, so
each result is the same alone and served.
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
    lane: str = "batch"           # "small", "batch" or "solo"; "plain" in the one-at-a-time form
    footprint: int = 0
    slot: int = -1
    admitted_at: float = math.nan
    finished_at: float = math.nan
    result: Optional[dict] = None
    status: str = "new"           # new, building, queued, running, done, rejected, cancelled

    @property
    def arcs(self) -> int:
        return int(self.graph.n_arcs) if self.graph is not None else 0

    @property
    def latency(self) -> float:
        return self.finished_at - self.arrival


class AdmissionController:
    """FCFS admission by device-memory budget (host logic only).

    Batch-lane jobs also need a free batch slot; solo-lane jobs run up to
    `solo_slots` at a time; small-lane jobs go out in groups.  Each lane keeps
    its own FCFS queue; all draw on one budget.
    """

    def __init__(self, capacity: int, budget_bytes: int, batch_arcs: int | None = None,
                 solo_slots: int = 1):
        self.capacity = capacity
        self.solo_slots = solo_slots
        self.budget = int(budget_bytes)
        self.batch_arcs = batch_arcs    # cap on the arcs one batch launch advances (None: none)
        self.arcs_running = 0
        self.used = 0
        self.free_slots = list(range(capacity - 1, -1, -1))
        self.queue: deque[Job] = deque()        # batch lane
        self.solo_queue: deque[Job] = deque()   # solo lane
        self.small_queue: deque[Job] = deque()  # small lane
        self.small: list[Job] = []              # running small-lane jobs
        self.running: dict[int, Job] = {}       # batch slot -> job
        self.solo: list[Job] = []               # running solo-lane jobs

    def offer(self, job: Job) -> bool:
        """Queue a job whose footprint is known; reject it if it can never fit."""
        if job.footprint > self.budget:
            job.status = "rejected"
            return False
        job.status = "queued"
        {"solo": self.solo_queue, "small": self.small_queue}.get(job.lane, self.queue).append(job)
        return True

    def admit(self) -> list[Job]:
        """Pop batch-lane jobs in arrival order while a slot and the budget allow."""
        out = []
        while self.queue and self.free_slots and self.queue[0].footprint <= self.budget - self.used:
            head = self.queue[0]
            if (self.batch_arcs is not None and self.running
                    and self.arcs_running + head.arcs > self.batch_arcs):
                break  # the launch would grow past its arc cap: wait for running jobs to finish
            job = self.queue.popleft()
            job.slot = self.free_slots.pop()
            job.status = "running"
            self.used += job.footprint
            self.arcs_running += job.arcs
            self.running[job.slot] = job
            out.append(job)
        return out

    def admit_solo(self) -> Optional[Job]:
        """Pop the next solo-lane job if a solo slot is free and the budget allows."""
        if (len(self.solo) < self.solo_slots and self.solo_queue
                and self.solo_queue[0].footprint <= self.budget - self.used):
            job = self.solo_queue.popleft()
            job.status = "running"
            self.used += job.footprint
            self.solo.append(job)
            return job
        return None

    def admit_small(self, limit: int) -> list[Job]:
        """Pop up to `limit` small-lane jobs in arrival order while the budget allows."""
        out = []
        while (len(out) < limit and self.small_queue
               and self.small_queue[0].footprint <= self.budget - self.used):
            job = self.small_queue.popleft()
            job.status = "running"
            self.used += job.footprint
            self.small.append(job)
            out.append(job)
        return out

    def release(self, job: Job) -> None:
        if job.lane == "small":
            if job not in self.small:
                raise ValueError("job is not running")
            self.small.remove(job)
        elif job.lane == "solo":
            if job not in self.solo:
                raise ValueError("job is not running")
            self.solo.remove(job)
        else:
            if self.running.get(job.slot) is not job:
                raise ValueError("job is not running")
            del self.running[job.slot]
            self.free_slots.append(job.slot)
            self.arcs_running -= job.arcs
            job.slot = -1
        self.used -= job.footprint

    def cancel(self, job: Job) -> bool:
        """Drop a queued job; running jobs are cancelled by the server."""
        for q in (self.queue, self.solo_queue, self.small_queue):
            try:
                q.remove(job)
            except ValueError:
                continue
            job.status = "cancelled"
            return True
        return False

    def busy(self) -> bool:
        return bool(self.queue or self.solo_queue or self.small_queue or self.running or self.solo
                    or self.small)


class WalkServer:
    """Serve walk jobs on one GPU (complex64 by default): groups of whole-walk
    launches for jobs that fit one workgroup (up to `small_group` per launch, on
    `small_streams` streams), a continuous batch for mid-size jobs, and
    `solo_slots` solo lanes for jobs of at least `solo_arcs` arcs or at least
    `solo_units` launches (steps, times the Taylor order for a CTQW).
    The batch admits jobs while their arcs total at most `batch_arcs`, which
    bounds the time of one batch launch and so the latency of every job in it.
    With `idle_solo`, a mid-size job whose plan is built while the batch holds
    and awaits no job and a solo lane is free goes to that solo lane: at light
    load it then runs alone on its fastest path instead of on the batch
    kernel."""

    def __init__(self, capacity: int = 64, budget_bytes: int | None = None, chunk: int = 64,
                 dtype: str = "c64", max_tiles: int = 1 << 18, workers: int = 4, device=None,
                 keep_states: bool = False, solo_arcs: int = 1 << 19, solo_chunk: int = 64,
                 batch_arcs: int | None = 1 << 21, solo_slots: int = 3, small_group: int = 16,
                 small_streams: int = 3, solo_units: int | None = 16384, idle_solo: bool = True):
        import torch

        from .walk import Batch
        self.torch = torch
        self.device = torch.device(device) if device is not None else torch.device("cuda", 0)
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            budget_bytes = int(0.5 * free)
        self.dtype = dtype
        self.chunk = chunk
        self.solo_arcs = solo_arcs
        self.solo_units = solo_units
        self.idle_solo = idle_solo
        self.solo_chunk = solo_chunk
        self.keep_states = keep_states
        self.s_batch = torch.cuda.Stream(self.device)
        self.small_group = small_group
        # small-lane launches in flight: [jobs, stream, event, descriptor buffer]
        self.small_lanes = [[[], torch.cuda.Stream(self.device), None, None] for _ in range(small_streams)]
        # one stream per solo lane: [job, stream, event after its last chunk, steps left]
        self.solo_lanes = [[None, torch.cuda.Stream(self.device), None, 0] for _ in range(solo_slots)]
        self.batch = Batch(capacity, max_tiles, dtype, device=self.device, stream=self.s_batch)
        self.adm = AdmissionController(capacity, budget_bytes, batch_arcs, solo_slots)
        self.pool = ThreadPoolExecutor(max_workers=workers)
        self.building: list[tuple[Job, Future]] = []
        self.live: dict[int, tuple] = {}
        self.done: list[Job] = []
        self.t0 = time.perf_counter()
        self.cycles = 0
        self._cancel: set[int] = set()
        self._batch_ev = None       # event after the batch lane's last chunk

    def now(self) -> float:
        return time.perf_counter() - self.t0

    # -- intake ------------------------------------------------------------
    def submit(self, job: Job) -> None:
        """Accept a job now: its host-side plan is built in the background, and
        the plan's path picks the lane."""
        from .walk import Plan
        job.status = "building"
        solo = job.arcs >= self.solo_arcs

        def build():
            # alone, the plan picks its fastest path; a graph that fits one
            # workgroup goes to the small lane, the rest of the mid-size jobs
            # to the batch (coined walks on cycles, grids and hypercubes in the
            # index-free slot-major layout, everything else on CSR)
            plan = Plan(job.graph, job.kind, dtype=self.dtype, layout="auto", device=self.device,
                        upload=False, **job.params)
            if plan.structure == "small" and not solo:
                return plan, "small"
            units = job.steps * (int(plan.info.taylor_order) if job.kind == "ctqw" else 1)
            if solo or (self.solo_units is not None and units >= self.solo_units):
                return plan, "solo"
            if self.idle_solo and self._batch_idle():
                return plan, "solo"
            plan.close()
            layout = "structured" if job.kind == "coined" else "csr"
            return Plan(job.graph, job.kind, dtype=self.dtype, layout=layout, device=self.device,
                        upload=False, **job.params), "batch"

        self.building.append((job, self.pool.submit(build)))

    def _batch_idle(self) -> bool:
        """No job in or waiting for the batch, and a solo lane free (read from
        a plan-building thread: the sizes are a routing hint only, and either
        lane runs any job)."""
        a = self.adm
        return not a.running and not a.queue and len(a.solo) + len(a.solo_queue) < len(self.solo_lanes)

    def cancel(self, job: Job) -> None:
        if not self.adm.cancel(job) and job.status == "running":
            self._cancel.add(job.job_id)

    def _collect_built(self) -> None:
        still = []
        for job, fut in self.building:
            if fut.done():
                plan, job.lane = fut.result()
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

    def _upload(self, job: Job, stream):
        """Device tables and state of an admitted job (later launches on a lane's
        stream wait for this upload on torch's current stream)."""
        plan, _ = self.live[job.job_id]
        plan.upload()
        psi = plan.state(job.psi0)
        self.live[job.job_id] = (plan, psi)
        job.admitted_at = self.now()
        return plan, psi

    # -- one scheduling cycle -------------------------------------------------
    def cycle(self) -> int:
        """Poll both lanes once; returns the number of launches or steps enqueued."""
        self._collect_built()
        work = self._small_lane() + self._batch_lane() + self._solo_lane()
        self.cycles += 1
        return work

    def _batch_lane(self) -> int:
        if self._batch_ev is not None and not self._batch_ev.query():
            return 0
        self._batch_ev = None
        changed = False
        for job in list(self.adm.running.values()):
            if job.job_id in self._cancel:
                self._cancel.discard(job.job_id)
                self._finish(job, cancelled=True)
                changed = True
            elif self.batch.remaining(job.slot) == 0:
                self._finish(job)
                changed = True
        for job in self.adm.admit():
            plan, psi = self._upload(job, self.s_batch)
            self.batch.set_slot(job.slot, plan, psi, job.steps)
            changed = True
        if changed:
            self.batch.commit(stream=self.s_batch)
        pending = [r for r in (self.batch.remaining(j.slot) for j in self.adm.running.values()) if r > 0]
        n = min(self.chunk, min(pending)) if pending else 0
        if n or changed:
            if n:
                self.batch.run(n, stream=self.s_batch)
            self._batch_ev = self.torch.cuda.Event()
            self._batch_ev.record(self.s_batch)
        return n

    def _small_lane(self) -> int:
        from .walk import evolve_many
        work = 0
        for lane in self.small_lanes:
            jobs, stream, ev, _ = lane
            if ev is not None and not ev.query():
                continue
            for job in jobs:
                self._cancel.discard(job.job_id)
                self._finish(job, stream=stream)
            lane[0], lane[2], lane[3] = [], None, None
            jobs = self.adm.admit_small(self.small_group)
            if not jobs:
                continue
            plans, states = [], []
            for job in jobs:
                plan, psi = self._upload(job, stream)
                plans.append(plan)
                states.append(psi)
            lane[3] = evolve_many(plans, states, [j.steps for j in jobs], stream=stream)
            lane[0] = jobs
            lane[2] = self.torch.cuda.Event()
            lane[2].record(stream)
            work += len(jobs)
        return work

    def _solo_lane(self) -> int:
        work = 0
        for lane in self.solo_lanes:
            job, stream, ev, left = lane
            if ev is not None and not ev.query():
                continue
            lane[2] = None
            if job is not None and (job.job_id in self._cancel or left == 0):
                cancelled = job.job_id in self._cancel
                self._cancel.discard(job.job_id)
                self._finish(job, cancelled=cancelled, stream=stream)
                job = lane[0] = None
            if job is None:
                job = self.adm.admit_solo()
                if job is None:
                    continue
                self._upload(job, stream)
                lane[0], left = job, job.steps
            plan, psi = self.live[job.job_id]
            k = min(self.solo_chunk, left)
            if k:
                plan.evolve(psi, k, stream=stream)
            lane[3] = left - k
            lane[2] = self.torch.cuda.Event()
            lane[2].record(stream)
            work += k
        return work

    def _finish(self, job: Job, cancelled: bool = False, stream=None) -> None:
        plan, psi = self.live.pop(job.job_id)
        stream = stream if stream is not None else self.s_batch
        if not cancelled:
            if job.lane == "small":
                p, norm, pm = plan.probabilities(psi, stream=stream)
            elif job.lane == "solo":
                p, norm, pm = plan.evolve(psi, 0, readout=True, stream=stream)
            else:
                p, norm, pm = self.batch.readout(job.slot, stream=stream)
            stream.synchronize()
            job.result = {"norm": float(norm), "p_marked": float(pm),
                          "p": p.cpu().numpy() if self.keep_states else None,
                          "psi": psi.cpu().numpy() if self.keep_states else None}
            job.status = "done"
        else:
            stream.synchronize()
            job.status = "cancelled"
        job.finished_at = self.now()
        if job.lane == "batch":
            self.batch.clear_slot(job.slot)
        self.adm.release(job)
        plan.release_device()
        plan.close()
        self.done.append(job)

    def busy(self) -> bool:
        return bool(self.building or self.adm.busy())

    def close(self) -> None:
        self.pool.shutdown(wait=True)
        self.torch.cuda.synchronize(self.device)
        self.batch.close()


def serve_stream(server: WalkServer, jobs: list[Job], time_limit: float = 600.0, progress=None,
                 progress_every: int = 200) -> list[Job]:
    """Release jobs at their arrival times (seconds after start) and serve until all finish.
    `progress(done, seconds)` is called each time another `progress_every` jobs have finished."""
    pending = deque(sorted(jobs, key=lambda j: j.arrival))
    server.t0 = time.perf_counter()
    reported = 0
    while pending or server.busy():
        t = server.now()
        if t > time_limit:
            raise TimeoutError("serving stream exceeded its time limit")
        while pending and pending[0].arrival <= t:
            server.submit(pending.popleft())
        if server.cycle() == 0:
            time.sleep(0.0002)
        if progress is not None and len(server.done) // progress_every > reported:
            reported = len(server.done) // progress_every
            progress(len(server.done), server.now())
    return server.done


def serve_sequential(jobs: list[Job], dtype: str = "c64", device=None, time_limit: float = 600.0, progress=None,
                     progress_every: int = 200):
    """The plain form: one job at a time, in arrival order, each on its fastest single-walk path.
    `progress(done, seconds)` is called after every `progress_every` finished jobs."""
    import torch

    from .walk import Plan
    dev = torch.device(device) if device is not None else torch.device("cuda", 0)
    t0 = time.perf_counter()
    for job in sorted(jobs, key=lambda j: j.arrival):
        while time.perf_counter() - t0 < job.arrival:
            time.sleep(0.0005)
        plan = Plan(job.graph, job.kind, dtype=dtype, layout="auto", device=dev, **job.params)
        psi = plan.state(job.psi0)
        p, norm, pm = plan.evolve(psi, job.steps, readout=True)
        torch.cuda.synchronize(dev)
        job.result = {"norm": float(norm), "p_marked": float(pm)}
        job.status = "done"
        job.lane = "plain"
        job.finished_at = time.perf_counter() - t0
        plan.close()
        if job.finished_at > time_limit:
            raise TimeoutError("sequential stream exceeded its time limit")
        done = sum(1 for j in jobs if j.status == "done")
        if progress is not None and done % progress_every == 0:
            progress(done, job.finished_at)
    return jobs


def latency_stats(jobs: list[Job]) -> dict:
    """p50 / p99 / mean / max latency of the finished jobs, with the sample count:
    p99 is interpolated between order statistics, so with n samples it rests on
    the ceil(n / 100) slowest jobs (`p99_tail_jobs`)."""
    lat = np.array([j.latency for j in jobs if j.status == "done"])
    if lat.size == 0:
        return {"p50_s": None, "p99_s": None, "mean_s": None, "max_s": None, "samples": 0, "p99_tail_jobs": 0}
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "max_s": float(lat.max()), "samples": int(lat.size),
            "p99_tail_jobs": int(-(-lat.size // 100))}


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
