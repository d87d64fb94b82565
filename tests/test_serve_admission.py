"""Admission control of the walk server (host logic, CPU only)."""
import numpy as np
import pytest

from paper_2406_08186_amd.serve import AdmissionController, Job, make_job, poisson_arrivals


def _job(i, fp):
    j = Job(i, graph=None, kind="ctqw", params={}, psi0=None, steps=1)
    j.footprint = fp
    return j


def test_fcfs_and_budget():
    a = AdmissionController(capacity=3, budget_bytes=100)
    jobs = [_job(i, fp) for i, fp in enumerate([40, 50, 30, 10, 5])]
    for j in jobs:
        assert a.offer(j)
    got = a.admit()
    assert [j.job_id for j in got] == [0, 1]          # 40 + 50; job 2 (30) does not fit
    assert a.used == 90 and len(a.free_slots) == 1
    a.release(got[0])
    got2 = a.admit()
    assert [j.job_id for j in got2] == [2, 3]         # FCFS: 30 then 10, slots 2 free
    assert a.used == 90 and a.used <= a.budget
    assert not a.free_slots
    assert [j.job_id for j in a.queue] == [4]          # head waits for a slot


def test_oversize_job_rejected_not_queued():
    a = AdmissionController(capacity=2, budget_bytes=100)
    big = _job(0, 101)
    assert not a.offer(big) and big.status == "rejected"
    assert not a.queue


def test_head_of_line_blocks_smaller_followers():
    a = AdmissionController(capacity=4, budget_bytes=100)
    first = _job(0, 90)
    a.offer(first)
    assert a.admit() == [first]
    a.offer(_job(1, 50))
    a.offer(_job(2, 5))
    assert a.admit() == []             # job 1 does not fit; job 2 waits behind it (FCFS)
    a.release(first)
    assert [j.job_id for j in a.admit()] == [1, 2]


def test_cancel_and_release_free_resources():
    a = AdmissionController(capacity=1, budget_bytes=100)
    j0, j1 = _job(0, 10), _job(1, 10)
    a.offer(j0)
    a.offer(j1)
    assert a.admit() == [j0]
    assert a.cancel(j1) and j1.status == "cancelled" and not a.queue
    assert not a.cancel(j0)            # running jobs are cancelled by the server
    a.release(j0)
    assert a.used == 0 and a.free_slots == [0]
    with pytest.raises(ValueError):
        a.release(j0)


def test_job_stream_recipe():
    rng = np.random.default_rng(3)
    jobs = [make_job(i, rng, arc_range=(1e3, 2e4), steps_range=(100, 500)) for i in range(40)]
    kinds = {j.kind for j in jobs}
    assert kinds == {"coined", "ctqw"}
    for j in jobs:
        assert 100 <= j.steps <= 500
        assert j.psi0.size == (j.graph.n_arcs if j.kind == "coined" else j.graph.n)
        assert abs(np.linalg.norm(j.psi0) - 1) < 1e-12
    t = poisson_arrivals(1000, 4.0, np.random.default_rng(1))
    assert np.all(np.diff(t) > 0) and abs(1000 / t[-1] - 4.0) < 0.5


def test_batch_arc_cap_and_solo_lane():
    a = AdmissionController(capacity=8, budget_bytes=1000, batch_arcs=100)
    jobs = [_job(i, 10) for i in range(4)]
    for j, arcs in zip(jobs, [60, 30, 20, 5]):
        j.graph = type("G", (), {"n_arcs": arcs})()
        assert a.offer(j)
    assert [j.job_id for j in a.admit()] == [0, 1]    # 60 + 30; 20 would pass the cap of 100
    assert a.arcs_running == 90
    a.release(jobs[0])
    assert [j.job_id for j in a.admit()] == [2, 3]
    assert a.arcs_running == 55
    big = _job(9, 10)
    big.graph = type("G", (), {"n_arcs": 500})()
    big.lane = "solo"
    assert a.offer(big) and list(a.solo_queue) == [big]
    assert a.admit_solo() is big and a.admit_solo() is None   # one solo slot by default
    assert a.used == 30 + 10
    a.release(big)
    assert a.solo == [] and a.used == 30
    b = AdmissionController(capacity=1, budget_bytes=100, solo_slots=2)
    s = [_job(20 + i, 30) for i in range(3)]
    for j in s:
        j.lane = "solo"
        b.offer(j)
    assert b.admit_solo() is s[0] and b.admit_solo() is s[1] and b.admit_solo() is None
    b.release(s[0])
    assert b.admit_solo() is s[2] and b.used == 60


def test_idle_solo_routing_predicate():
    """A mid-size job goes to a solo lane only while the batch holds and awaits
    no job and a solo lane is free (the predicate the plan-building threads read)."""
    from types import SimpleNamespace

    from paper_2406_08186_amd.serve import WalkServer
    a = AdmissionController(capacity=4, budget_bytes=1000, solo_slots=2)
    srv = SimpleNamespace(adm=a, solo_lanes=[None, None])
    idle = lambda: WalkServer._batch_idle(srv)  # noqa: E731
    assert idle()
    batch_job = _job(1, 10)
    a.offer(batch_job)                       # waiting for the batch
    assert not idle()
    a.admit()                                # now running in the batch
    assert not idle()
    a.release(batch_job)
    assert idle()
    solos = []
    for i in range(2):
        j = _job(10 + i, 10)
        j.lane = "solo"
        a.offer(j)
        solos.append(j)
    assert not idle()                        # both solo lanes spoken for (two jobs queued)
    a.admit_solo()
    assert not idle()                        # one running, one queued
    a.release(solos[0])
    assert idle()                            # one queued, one lane free
    a.admit_solo()
    assert idle()                            # one running, one lane free
