"""GPU test of the serving loop: each job's result is the same alone and in the
mix (bitwise against a one-slot batch, to rounding against the plain path),
jobs arriving while others run overlap with them, and the device budget is
respected."""
import numpy as np
import pytest
import torch

from paper_2406_08186_amd.serve import WalkServer, make_job, serve_stream

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone():
    from paper_2406_08186_amd.walk import Batch, Plan
    rng = np.random.default_rng(11)
    jobs = [make_job(i, rng, arc_range=(1e3, 6e4), steps_range=(20, 120)) for i in range(14)]
    for i, j in enumerate(jobs):
        j.arrival = 0.01 * i
    print(f"[case] serve {len(jobs)} jobs", flush=True)
    budget = 64 * 2**20
    srv = WalkServer(capacity=6, budget_bytes=budget, chunk=16, dtype="c64", max_tiles=1 << 14,
                     keep_states=True)
    peak = [0]
    orig = srv.adm.admit

    def admit_and_track():
        out = orig()
        peak[0] = max(peak[0], srv.adm.used)
        return out

    srv.adm.admit = admit_and_track
    done = serve_stream(srv, jobs, time_limit=300)
    srv.close()
    assert len(done) == len(jobs) and all(j.status == "done" for j in done)
    assert peak[0] <= budget
    overlapped = sum(1 for a in done for b in done
                     if a is not b and a.admitted_at < b.admitted_at < a.finished_at)
    assert overlapped > 0, "no job joined while another was running"
    for j in done:
        plan = Plan(j.graph, j.kind, dtype="c64", layout="structured" if j.kind == "coined" else "csr",
                    **j.params)
        b = Batch(capacity=1, max_tiles=1 << 14, dtype="c64")
        psi = plan.state(j.psi0)
        b.set_slot(0, plan, psi, j.steps)
        b.commit()
        b.run_to_completion()
        b.readout(0)
        torch.cuda.synchronize()
        alone = psi.cpu().numpy()
        assert np.array_equal(alone, j.result["psi"]), f"job {j.job_id} differs alone vs in the mix"
        plain = plan.state(j.psi0)
        plan.evolve(plain, j.steps)
        torch.cuda.synchronize()
        assert np.abs(plain.cpu().numpy() - j.result["psi"]).max() < 1e-5
        assert abs(j.result["norm"] - 1.0) < 1e-5
        b.close()
