"""GPU parity of the lattice coined walks: Fourier and arbitrary matrix coins
and the persistent shift on cycles and periodic grids (index-free structured
kernels) against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2406_08186_amd import _lib as L
from paper_2406_08186_amd import inputs as I

pytestmark = pytest.mark.gpu


def _unitary(d, seed):
    r = np.random.default_rng(seed)
    q, _ = np.linalg.qr(r.normal(size=(d, d)) + 1j * r.normal(size=(d, d)))
    return q


CASES = [
    ("cycle", 61, "hadamard", "persistent"), ("cycle", 61, "fourier", "flipflop"),
    ("cycle", 61, "fourier", "persistent"), ("cycle", 61, "random", "persistent"),
    ("cycle", 61, "grover", "persistent"),
    ("grid", (12, 9), "fourier", "persistent"), ("grid", (12, 9), "fourier", "flipflop"),
    ("grid", (7, 33), "random", "persistent"), ("grid", (7, 33), "random", "flipflop"),
    ("grid", (10, 10), "grover", "persistent"),
]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("family,size,coin,shift", CASES)
def test_lattice_walk_matches_oracle(family, size, coin, shift, dtype):
    from paper_2406_08186_amd.walk import Coined
    if family == "cycle":
        g, dims, d = I.cycle(size), (size,), 2
    else:
        g, dims, d = I.torus_directed(*size), size, 4
    c = _unitary(d, 7) if coin == "random" else coin
    marked = [3, g.n - 2]
    print(f"[case] lattice {g.name} {coin} {shift} {dtype}", flush=True)
    w = Coined(g, shift=shift, coin=c, marked=marked, dtype=dtype)
    assert w.plan.structure == family.replace("grid", "torus")
    psi0 = I.random_state(g.n_arcs, 11)
    steps = 37
    psi = w.plan.state(psi0)
    p, norm, pm = w.plan.evolve(psi, steps, readout=True)
    torch.cuda.synchronize()
    ref = oracle.coined_evolve_general(g.row_ptr, g.col, psi0, steps, coin=c, shift=shift, dims=dims,
                                       marked=marked)
    got = psi.cpu().numpy().astype(np.complex128)
    pref = oracle.coined_prob(g.row_ptr, g.col, ref)
    if dtype == "c128":
        assert np.abs(got - ref).max() < 1e-12
        assert np.abs(p.cpu().numpy() - pref).max() < 1e-12
    else:
        assert np.linalg.norm(got - ref) < 1e-5
    assert abs(float(pm) - pref[marked].sum()) < (1e-12 if dtype == "c128" else 1e-6)


def test_lattice_snapshots_and_batch_rejection():
    from paper_2406_08186_amd.walk import Batch, Coined
    g = I.torus_directed(9, 8)
    w = Coined(g, shift="persistent", coin="fourier", dtype="c128")
    psi0 = I.random_state(g.n_arcs, 3)
    states = w.simulate(range=(0, 12, 4), state=psi0)
    for k, s in zip(range(0, 12, 4), states):
        ref = oracle.coined_evolve_general(g.row_ptr, g.col, psi0, k, coin="fourier", shift="persistent",
                                           dims=(9, 8))
        assert np.abs(s.cpu().numpy() - ref).max() < 1e-12
    b = Batch(capacity=1, max_tiles=64, dtype="c128")
    with pytest.raises(L.QwError):
        b.set_slot(0, w.plan, w.plan.state(psi0), 3)
    b.close()
