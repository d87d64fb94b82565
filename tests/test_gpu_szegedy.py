"""GPU parity of Szegedy's walk (the Szegedy reflection coin with the flip-flop
shift) on the one-workgroup and general CSR paths against the pinned oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2406_08186_amd import inputs as I

pytestmark = pytest.mark.gpu


def _transition(g, seed):
    rng = np.random.default_rng(seed)
    raw = rng.uniform(0.05, 1.0, size=g.n_arcs)
    deg = np.diff(g.row_ptr)
    sums = np.zeros(g.n)
    np.add.at(sums, np.repeat(np.arange(g.n), deg), raw)
    return raw / np.repeat(np.where(sums > 0, sums, 1.0), deg)


GRAPHS = {
    "small": lambda: I.random_mixed(40, seed=2),           # one workgroup under "auto"
    "mixed": lambda: I.random_mixed(300, seed=4),          # isolated vertices, leaves, a hub
    "er": lambda: I.erdos_renyi(3000, 0.004, seed=5),
    "hub": lambda: I.from_edges(2600, np.stack([np.zeros(2599, int), np.arange(1, 2600)], 1), name="star2600"),
}                                                          # a vertex of degree > one LDS tile


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("layout", ["auto", "csr"])
@pytest.mark.parametrize("name", list(GRAPHS))
def test_szegedy_matches_oracle(name, layout, dtype):
    from paper_2406_08186_amd.walk import Coined
    g = GRAPHS[name]()
    p = _transition(g, 3)
    marked = [1, 7]
    print(f"[case] szegedy {g.name} {layout} {dtype}", flush=True)
    w = Coined(g, coin="szegedy", transition=p, marked=marked, dtype=dtype, layout=layout)
    psi0 = I.random_state(g.n_arcs, 8)
    psi = w.plan.state(psi0)
    pr, norm, pm = w.plan.evolve(psi, 23, readout=True)
    torch.cuda.synchronize()
    ref = oracle.szegedy_evolve(g.row_ptr, g.col, psi0, 23, p, marked=marked)
    got = psi.cpu().numpy().astype(np.complex128)
    if dtype == "c128":
        assert np.abs(got - ref).max() < 1e-12
        assert np.abs(pr.cpu().numpy() - oracle.coined_prob(g.row_ptr, g.col, ref)).max() < 1e-12
    else:
        assert np.linalg.norm(got - ref) < 1e-5
    assert abs(float(norm) - 1) < (1e-12 if dtype == "c128" else 1e-5)
