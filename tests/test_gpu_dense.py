"""GPU parity of the dense-H path (MFMA GEMM Horner stages) against the oracle.

Each of the `columns` walks sharing H is compared with the oracle run on its
own initial state.  c128 (FP64 matrix cores) within 1e-12; c64 (FP32 matrix
cores, FP64 re-accumulation every 256 terms) within L2 1e-5.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import closed_forms as cf
from paper_2406_08186_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    yield
    torch.cuda.synchronize()


def _dense_run(g, columns, dtype, gamma, dt, K, steps, marked, seed):
    from paper_2406_08186_amd.walk import Plan
    print(f"[case] dense {g.name} n={g.n} cols={columns} {dtype} K={K} steps={steps}", flush=True)
    pl = Plan(g, "ctqw", dtype=dtype, layout="dense", gamma=gamma, dt=dt, taylor_order=K, marked=marked,
              columns=columns)
    assert pl.structure == "dense"
    states = np.stack([I.random_state(g.n, seed + b) for b in range(columns)], axis=1)  # n x C
    psi = pl.state(states.reshape(-1))
    p, norm, pm = pl.evolve(psi, steps, readout=True)
    torch.cuda.synchronize()
    got = psi.cpu().numpy().astype(np.complex128).reshape(g.n, columns)
    return states, got, p.cpu().numpy().reshape(g.n, columns), float(norm), float(pm)


GRAPHS = {
    "complete130": (I.complete(130), [5]),
    "er301": (I.erdos_renyi(301, 0.3, seed=3), [0, 300]),
    "rr200": (I.random_regular(200, 7, seed=4), []),
    "er64": (I.erdos_renyi(64, 0.5, seed=5), [17]),
}


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("columns", [1, 3, 8, 40])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_dense_matches_oracle(name, columns, dtype):
    g, marked = GRAPHS[name]
    dmax = int(np.diff(g.row_ptr).max())
    gamma = 1.0 / dmax
    states, got, p, norm, pm = _dense_run(g, columns, dtype, gamma, 0.25, 12, 6, marked, seed=10)
    for b in range(columns):
        ref = oracle.ctqw_evolve(g.row_ptr, g.col, states[:, b], 6, gamma=gamma, dt=0.25, K=12, marked=marked)
        if dtype == "c128":
            assert np.abs(got[:, b] - ref).max() < 1e-12, b
            assert np.abs(p[:, b] - np.abs(ref) ** 2).max() < 1e-12
        else:
            assert np.linalg.norm(got[:, b] - ref) < 1e-5, b
    assert abs(norm - columns) < (1e-11 if dtype == "c128" else 1e-4)
    if marked:
        assert abs(pm - p[marked, :].sum()) < 1e-12


@pytest.mark.parametrize("K", [1, 2, 5])
def test_dense_orders_and_sparse_agreement(K):
    """Low orders (buffer cases) and agreement with the sparse CSR path."""
    from paper_2406_08186_amd.walk import Plan
    g = I.erdos_renyi(257, 0.1, seed=9)
    states, got, *_ = _dense_run(g, 4, "c128", 0.1, 0.1, K, 5, [3], seed=30)
    for b in range(4):
        pl = Plan(g, "ctqw", dtype="c128", layout="csr", gamma=0.1, dt=0.1, taylor_order=K, marked=[3])
        x = pl.state(states[:, b])
        pl.evolve(x, 5)
        torch.cuda.synchronize()
        assert np.abs(x.cpu().numpy() - got[:, b]).max() < 1e-13


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-12), ("c64", 1e-5)])
def test_dense_complete_graph_search(dtype, tol):
    """K_N with gamma = 1/N: p_w reaches 1 at t = (pi/2) sqrt(N), on the dense path."""
    from paper_2406_08186_amd.walk import Plan
    n = 1024
    g = I.complete(n)
    t = math.pi / 2 * math.sqrt(n)
    steps = 120
    pl = Plan(g, "ctqw", dtype=dtype, layout="dense", gamma=1.0 / n, dt=t / steps, taylor_order=24,
              marked=[33], columns=2)
    u = np.full(n, 1 / math.sqrt(n), dtype=np.complex128)
    psi = pl.state(np.stack([u, u], axis=1).reshape(-1))
    p, norm, pm = pl.evolve(psi, steps, readout=True)
    torch.cuda.synchronize()
    assert abs(float(pm) - 2.0) < 2 * tol  # both columns reach p_w = 1
    assert abs(cf.complete_search_prob(n, t) - 1.0) < 1e-15


WIDE = {
    # n = 301: two k splits of 160 (the split-k partial products and their reduction)
    "er301": (I.erdos_renyi(301, 0.3, seed=3), [0, 300]),
    # n = 2100: eight k splits of 288, so the FP32 products fold into FP64 inside a split
    "er2100": (I.erdos_renyi(2100, 0.02, seed=21), [5, 2099]),
}


@pytest.mark.parametrize("name", list(WIDE))
@pytest.mark.parametrize("columns", [12, 16, 20, 32, 100, 128])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_dense_wide_tiles(name, columns, dtype):
    """Every accumulator width of the matrix-core stage: 9-16 columns (two
    16-wide real tiles), 17-32 (four), 65-128 (sixteen), full and ragged,
    each walk against the oracle run on its own initial state (the dense
    product that the paper times, Sec. 4.6.1, inside the Taylor step of
    Sec. 3.1)."""
    g, marked = WIDE[name]
    dmax = int(np.diff(g.row_ptr).max())
    gamma = 1.0 / dmax
    steps, K, dt = 4, 12, 0.3
    states, got, p, norm, pm = _dense_run(g, columns, dtype, gamma, dt, K, steps, marked, seed=50)
    for b in range(columns):
        ref = oracle.ctqw_evolve(g.row_ptr, g.col, states[:, b], steps, gamma=gamma, dt=dt, K=K, marked=marked)
        if dtype == "c128":
            assert np.abs(got[:, b] - ref).max() < 1e-12, b
            assert np.abs(p[:, b] - np.abs(ref) ** 2).max() < 1e-12, b
        else:
            assert np.linalg.norm(got[:, b] - ref) < 1e-5, b
    assert abs(norm - columns) < (1e-10 if dtype == "c128" else 1e-4)
    assert abs(pm - p[marked, :].sum()) < 1e-11
