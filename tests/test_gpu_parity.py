"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle and
the closed forms, element by element, on seeded inputs.

Bars: complex128 states within 1e-12 (max abs) of the oracle; complex64
states within an L2 distance of 1e-4 and a norm drift of 1e-5 after 10^4
steps (looser per-case bounds noted where the run is short).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import closed_forms as cf
from paper_2406_08186_amd import inputs as I

pytestmark = pytest.mark.gpu

C128_TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    from paper_2406_08186_amd import _lib
    _lib.lib()  # fail loudly if the HIP library is not built
    yield
    torch.cuda.synchronize()


def _plan(g, kind, **kw):
    from paper_2406_08186_amd.walk import Plan
    return Plan(g, kind, **kw)


def run_coined(g, psi0, steps, dtype="c128", layout="auto", coin="grover", marked=()):
    print(f"[case] coined {g.name} n={g.n} arcs={g.n_arcs} {dtype} {layout} {coin} steps={steps}",
          flush=True)
    pl = _plan(g, "coined", dtype=dtype, layout=layout, coin=coin, marked=marked)
    psi = pl.state(psi0)
    p, norm, pm = pl.evolve(psi, steps, readout=True)
    torch.cuda.synchronize()
    return (psi.cpu().numpy().astype(np.complex128), p.cpu().numpy(), float(norm), float(pm),
            pl.structure)


def run_ctqw(g, psi0, steps, gamma, dt, K, dtype="c128", layout="auto", marked=()):
    print(f"[case] ctqw {g.name} n={g.n} {dtype} {layout} K={K} steps={steps}", flush=True)
    pl = _plan(g, "ctqw", dtype=dtype, layout=layout, gamma=gamma, dt=dt, taylor_order=K,
               marked=marked)
    psi = pl.state(psi0)
    p, norm, pm = pl.evolve(psi, steps, readout=True)
    torch.cuda.synchronize()
    return (psi.cpu().numpy().astype(np.complex128), p.cpu().numpy(), float(norm), float(pm),
            pl.structure)


def _graphs():
    return {
        "cycle_dir": I.cycle(1001),
        "cycle_sorted": I.cycle_sorted(777),
        "torus": I.torus(37, 29),
        "hypercube": I.hypercube(11),
        "rr": I.random_regular(2000, 5, seed=1),
        "er": I.erdos_renyi(3000, 6.0 / 2999, seed=2),
        "mixed": I.random_mixed(40, seed=3),
        "hub": _hub_graph(),
        "complete": I.complete(70),
    }


def _hub_graph():
    n = 3500
    rng = np.random.default_rng(5)
    edges = {(0, w) for w in range(1, 3001)}
    for _ in range(4000):
        u, w = sorted(rng.integers(1, n, size=2).tolist())
        if u != w:
            edges.add((u, w))
    return I.from_edges(n, sorted(edges), name="hub3500")


GRAPHS = _graphs()

_ORACLE_CACHE = {}


def _cached(key, fn):
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = fn()
    return _ORACLE_CACHE[key]


def _marks(g):
    return [0, g.n // 2] if g.n > 2 else []


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("layout", ["auto", "csr", "structured"])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_coined_grover_parity(name, layout, dtype):
    g = GRAPHS[name]
    steps = 37
    marked = _marks(g)
    psi0 = I.random_state(g.n_arcs, seed=11)
    ref = _cached(("coined", name), lambda: oracle.coined_evolve(g.row_ptr, g.col, psi0, steps,
                                                                   marked=marked))
    pref = oracle.coined_prob(g.row_ptr, g.col, ref)
    got, p, norm, pm, _ = run_coined(g, psi0, steps, dtype, layout, marked=marked)
    if dtype == "c128":
        assert np.abs(got - ref).max() < C128_TOL
        assert np.abs(p - pref).max() < C128_TOL
    else:
        assert np.linalg.norm(got - ref) < 1e-5
        assert np.abs(p - pref).max() < 1e-6
    assert abs(norm - pref.sum()) < (1e-12 if dtype == "c128" else 1e-6)
    assert abs(pm - pref[marked].sum()) < (1e-12 if dtype == "c128" else 1e-6)


@pytest.mark.parametrize("layout", ["auto", "csr", "structured"])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [64, 1001])
def test_coined_hadamard_cycle_parity(layout, dtype, n):
    g, psi0 = I.cycle_hadamard_state(n)
    ref = oracle.coined_evolve(g.row_ptr, g.col, psi0, 100, coin=oracle.HADAMARD)
    got, p, norm, _, _ = run_coined(g, psi0, 100, dtype, layout, coin="hadamard")
    tol = C128_TOL if dtype == "c128" else 1e-5
    assert np.abs(got - ref).max() < tol
    assert abs(norm - 1.0) < (1e-12 if dtype == "c128" else 1e-6)


def _two_regular(name):
    """Degree-2 graphs of at most 64 vertices (the one-workgroup kernel keeps
    them in registers of one wavefront) and graphs just outside that case."""
    if name == "union27_37":  # two cycles, labels shuffled so reverse arcs lie far apart
        perm = np.random.default_rng(4).permutation(64)
        edges = [(perm[i], perm[(i + 1) % 27]) for i in range(27)]
        edges += [(perm[27 + i], perm[27 + (i + 1) % 37]) for i in range(37)]
        return I.from_edges(64, sorted((min(a, b), max(a, b)) for a, b in edges), name=name)
    if name == "deg123":  # as many arcs as 2n, but degrees 3, 2, 2, 2, 2, 1
        return I.from_edges(6, [(0, 1), (1, 2), (2, 3), (0, 3), (0, 4), (4, 5)], name=name)
    kind, n = name.split("_")
    return I.cycle(int(n)) if kind == "dir" else I.cycle_sorted(int(n))


@pytest.mark.parametrize("name", ["dir_3", "dir_17", "sorted_40", "dir_64", "union27_37", "deg123", "dir_65"])
@pytest.mark.parametrize("coin", ["grover", "hadamard"])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_coined_two_regular_small(name, coin, dtype):
    g = _two_regular(name)
    if coin == "hadamard" and name == "deg123":
        pytest.skip("the Hadamard coin needs degree 2 everywhere")
    marked = sorted({1, g.n // 2})
    psi0 = I.random_state(g.n_arcs, seed=g.n)
    for steps in (0, 1, 37, 100):
        ref = oracle.coined_evolve(g.row_ptr, g.col, psi0, steps, marked=marked,
                                   coin=oracle.HADAMARD if coin == "hadamard" else oracle.GROVER)
        pref = oracle.coined_prob(g.row_ptr, g.col, ref)
        got, p, norm, pm, path = run_coined(g, psi0, steps, dtype, "auto", coin=coin, marked=marked)
        assert path == "small"
        if dtype == "c128":
            assert np.abs(got - ref).max() < C128_TOL
            assert np.abs(p - pref).max() < C128_TOL
        else:
            assert np.linalg.norm(got - ref) < 1e-5
            assert np.abs(p - pref).max() < 1e-6
        assert abs(norm - pref.sum()) < (1e-12 if dtype == "c128" else 1e-6)
        assert abs(pm - pref[marked].sum()) < (1e-12 if dtype == "c128" else 1e-6)


@pytest.mark.parametrize("name,coin", [("dir_64", "hadamard"), ("dir_17", "hadamard"), ("union27_37", "grover")])
def test_c64_drift_after_1e4_steps_two_regular(name, coin):
    """complex64 on the one-wavefront register path: L2 <= 1e-4 and norm drift
    <= 1e-5 against the FP64 oracle after 10^4 steps."""
    g = _two_regular(name)
    marked = [] if coin == "hadamard" else [5]
    psi0 = I.random_state(g.n_arcs, seed=3)
    steps = 10000
    ref = oracle.coined_evolve(g.row_ptr, g.col, psi0, steps, marked=marked,
                               coin=oracle.HADAMARD if coin == "hadamard" else oracle.GROVER)
    got, _, norm, _, path = run_coined(g, psi0, steps, "c64", "auto", coin=coin, marked=marked)
    assert path == "small"
    assert np.linalg.norm(got - ref) < 1e-4
    assert abs(norm - 1.0) < 1e-5


def test_cycle64_hadamard_golden():
    """The 64-cycle workload: 100 steps, c128, one-workgroup path, vs the stored values."""
    import os
    ref = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "cycle64_hadamard_100.txt"))
    g, psi0 = I.cycle_hadamard_state(64)
    _, p, _, _, structure = run_coined(g, psi0, 100, "c128", "auto", coin="hadamard")
    assert structure == "small"
    assert np.abs(p - ref).max() < C128_TOL


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("layout", ["auto", "csr", "structured"])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_ctqw_parity(name, layout, dtype):
    g = GRAPHS[name]
    marked = _marks(g)
    gamma = 1.0 / max(1, int(np.diff(g.row_ptr).max()))
    psi0 = I.random_state(g.n, seed=12)
    ref = _cached(("ctqw", name), lambda: oracle.ctqw_evolve(g.row_ptr, g.col, psi0, 7, gamma=gamma,
                                                               dt=0.2, K=12, marked=marked))
    got, p, norm, pm, _ = run_ctqw(g, psi0, 7, gamma, 0.2, 12, dtype, layout, marked=marked)
    pref = oracle.vertex_prob(ref)
    if dtype == "c128":
        assert np.abs(got - ref).max() < C128_TOL
        assert np.abs(p - pref).max() < C128_TOL
        assert abs(pm - pref[marked].sum()) < 1e-12
    else:
        assert np.linalg.norm(got - ref) < 1e-5
        assert abs(pm - pref[marked].sum()) < 1e-6
    assert abs(norm - pref.sum()) < (1e-12 if dtype == "c128" else 1e-6)


@pytest.mark.parametrize("K", [1, 2, 3, 20])
@pytest.mark.parametrize("layout", ["auto", "csr", "structured"])
def test_ctqw_orders(K, layout):
    """Odd/even and the K = 1, 2 buffer cases of the Horner chain."""
    g = I.torus(20, 23)
    psi0 = I.random_state(g.n, seed=K)
    ref = oracle.ctqw_evolve(g.row_ptr, g.col, psi0, 5, gamma=0.25, dt=0.05, K=K, marked=[7])
    got, *_ = run_ctqw(g, psi0, 5, 0.25, 0.05, K, "c128", layout, marked=[7])
    assert np.abs(got - ref).max() < C128_TOL


@pytest.mark.parametrize("l1,l2,K,dtype,depth", [
    (64, 64, 20, "c64", 5), (64, 128, 12, "c64", 4), (96, 64, 9, "c64", 3), (32, 64, 14, "c64", 2),
    (64, 64, 7, "c64", 1), (18, 100, 20, "c64", 5), (37, 201, 10, "c64", 5), (96, 32, 20, "c128", 1),
    (32, 64, 8, "c128", 4), (64, 96, 6, "c128", 3), (17, 65, 15, "c128", 5), (50, 130, 20, "c128", 5),
    (300, 64, 20, "c64", 5), (257, 130, 8, "c128", 4),
])
def test_ctqw_torus_blocked(l1, l2, K, dtype, depth):
    """Temporal blocking (S stages per launch on register-resident strips):
    strips clamped at ragged grid edges, windows that wrap the torus, the
    smallest grids a strip fits, marked vertices on strip edges and corners,
    and grids too narrow to block (one stage per launch)."""
    from paper_2406_08186_amd.walk import Plan
    g = I.torus(l1, l2)
    marked = [0, 31, 32 * l2 + 63 % l2, 8 * l2 + 53, 13 * l2 + 54, g.n - 1]
    marked = sorted(set(m for m in marked if m < g.n))
    psi0 = I.random_state(g.n, seed=l1 + l2 + K)
    ref = oracle.ctqw_evolve(g.row_ptr, g.col, psi0, 7, gamma=0.25, dt=0.07, K=K, marked=marked)
    pl = Plan(g, "ctqw", dtype=dtype, gamma=0.25, dt=0.07, taylor_order=K, marked=marked, layout="structured")
    assert pl.structure == "torus" and pl.info.block_depth == depth
    psi = pl.state(psi0)
    p, norm, pm = pl.evolve(psi, 7, readout=True)
    torch.cuda.synchronize()
    got = psi.cpu().numpy().astype(np.complex128)
    if dtype == "c128":
        assert np.abs(got - ref).max() < C128_TOL
    else:
        assert np.linalg.norm(got - ref) < 1e-5
    assert abs(float(pm) - (np.abs(ref[marked]) ** 2).sum()) < (1e-12 if dtype == "c128" else 1e-6)


@pytest.mark.parametrize("l1,l2,K,dtype,depth", [
    (64, 64, 20, "c128", 5), (50, 130, 15, "c128", 5), (64, 96, 12, "c128", 4),
    (64, 64, 20, "c64", 5), (96, 64, 15, "c64", 5), (64, 128, 12, "c64", 4),
])
def test_ctqw_torus_blocked_every_stage(l1, l2, K, dtype, depth):
    """The blocked grid sweep at rho = dt ||H||_inf = 5 (gamma 1 with marks,
    dt 1; the spectral radius of H is about 4): the Taylor terms of the
    Sec. 3.1 propagator up to k = 20 are then all far above the tolerance
    (4^20/20! = 4.5e-7), so a wrong coefficient, buffer or skipped stage in
    any launch of a time step, including the first ones (k = K..K-2S+1),
    moves the result out of it.  The order K-1 propagator is shown to
    differ from order K by more than the tolerance."""
    from paper_2406_08186_amd.walk import Plan
    g = I.torus(l1, l2)
    marked = sorted({0, 8 * l2 + 53, g.n // 2 + 7, g.n - 1})
    gamma, dt, steps = 1.0, 1.0, 3
    psi0 = I.random_state(g.n, seed=l1 * l2 + K)
    pl = Plan(g, "ctqw", dtype=dtype, gamma=gamma, dt=dt, taylor_order=K, marked=marked, layout="structured")
    assert pl.structure == "torus" and pl.info.block_depth == depth
    assert abs(pl.info.h_norm_bound * dt - 5.0) < 1e-12
    ref = oracle.ctqw_evolve(g.row_ptr, g.col, psi0, steps, gamma=gamma, dt=dt, K=K, marked=marked)
    ref_short = oracle.ctqw_evolve(g.row_ptr, g.col, psi0, steps, gamma=gamma, dt=dt, K=K - 1, marked=marked)
    psi = pl.state(psi0)
    p, norm, pm = pl.evolve(psi, steps, readout=True)
    torch.cuda.synchronize()
    got = psi.cpu().numpy().astype(np.complex128)
    if dtype == "c128":
        assert np.abs(ref - ref_short).max() > 1e3 * C128_TOL
        assert np.abs(got - ref).max() < C128_TOL
        assert abs(float(pm) - (np.abs(ref[marked]) ** 2).sum()) < 1e-12
    else:
        assert np.linalg.norm(got - ref) < 1e-5
        if K < 20:
            assert np.linalg.norm(ref - ref_short) > 10 * 1e-5


def test_zero_steps_is_readout_only():
    g = GRAPHS["rr"]
    psi0 = I.random_state(g.n_arcs, seed=3)
    for layout in ("auto", "csr"):
        got, p, norm, _, _ = run_coined(g, psi0, 0, "c128", layout)
        assert np.array_equal(got, psi0)
        assert np.abs(p - oracle.coined_prob(g.row_ptr, g.col, psi0)).max() < 1e-15


def test_empty_graph_and_isolated():
    g = I.Graph(n=0, row_ptr=np.zeros(1, np.int64), col=np.zeros(0, np.int32), name="empty")
    pl = _plan(g, "coined")
    psi = torch.zeros(0, dtype=torch.complex128, device="cuda")
    pl.evolve(psi, 5)
    torch.cuda.synchronize()
    g = I.from_edges(6, [(0, 1), (1, 2)], name="iso")  # vertices 3..5 isolated
    psi0 = I.random_state(g.n, 1)
    ref = oracle.ctqw_evolve(g.row_ptr, g.col, psi0, 9, gamma=0.5, dt=0.1, K=10, marked=[5])
    for layout in ("auto", "csr"):
        got, *_ = run_ctqw(g, psi0, 9, 0.5, 0.1, 10, "c128", layout, marked=[5])
        assert np.abs(got - ref).max() < C128_TOL


def test_deterministic_and_resumable():
    """Two runs agree bitwise; evolve(a) then evolve(b) equals evolve(a+b) bitwise."""
    from paper_2406_08186_amd.walk import Plan
    for g, kind in ((GRAPHS["er"], "coined"), (GRAPHS["hypercube"], "coined"),
                    (GRAPHS["er"], "ctqw"), (GRAPHS["torus"], "ctqw")):
        kw = dict(gamma=0.2, dt=0.1, taylor_order=10) if kind == "ctqw" else {}
        pl = Plan(g, kind, dtype="c64", marked=[1], **kw)
        psi0 = I.random_state(pl.state_len, 4)
        a = pl.state(psi0)
        pl.evolve(a, 13)
        b = pl.state(psi0)
        pl.evolve(b, 13)
        c = pl.state(psi0)
        pl.evolve(c, 6)
        pl.evolve(c, 7)
        torch.cuda.synchronize()
        assert torch.equal(a, b) and torch.equal(a, c)


# ------------------------------------------------------------- full sizes

def test_hypercube20_search_full_size():
    """Hypercube dim 20, Grover + -I at vertex 0, uniform start, ceil((pi/2) sqrt(N ln N)) steps,
    c128 against the symmetric-subspace closed form on every arc; c64 L2 and p_marked."""
    dim = 20
    n = 1 << dim
    steps = math.ceil(math.pi / 2 * math.sqrt(n * math.log(n)))
    assert steps == 5989
    g = I.hypercube(dim)
    o, i, _ = cf.hypercube_search_reduced(dim, steps)
    pm_ref = abs(o[0]) ** 2
    ref = cf.hypercube_search_state(dim, steps, g.row_ptr, g.col)
    psi0 = np.full(g.n_arcs, 1 / math.sqrt(g.n_arcs), dtype=np.complex128)
    got, p, norm, pm, structure = run_coined(g, psi0, steps, "c128", "auto", marked=[0])
    assert structure == "hypercube"
    assert np.abs(got - ref).max() < C128_TOL
    assert abs(pm - pm_ref) < 1e-12 and abs(norm - 1) < 1e-12
    del got
    got, p, norm, pm, _ = run_coined(g, psi0, steps, "c64", "auto", marked=[0])
    assert np.linalg.norm(got - ref) < 1e-4
    assert abs(norm - 1) < 1e-5 and abs(pm - pm_ref) < 1e-5


def test_torus1024_ctqw_full_size():
    """Torus 1024 x 1024, gamma 0.25, K = 20, dt = 0.1, 1000 steps from vertex (512, 512):
    every amplitude against the Kronecker product of cycle closed forms."""
    L_ = 1024
    g = I.torus(L_, L_)
    v0 = 512 * L_ + 512
    ref_1d = cf.cycle_ctqw(L_, 0.25, 100.0, 512)
    ref = np.outer(ref_1d, ref_1d).reshape(-1)
    psi0 = I.ket_vertex(g.n, v0)
    got, p, norm, pm, structure = run_ctqw(g, psi0, 1000, 0.25, 0.1, 20, "c128", "auto")
    assert structure == "torus"
    assert np.abs(got - ref).max() < C128_TOL
    assert abs(norm - 1) < 1e-12
    got, p, norm, pm, _ = run_ctqw(g, psi0, 1000, 0.25, 0.1, 20, "c64", "auto")
    assert np.linalg.norm(got - ref) < 1e-4 and abs(norm - 1) < 1e-5
    # the general CSR path on the same graph, c128
    got, *_ = run_ctqw(g, psi0, 50, 0.25, 0.1, 20, "c128", "csr")
    ref5 = np.outer(cf.cycle_ctqw(L_, 0.25, 5.0, 512), cf.cycle_ctqw(L_, 0.25, 5.0, 512)).reshape(-1)
    assert np.abs(got - ref5).max() < C128_TOL


@pytest.mark.parametrize("layout", ["auto", "csr"])
def test_c64_drift_after_1e4_steps_coined(layout):
    dim = 14
    g = I.hypercube(dim)
    steps = 10**4
    ref = cf.hypercube_search_state(dim, steps, g.row_ptr, g.col)
    psi0 = np.full(g.n_arcs, 1 / math.sqrt(g.n_arcs), dtype=np.complex128)
    got, p, norm, pm, _ = run_coined(g, psi0, steps, "c64", layout, marked=[0])
    assert np.linalg.norm(got - ref) <= 1e-4
    assert abs(norm - 1.0) <= 1e-5


@pytest.mark.parametrize("layout", ["auto", "csr"])
def test_c64_drift_after_1e4_steps_ctqw(layout):
    l1, l2 = 64, 48
    g = I.torus(l1, l2)
    v0 = 5 * l2 + 7
    steps = 10**4
    ref = cf.torus_ctqw(l1, l2, 0.25, 0.1 * steps, v0)
    got, p, norm, pm, _ = run_ctqw(g, I.ket_vertex(g.n, v0), steps, 0.25, 0.1, 20, "c64", layout)
    assert np.linalg.norm(got - ref) <= 1e-4
    assert abs(norm - 1.0) <= 1e-5


def test_complete_graph_search_reaches_one():
    """CTQW search on K_N (gamma = 1/N) reaches p_w = 1 at t = (pi/2) sqrt(N)."""
    n = 4096
    g = I.complete(n)
    t = math.pi / 2 * math.sqrt(n)
    steps = 200
    for dtype, tol in (("c128", 1e-12), ("c64", 1e-5)):
        got, p, norm, pm, _ = run_ctqw(g, I.uniform(n), steps, 1.0 / n, t / steps, 24, dtype, "auto",
                                       marked=[17])
        assert abs(pm - 1.0) < tol
