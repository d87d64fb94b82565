"""GPU parity of the staggered walk against the oracle, through the C ABI.

All engine paths are covered: the one-workgroup path (layout "auto" on
graphs whose state fits LDS), the per-tessellation polygon kernels (layout
"csr") and the fused square-lattice kernel (layout "structured", or "auto"
on lattices too large for LDS), with uniform and weighted polygons, the reflection and
Hamiltonian forms, marked vertices, thread-path polygons of one size
(column-major table) and of mixed sizes (CSR), and big polygons cut into
several chunks.  complex128 within 1e-12 (max abs), complex64 within L2 1e-5;
the readout (p, norm, p_marked) against the oracle's state.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2406_08186_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    yield
    torch.cuda.synchronize()


def _big_polygon_case():
    """6000 vertices: tessellation 1 holds one 2500-vertex polygon (two chunks)
    and pairs; tessellation 2 random polygons of 1..6 vertices."""
    rng = np.random.default_rng(17)
    perm = rng.permutation(6000)
    big = perm[:2500]
    rest = perm[2500:].reshape(-1, 2)
    t1 = I.tessellation([list(big)] + [list(x) for x in rest])
    _, (t2,) = I.stag_random(6000, 1, 6, seed=5)
    return I.union_graph(6000, [t1, t2], name="stag_big6000"), [t1, t2]


def _case(name):
    if name == "cycle64":
        return I.stag_cycle(64)
    if name == "lattice16x12":
        return I.stag_lattice(16, 12)
    if name == "arcs_mixed":
        return I.stag_arcs(I.random_mixed(40, seed=2))
    if name == "arcs_hypercube5":
        return I.stag_arcs(I.hypercube(5))
    if name == "random_w":
        return I.stag_random(700, 3, 24, seed=3, weighted=True)
    if name == "random_ham":
        g, t = I.stag_random(500, 2, 9, seed=4, weighted=True)
        t[0].theta = 0.61
        t[1].theta = -1.3
        return g, t
    if name == "big6000":
        return _big_polygon_case()
    raise KeyError(name)


CASES = ["cycle64", "lattice16x12", "arcs_mixed", "arcs_hypercube5", "random_w", "random_ham", "big6000"]


def _run(g, tess, dtype, layout, steps, marked, seed):
    from paper_2406_08186_amd.walk import Plan
    print(f"[case] staggered {g.name} n={g.n} T={len(tess)} {dtype} {layout} steps={steps}", flush=True)
    pl = Plan(g, "staggered", dtype=dtype, layout=layout, marked=marked, tessellations=tess)
    psi0 = I.random_state(g.n, seed)
    psi = pl.state(psi0)
    p, norm, pm = pl.evolve(psi, steps, readout=True)
    torch.cuda.synchronize()
    return pl, psi0, psi.cpu().numpy().astype(np.complex128), p.cpu().numpy(), float(norm), float(pm)


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("layout", ["auto", "csr"])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_staggered_matches_oracle(name, layout, dtype):
    g, tess = _case(name)
    marked = [1, g.n // 2] if g.n > 4 else []
    steps = 23
    pl, psi0, got, p, norm, pm = _run(g, tess, dtype, layout, steps, marked, seed=7)
    assert pl.structure == ("small" if layout == "auto" and g.n * (16 if dtype == "c128" else 8) <= 156 * 1024
                            else "general")
    ref = oracle.staggered_evolve(g.n, tess, psi0, steps, marked=marked)
    if dtype == "c128":
        assert np.abs(got - ref).max() < 1e-12
        assert np.abs(p - np.abs(ref) ** 2).max() < 1e-12
        assert abs(norm - 1.0) < 1e-12
    else:
        assert np.linalg.norm(got - ref) < 1e-5
        assert np.abs(p - np.abs(got) ** 2).max() < 1e-6
        assert abs(norm - 1.0) < 1e-5
    assert abs(pm - p[marked].sum()) < 1e-12


@pytest.mark.parametrize("layout", ["auto", "csr"])
def test_staggered_zero_steps_and_readout_only(layout):
    from paper_2406_08186_amd.walk import Plan
    g, tess = I.stag_lattice(8, 8)
    pl = Plan(g, "staggered", dtype="c128", layout=layout, marked=[3], tessellations=tess)
    psi0 = I.random_state(g.n, 2)
    psi = pl.state(psi0)
    p, norm, pm = pl.evolve(psi, 0, readout=True)
    torch.cuda.synchronize()
    assert np.array_equal(psi.cpu().numpy(), psi0)
    assert np.abs(p.cpu().numpy() - np.abs(psi0) ** 2).max() < 1e-15
    p2, norm2, pm2 = pl.probabilities(psi)
    assert abs(float(pm2) - abs(psi0[3]) ** 2) < 1e-15


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_staggered_paths_agree_and_repeat_bitwise(dtype):
    """The same walk on both paths agrees to rounding; each path repeats bitwise."""
    from paper_2406_08186_amd.walk import Plan
    g, tess = I.stag_random(900, 3, 30, seed=12, weighted=True)
    psi0 = I.random_state(g.n, 5)
    out = {}
    for layout in ("auto", "csr"):
        pl = Plan(g, "staggered", dtype=dtype, layout=layout, marked=[4], tessellations=tess)
        runs = []
        for _ in range(2):
            x = pl.state(psi0)
            pl.evolve(x, 40)
            torch.cuda.synchronize()
            runs.append(x.cpu().numpy())
        assert np.array_equal(runs[0], runs[1])
        out[layout] = runs[0].astype(np.complex128)
    assert np.linalg.norm(out["auto"] - out["csr"]) < (1e-12 if dtype == "c128" else 1e-5)


def test_staggered_arc_walk_equals_engine_coined_walk():
    """Star and pair tessellations of a graph's arcs on the engine give the
    engine's own Grover coined walk (different kernels, same operator)."""
    from paper_2406_08186_amd.walk import Plan
    h = I.random_regular(3000, 5, seed=8)
    sg, tess = I.stag_arcs(h)
    psi0 = I.random_state(h.n_arcs, 3)
    st = Plan(sg, "staggered", dtype="c128", layout="csr", tessellations=tess)
    co = Plan(h, "coined", dtype="c128", layout="csr")
    a, b = st.state(psi0), co.state(psi0)
    st.evolve(a, 30)
    co.evolve(b, 30)
    torch.cuda.synchronize()
    assert np.abs(a.cpu().numpy() - b.cpu().numpy()).max() < 1e-12


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_staggered_lattice_full_size(dtype):
    """The benchmark's 1024 x 1024 square-lattice walk (two tessellations of
    2 x 2 squares, one marked vertex), whole state against the oracle."""
    g, tess = I.stag_lattice(1024)
    marked = [1024 * 512 + 512]
    steps = 12
    pl, psi0, got, p, norm, pm = _run(g, tess, dtype, "auto", steps, marked, seed=1)
    assert pl.structure == "stag_lattice"
    ref = oracle.staggered_evolve(g.n, tess, psi0, steps, marked=marked)
    if dtype == "c128":
        assert np.abs(got - ref).max() < 1e-12
    else:
        assert np.linalg.norm(got - ref) < 1e-4
    assert abs(norm - 1.0) < (1e-12 if dtype == "c128" else 1e-5)


@pytest.mark.parametrize("layout", ["csr", "structured"])
def test_staggered_lattice_search_long_run_c64(layout):
    """complex64 norm drift after 10^4 steps of the lattice search stays
    within 1e-5; the state matches complex128 within L2 1e-4."""
    from paper_2406_08186_amd.walk import Plan
    g, tess = I.stag_lattice(64)
    marked = [64 * 20 + 33]
    psi0 = I.uniform(g.n)
    out = {}
    for dtype in ("c64", "c128"):
        pl = Plan(g, "staggered", dtype=dtype, layout=layout, marked=marked, tessellations=tess)
        x = pl.state(psi0)
        _, norm, _ = pl.evolve(x, 10000, readout=True)
        torch.cuda.synchronize()
        out[dtype] = (x.cpu().numpy().astype(np.complex128), float(norm))
    assert abs(out["c64"][1] - 1.0) < 1e-5
    assert np.linalg.norm(out["c64"][0] - out["c128"][0]) < 1e-4


def test_staggered_in_many_small_walks():
    """qw_small_many runs staggered walks beside CTQW and coined ones, with
    results bitwise those of evolve on each plan."""
    from paper_2406_08186_amd.walk import Plan, evolve_many
    specs = [("stag", I.stag_lattice(8, 6)), ("ctqw", I.cycle(50)), ("stag", I.stag_random(300, 2, 20, seed=2)),
             ("coined", I.hypercube(5)), ("stag", I.stag_arcs(I.complete(6)))]
    plans, states, ref, steps = [], [], [], []
    for i, (kind, spec) in enumerate(specs):
        if kind == "stag":
            g, tess = spec
            pl = Plan(g, "staggered", dtype="c128", marked=[0], tessellations=tess)
        elif kind == "ctqw":
            pl = Plan(spec, "ctqw", dtype="c128", gamma=0.5, dt=0.2, taylor_order=8, marked=[0])
        else:
            pl = Plan(spec, "coined", dtype="c128", marked=[0])
        assert pl.structure == "small"
        psi0 = I.random_state(pl.state_len, i)
        x, y = pl.state(psi0), pl.state(psi0)
        n = 11 + 3 * i
        pl.evolve(y, n)
        plans.append(pl)
        states.append(x)
        ref.append(y)
        steps.append(n)
    keep = evolve_many(plans, states, steps)
    torch.cuda.synchronize()
    del keep
    for x, y in zip(states, ref):
        assert torch.equal(x, y)


def test_staggered_cannot_join_a_batch():
    from paper_2406_08186_amd import _lib as L
    from paper_2406_08186_amd.walk import Batch, Plan
    g, tess = I.stag_cycle(40)
    pl = Plan(g, "staggered", dtype="c64", layout="csr", tessellations=tess)
    b = Batch(capacity=2, max_tiles=64, dtype="c64")
    with pytest.raises(L.QwError) as e:
        b.set_slot(0, pl, pl.state(I.uniform(40)), 5)
    assert e.value.code == L.QW_EUNSUPPORTED
    b.close()


def test_hamiltonian_quarter_turn_on_engine():
    """theta = pi/2 is i times the reflection, step by step, on the engine."""
    from paper_2406_08186_amd.walk import Plan
    g, tess = I.stag_random(5000, 2, 12, seed=21, weighted=True)
    ham = [I.Tessellation(t.poly_ptr, t.poly_vert, t.amp, math.pi / 2) for t in tess]
    psi0 = I.random_state(g.n, 8)
    a = Plan(g, "staggered", dtype="c128", layout="csr", tessellations=tess)
    b = Plan(g, "staggered", dtype="c128", layout="csr", tessellations=ham)
    x, y = a.state(psi0), b.state(psi0)
    a.evolve(x, 7)
    b.evolve(y, 7)
    torch.cuda.synchronize()
    assert np.abs((1j) ** 14 * x.cpu().numpy() - y.cpu().numpy()).max() < 1e-12


LATTICES = [(4, 4), (6, 8), (16, 64), (18, 66), (34, 130), (100, 62), (4, 200)]


@pytest.mark.parametrize("l1,l2", LATTICES)
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("form", ["reflection", "hamiltonian"])
def test_square_lattice_kernel_matches_oracle(l1, l2, dtype, form):
    """The fused index-free kernels (both tessellations of a step in one
    launch, tiles of 16 x 64 with a periodic halo; two steps per launch with
    a four-cell halo, an odd last step alone): lattices smaller than one tile
    (staged vertices repeat), ragged tiles in both directions, marked
    vertices on tile edges and corners, both forms."""
    from paper_2406_08186_amd.walk import Plan
    g, tess = I.stag_lattice(l1, l2)
    if form == "hamiltonian":
        tess = [I.Tessellation(tess[0].poly_ptr, tess[0].poly_vert, None, 0.83),
                I.Tessellation(tess[1].poly_ptr, tess[1].poly_vert, None, -0.41)]
    marked = sorted({0, l2 - 1, 15 * l2 % g.n, (16 * l2 + 63) % g.n, g.n - 1})
    print(f"[case] stag lattice {l1}x{l2} {dtype} {form}", flush=True)
    pl = Plan(g, "staggered", dtype=dtype, layout="structured", marked=marked, tessellations=tess)
    assert pl.structure == "stag_lattice"
    psi0 = I.random_state(g.n, l1 + l2)
    for steps in (0, 1, 3, 8):  # one-step and two-step launches
        x = pl.state(psi0)
        p, norm, pm = pl.evolve(x, steps, readout=True)
        torch.cuda.synchronize()
        got = x.cpu().numpy().astype(np.complex128)
        ref = oracle.staggered_evolve(g.n, tess, psi0, steps, marked=marked)
        if dtype == "c128":
            assert np.abs(got - ref).max() < 1e-12, steps
            assert np.abs(p.cpu().numpy() - np.abs(ref) ** 2).max() < 1e-12
        else:
            assert np.linalg.norm(got - ref) < 1e-5, steps
        assert abs(float(pm) - float(p.cpu().numpy()[marked].sum())) < 1e-12


def test_square_lattice_kernel_agrees_with_polygon_kernels_and_repeats():
    from paper_2406_08186_amd.walk import Plan
    g, tess = I.stag_lattice(258, 130)
    psi0 = I.random_state(g.n, 9)
    out = {}
    for layout in ("structured", "csr"):
        pl = Plan(g, "staggered", dtype="c128", layout=layout, marked=[7, 1000], tessellations=tess)
        runs = []
        for _ in range(2):
            x = pl.state(psi0)
            pl.evolve(x, 33)
            torch.cuda.synchronize()
            runs.append(x.cpu().numpy())
        assert np.array_equal(runs[0], runs[1])
        out[pl.structure] = runs[0]
    assert np.abs(out["stag_lattice"] - out["general"]).max() < 1e-12


def test_staggered_class_simulate_and_distributions():
    """The paper-style surface: simulate(range=...) snapshots, their FP64
    distributions, and the host-streamed snapshots, on the lattice kernel."""
    from paper_2406_08186_amd.walk import Staggered
    g, tess = I.stag_lattice(40, 132)
    w = Staggered(g, tess, marked=[5, 700], dtype="c128", layout="structured")
    assert w.plan.structure == "stag_lattice"
    psi0 = I.random_state(g.n, 1)
    idx = list(range(0, 9, 3))
    states = w.simulate(range=(0, 9, 3), state=psi0)
    dists = w.probability_distribution(states)
    host = w.simulate_host(range=(0, 9, 3), state=psi0)
    for k, s, d, h in zip(idx, states, dists, host):
        ref = oracle.staggered_evolve(g.n, tess, psi0, k, marked=[5, 700])
        assert np.abs(s.cpu().numpy() - ref).max() < 1e-12
        assert np.abs(d.cpu().numpy() - np.abs(ref) ** 2).max() < 1e-12
        assert np.array_equal(h, s.cpu().numpy())
    assert np.array_equal(w.ket(3), I.ket_vertex(g.n, 3))
