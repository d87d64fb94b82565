"""GPU tests of batched execution (qw_batch_*): every walk's result in a mixed
batch equals the same walk run alone (bitwise), the plain single-walk path
(to rounding) and the FP64 oracle (c128 within 1e-12)."""
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


def _walks(dtype):
    """(graph, kind, params, steps) of a ragged mix."""
    return [
        (I.random_regular(500, 3, seed=1), "ctqw", dict(gamma=1 / 3, dt=0.3, taylor_order=14, marked=[7],
                                                       layout="structured"), 9),
        (I.random_regular(1200, 5, seed=2), "ctqw", dict(gamma=0.2, dt=0.5, taylor_order=16, marked=[0]), 5),
        (I.random_regular(3001 + 1, 7, seed=12), "ctqw", dict(gamma=1 / 7, dt=0.2, taylor_order=12, marked=[5],
                                                             layout="structured"), 6),
        (I.random_regular(700, 12, seed=13), "ctqw", dict(gamma=1 / 12, dt=0.2, taylor_order=10, marked=[9],
                                                         layout="structured"), 4),
        (I.random_regular(2000, 8, seed=3), "ctqw", dict(gamma=0.125, dt=0.4, taylor_order=12, marked=[1999]), 12),
        (I.erdos_renyi(1500, 6 / 1499, seed=4), "ctqw", dict(gamma=0.2, dt=0.25, taylor_order=10, marked=[3]), 7),
        (I.cycle(300), "coined", dict(coin="hadamard"), 31),
        (I.erdos_renyi(900, 8 / 899, seed=5), "coined", dict(coin="grover", marked=[2]), 24),
        (I.hypercube(9), "coined", dict(coin="grover", marked=[0]), 17),
        (I.random_regular(4000, 4, seed=6), "coined", dict(coin="grover", marked=[11]), 10),
    ]


def _plan(g, kind, params, dtype):
    from paper_2406_08186_amd.walk import Plan
    params = dict(params)
    layout = params.pop("layout", "csr")
    return Plan(g, kind, dtype=dtype, layout=layout, **params)


def _psi0(pl, seed):
    return I.random_state(pl.state_len, seed)


def _run_batch(entries, dtype, schedule=None, autotune=False):
    from paper_2406_08186_amd.walk import Batch
    b = Batch(capacity=max(8, len(entries)), max_tiles=8192, dtype=dtype)
    states = []
    for slot, (pl, psi0, steps) in enumerate(entries):
        psi = pl.state(psi0)
        b.set_slot(slot, pl, psi, steps)
        states.append(psi)
    if schedule:
        b.set_schedule(*schedule)
    b.commit()
    if autotune:
        b.autotune(reps=2)
    b.run_to_completion()
    outs = []
    for slot in range(len(entries)):
        p, norm, pm = b.readout(slot)
        outs.append((states[slot].clone(), p.clone(), float(norm), float(pm)))
    torch.cuda.synchronize()
    b.close()
    return outs


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_alone_vs_mix_and_oracle(dtype):
    walks = _walks(dtype)
    print(f"[case] batch mix {dtype} walks={len(walks)}", flush=True)
    entries = []
    for i, (g, kind, params, steps) in enumerate(walks):
        pl = _plan(g, kind, params, dtype)
        entries.append((pl, _psi0(pl, 100 + i), steps))
    mixed = _run_batch(entries, dtype)
    for i, (pl, psi0, steps) in enumerate(entries):
        alone = _run_batch([(pl, psi0, steps)], dtype)[0]
        assert torch.equal(alone[0], mixed[i][0]), f"walk {i} differs alone vs in the mix"
        assert torch.equal(alone[1], mixed[i][1])
        g, kind, params, _ = walks[i]
        if kind == "ctqw":
            assert pl.structure == ("ell" if params.get("layout") == "structured" else "general")
            ref = oracle.ctqw_evolve(g.row_ptr, g.col, psi0, steps, gamma=params["gamma"], dt=params["dt"],
                                     K=params["taylor_order"], marked=params["marked"])
            pref = oracle.vertex_prob(ref)
        else:
            ref = oracle.coined_evolve(g.row_ptr, g.col, psi0, steps,
                                       coin=oracle.HADAMARD if params["coin"] == "hadamard" else oracle.GROVER,
                                       marked=params.get("marked", ()))
            pref = oracle.coined_prob(g.row_ptr, g.col, ref)
        got = mixed[i][0].cpu().numpy().astype(np.complex128)
        if dtype == "c128":
            assert np.abs(got - ref).max() < 1e-12, i
            assert np.abs(mixed[i][1].cpu().numpy() - pref).max() < 1e-12
        else:
            assert np.linalg.norm(got - ref) < 1e-5, i
        # the plain single-walk path agrees to rounding
        plain = pl.state(psi0)
        pl.evolve(plain, steps)
        torch.cuda.synchronize()
        tol = 1e-13 if dtype == "c128" else 1e-6
        assert (plain - mixed[i][0]).abs().max().item() < tol, i


def test_batch_continuous_join_and_schedules():
    """A walk that joins mid-run, or runs under another schedule, gives the same bits."""
    from paper_2406_08186_amd.walk import Batch
    dtype = "c64"
    walks = _walks(dtype)
    pls = [_plan(g, kind, params, dtype) for g, kind, params, _ in walks]
    late = 7
    ref = _run_batch([(pls[late], _psi0(pls[late], 7), walks[late][3])], dtype)[0]
    b = Batch(capacity=8, max_tiles=8192, dtype=dtype)
    keep = []
    for slot, wi in enumerate((0, 1, 6)):
        psi = pls[wi].state(_psi0(pls[wi], 50 + wi))
        keep.append(psi)
        b.set_slot(slot, pls[wi], psi, walks[wi][3])
    b.commit()
    b.run(23)  # replay path (>= 16) plus single launches
    psi = pls[late].state(_psi0(pls[late], 7))
    b.set_slot(5, pls[late], psi, walks[late][3])
    b.commit()
    assert b.remaining(5) == walks[late][3]
    b.run_to_completion()
    b.readout(5)
    torch.cuda.synchronize()
    assert torch.equal(psi, ref[0])
    for sched in ((256, False), (4096, True)):
        out = _run_batch([(pls[late], _psi0(pls[late], 7), walks[late][3])], dtype, schedule=sched)[0]
        assert torch.equal(out[0], ref[0])
    b.close()


def test_batch_autotune_keeps_results():
    dtype = "c64"
    walks = _walks(dtype)[:4]
    entries = []
    for i, (g, kind, params, steps) in enumerate(walks):
        pl = _plan(g, kind, params, dtype)
        entries.append((pl, _psi0(pl, 200 + i), steps))
    base = _run_batch(entries, dtype)
    tuned = _run_batch(entries, dtype, autotune=True)
    for a, t in zip(base, tuned):
        assert torch.equal(a[0], t[0])


def test_batch_marked_history():
    """CTQW search: p_marked after every step, recorded on the device, equals the oracle's."""
    from paper_2406_08186_amd.walk import Batch
    g = I.random_regular(800, 4, seed=9)
    params = dict(gamma=0.25, dt=0.5, taylor_order=16, marked=[17])
    steps = 30
    pl = _plan(g, "ctqw", params, "c128")
    b = Batch(capacity=2, max_tiles=1024, dtype="c128")
    psi = pl.state(I.uniform(g.n))
    hist = torch.zeros(steps, dtype=torch.float64, device="cuda")
    b.set_slot(0, pl, psi, steps, hist=hist)
    b.commit()
    b.run_to_completion()
    torch.cuda.synchronize()
    x = I.uniform(g.n)
    for s in range(steps):
        x = oracle.ctqw_evolve(g.row_ptr, g.col, x, 1, gamma=0.25, dt=0.5, K=16, marked=[17])
        assert abs(hist[s].item() - abs(x[17]) ** 2) < 1e-12
    b.close()


def test_batch_errors():
    from paper_2406_08186_amd import _lib as L
    from paper_2406_08186_amd.walk import Batch, Plan
    b = Batch(capacity=2, max_tiles=64, dtype="c64")
    g = I.torus(20, 20)
    auto = Plan(g, "ctqw", dtype="c64", gamma=0.25, dt=0.1, taylor_order=8, layout="structured")
    with pytest.raises(L.QwError) as e:
        b.set_slot(0, auto, auto.state(I.uniform(g.n)), 3)
    assert e.value.code == L.QW_EUNSUPPORTED
    p128 = Plan(g, "ctqw", dtype="c128", gamma=0.25, dt=0.1, taylor_order=8, layout="csr")
    with pytest.raises(L.QwError) as e:
        L.qw_batch_set_slot(b._b, 0, p128._plan, p128.state(I.uniform(g.n)).data_ptr(),
                            p128.work.data_ptr(), p128.work.numel(), 3, None)
    assert e.value.code == L.QW_EINVAL
    k1 = Plan(g, "ctqw", dtype="c64", gamma=0.25, dt=0.1, taylor_order=1, layout="csr")
    with pytest.raises(L.QwError) as e:
        b.set_slot(0, k1, k1.state(I.uniform(g.n)), 3)
    assert e.value.code == L.QW_EUNSUPPORTED
    ok = Plan(g, "ctqw", dtype="c64", gamma=0.25, dt=0.1, taylor_order=8, layout="csr")
    b.set_slot(1, ok, ok.state(I.uniform(g.n)), 3)
    b.commit()
    with pytest.raises(L.QwError) as e:
        b.readout(1)
    assert e.value.code == L.QW_ESTATE
    big = I.random_regular(20000, 4, seed=1)
    pb = Plan(big, "ctqw", dtype="c64", gamma=0.25, dt=0.1, taylor_order=8, layout="csr")
    b.set_slot(0, pb, pb.state(I.uniform(big.n)), 3)
    b.set_schedule(64, True)
    with pytest.raises(L.QwError) as e:
        b.commit()
    assert e.value.code == L.QW_ENOMEM
    b.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_structured_coined(dtype):
    """Coined walks on slot-major (index-free) plans inside a batch, mixed with CSR and
    ELL walks: bitwise equal alone and in the mix, equal to the oracle."""
    walks = [
        (I.hypercube(10), "coined", dict(coin="grover", marked=[0], layout="structured"), 21),
        (I.torus(24, 30), "coined", dict(coin="grover", marked=[5, 700], layout="structured"), 16),
        (I.cycle(301), "coined", dict(coin="hadamard", layout="structured"), 33),
        (I.hypercube(6), "coined", dict(coin="grover", layout="structured"), 8),
        (I.erdos_renyi(900, 8 / 899, seed=5), "coined", dict(coin="grover", marked=[2]), 11),
        (I.random_regular(1000, 5, seed=8), "ctqw", dict(gamma=0.2, dt=0.3, taylor_order=12, marked=[4],
                                                        layout="structured"), 6),
    ]
    print(f"[case] batch structured coined {dtype}", flush=True)
    entries = []
    for i, (g, kind, params, steps) in enumerate(walks):
        pl = _plan(g, kind, params, dtype)
        entries.append((pl, _psi0(pl, 300 + i), steps))
    assert [e[0].structure for e in entries[:4]] == ["hypercube", "torus", "cycle", "hypercube"]
    mixed = _run_batch(entries, dtype)
    for i, (pl, psi0, steps) in enumerate(entries):
        alone = _run_batch([(pl, psi0, steps)], dtype)[0]
        assert torch.equal(alone[0], mixed[i][0]), i
        assert torch.equal(alone[1], mixed[i][1]), i
        g, kind, params, _ = walks[i]
        if kind == "coined":
            ref = oracle.coined_evolve(g.row_ptr, g.col, psi0, steps,
                                       coin=oracle.HADAMARD if params["coin"] == "hadamard" else oracle.GROVER,
                                       marked=params.get("marked", ()))
            pref = oracle.coined_prob(g.row_ptr, g.col, ref)
        else:
            ref = oracle.ctqw_evolve(g.row_ptr, g.col, psi0, steps, gamma=params["gamma"], dt=params["dt"],
                                     K=params["taylor_order"], marked=params["marked"])
            pref = oracle.vertex_prob(ref)
        got = mixed[i][0].cpu().numpy().astype(np.complex128)
        if dtype == "c128":
            assert np.abs(got - ref).max() < 1e-12, i
            assert np.abs(mixed[i][1].cpu().numpy() - pref).max() < 1e-12, i
        else:
            assert np.linalg.norm(got - ref) < 1e-5, i


def _relabelled(n, edges, seed, name):
    """A graph with its vertices relabelled by a seeded permutation (no structure to recognise)."""
    perm = np.random.default_rng(seed).permutation(n)
    e = perm[np.asarray(edges, dtype=np.int64)]
    return I.from_edges(n, np.sort(e, axis=1), name=name)


def _lds_walks():
    """CTQW walks on regular graphs of degree 1..8 (the LDS-staged kernel), sized around its
    tiles (6912 complex64 / 6144 complex128 rows) and blocks (19968 / 9216 entries, and
    18432) edges, marks on those edges, odd and even n (complex64 stages pairs of entries with 16-byte loads, so an
    odd n leaves a last entry alone; the tiniest walks have 4 and 7 vertices); the largest
    also exceeds the size from which the single-walk path gathers in column slices
    (7.5 MiB)."""
    m = 6000
    matching = _relabelled(m, [(2 * i, 2 * i + 1) for i in range(m // 2)], 21, "matching")
    ring = _relabelled(9001, [(i, (i + 1) % 9001) for i in range(9001)], 22, "ring")

    def cyc(n, seed):
        return _relabelled(n, [(i, (i + 1) % n) for i in range(n)], seed, f"ring{n}")
    return [
        (_relabelled(4, [(0, 1), (2, 3)], 23, "edges2"), dict(gamma=1.0, dt=0.4, taylor_order=10, marked=[1]), 6),
        (_relabelled(7, [(0, 1), (1, 2), (2, 0), (3, 4), (4, 5), (5, 6), (6, 3)], 24, "tri_sq"),
         dict(gamma=0.5, dt=0.3, taylor_order=12, marked=[6]), 6),
        (cyc(6145, 25), dict(gamma=0.5, dt=0.3, taylor_order=12, marked=[6144]), 5),
        (cyc(16385, 26), dict(gamma=0.5, dt=0.3, taylor_order=12, marked=[16384]), 4),
        (I.random_regular(12289, 4, seed=39), dict(gamma=0.25, dt=0.4, taylor_order=13, marked=[12288]), 4),
        (cyc(18433, 27), dict(gamma=0.5, dt=0.3, taylor_order=12, marked=[18432]), 4),
        (cyc(19969, 28), dict(gamma=0.5, dt=0.3, taylor_order=12, marked=[19968]), 4),
        (I.random_regular(6914, 3, seed=43), dict(gamma=1 / 3, dt=0.5, taylor_order=12, marked=[6912]), 4),
        (I.random_regular(9218, 3, seed=40), dict(gamma=1 / 3, dt=0.5, taylor_order=12, marked=[9216]), 4),
        (I.random_regular(36865, 4, seed=42), dict(gamma=0.25, dt=0.4, taylor_order=12, marked=[36864]), 3),
        (matching, dict(gamma=1.0, dt=0.4, taylor_order=10, marked=[4095]), 5),
        (ring, dict(gamma=0.5, dt=0.3, taylor_order=12, marked=[8191]), 7),
        (I.random_regular(4096, 3, seed=31), dict(gamma=1 / 3, dt=0.5, taylor_order=14, marked=[4095]), 6),
        (I.random_regular(4097 + 1, 5, seed=32), dict(gamma=0.2, dt=0.5, taylor_order=14, marked=[4096]), 5),
        (I.random_regular(16384, 4, seed=33), dict(gamma=0.25, dt=0.4, taylor_order=13, marked=[16383]), 4),
        (I.random_regular(16386, 6, seed=34), dict(gamma=1 / 6, dt=0.5, taylor_order=12, marked=[16384]), 4),
        (I.random_regular(40001 + 1, 7, seed=35), dict(gamma=1 / 7, dt=0.5, taylor_order=14, marked=[32768]), 3),
        (I.random_regular(1000, 8, seed=36), dict(gamma=0.125, dt=0.5, taylor_order=2, marked=[999]), 9),
        (I.random_regular(200000, 8, seed=37), dict(gamma=0.125, dt=0.5, taylor_order=12, marked=[123456]), 2),
        # vectors above 7.5 MiB: the single-walk path takes the column-sliced ELL stage
        (I.random_regular(1000000, 6, seed=38), dict(gamma=1 / 6, dt=0.5, taylor_order=11, marked=[999999]), 2),
    ]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_lds_kernel(dtype):
    """The LDS-staged kernel on ragged tiles and blocks: bitwise equal to the gather kernel, to the
    walk alone in the batch, and to the single-walk path; equal to the FP64 oracle."""
    walks = _lds_walks()
    entries = []
    for i, (g, params, steps) in enumerate(walks):
        pl = _plan(g, "ctqw", dict(params, layout="structured"), dtype)
        assert pl.structure == "ell", (i, pl.structure)
        entries.append((pl, _psi0(pl, 400 + i), steps))
    print(f"[case] batch lds kernel {dtype} walks={len(walks)}", flush=True)
    from paper_2406_08186_amd.walk import Batch

    def run(kernel, ents):
        b = Batch(capacity=len(ents), max_tiles=16384, dtype=dtype)
        b.set_stage_kernel(kernel)
        states = []
        for slot, (pl, psi0, steps) in enumerate(ents):
            psi = pl.state(psi0)
            b.set_slot(slot, pl, psi, steps)
            states.append(psi)
        b.commit()
        assert b.schedule()["stage_kernel"] == kernel
        b.run_to_completion()
        outs = []
        for slot in range(len(ents)):
            p, norm, pm = b.readout(slot)
            outs.append((states[slot].clone(), p.clone(), float(norm), float(pm)))
        torch.cuda.synchronize()
        b.close()
        return outs

    lds = run("lds", entries)
    gat = run("gather", entries)
    for i, (pl, psi0, steps) in enumerate(entries):
        assert torch.equal(lds[i][0], gat[i][0]), f"walk {i}: LDS-staged and gather kernels differ"
        assert torch.equal(lds[i][1], gat[i][1]), i
        alone = run("lds", [entries[i]])[0]
        assert torch.equal(alone[0], lds[i][0]), f"walk {i} differs alone vs in the mix"
        plain = pl.state(psi0)
        pl.evolve(plain, steps)
        torch.cuda.synchronize()
        assert torch.equal(plain, lds[i][0]), f"walk {i}: single-walk path differs"
        g, params, _ = walks[i]
        ref = oracle.ctqw_evolve(g.row_ptr, g.col, psi0, steps, gamma=params["gamma"], dt=params["dt"],
                                 K=params["taylor_order"], marked=params["marked"])
        got = lds[i][0].cpu().numpy().astype(np.complex128)
        if dtype == "c128":
            assert np.abs(got - ref).max() < 1e-12, i
            assert np.abs(lds[i][1].cpu().numpy() - oracle.vertex_prob(ref)).max() < 1e-12, i
        else:
            assert np.linalg.norm(got - ref) < 1e-5, i
        assert abs(lds[i][2] - float(np.sum(np.abs(got) ** 2))) < 1e-6


def test_batch_lds_history_and_probe():
    """p_marked history from the LDS-staged kernel equals the oracle's, and the autotuner's
    probe launches leave states and the launch counter untouched."""
    from paper_2406_08186_amd.walk import Batch
    g = I.random_regular(20000, 6, seed=41)
    params = dict(gamma=1 / 6, dt=0.5, taylor_order=14, marked=[19999])
    steps = 12
    pl = _plan(g, "ctqw", dict(params, layout="structured"), "c128")
    b = Batch(capacity=2, max_tiles=1024, dtype="c128")
    psi = pl.state(I.uniform(g.n))
    hist = torch.zeros(steps, dtype=torch.float64, device="cuda")
    b.set_slot(0, pl, psi, steps, hist=hist)
    b.commit()
    b.autotune(reps=1)
    assert b.launches == 0 and b.remaining(0) == steps * 14
    torch.cuda.synchronize()
    assert torch.equal(psi, pl.state(I.uniform(g.n)))
    b.run_to_completion()
    torch.cuda.synchronize()
    x = I.uniform(g.n)
    for s in range(steps):
        x = oracle.ctqw_evolve(g.row_ptr, g.col, x, 1, K=14, gamma=params["gamma"], dt=params["dt"],
                               marked=params["marked"])
        assert abs(hist[s].item() - abs(x[19999]) ** 2) < 1e-12, s
    b.close()
