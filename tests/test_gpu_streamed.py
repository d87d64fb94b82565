"""GPU tests of out-of-core evolution (qw_plan_upload_streamed): the CSR
neighbour table in pinned host memory, either read by the stage kernel itself
with a device-resident prefix (direct mode) or streamed through a device ring
at every Horner stage (ring mode), under forced small device budgets.
Results equal the FP64 oracle (c128 within 1e-12, c64 L2 within 1e-5) and
are bitwise the same for every budget and both modes."""
import numpy as np
import pytest
import torch

import oracle
from paper_2406_08186_amd import _lib as L
from paper_2406_08186_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    yield
    torch.cuda.synchronize()


def _graphs():
    return [
        (I.erdos_renyi(3000, 8 / 2999, seed=4), dict(gamma=0.125, dt=0.5, taylor_order=12, marked=[17]), 6),
        # a hub of degree 696: gamma and dt keep rho = dt ||H||_inf below 1
        (I.random_mixed(700, seed=3), dict(gamma=0.002, dt=0.4, taylor_order=10, marked=[0, 5]), 9),
        (I.random_regular(20000, 5, seed=6), dict(gamma=0.2, dt=0.5, taylor_order=14, marked=[19999]), 3),
    ]


def _plan(g, params, dtype):
    from paper_2406_08186_amd.walk import Plan
    return Plan(g, "ctqw", dtype=dtype, layout="csr", upload=False, **params)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_streamed_matches_oracle_for_every_budget(dtype):
    for gi, (g, params, steps) in enumerate(_graphs()):
        psi0 = I.random_state(g.n, 60 + gi)
        ref = oracle.ctqw_evolve(g.row_ptr, g.col, psi0, steps, gamma=params["gamma"], dt=params["dt"],
                                 K=params["taylor_order"], marked=params["marked"])
        pref = oracle.vertex_prob(ref)
        first = None
        cases = [("ring", e) for e in (1 << 30, 8 * g.n + 64 * 1024, 8 * g.n + 16 * 1024)]
        cases += [("direct", e) for e in (1 << 30, 8 * g.n + 4 * g.n_arcs // 3, 8 * g.n + 16 * 1024, 0)]
        for mode, extra in cases:
            pl = _plan(g, params, dtype)
            walk = pl.info.state_bytes + pl.info.work_bytes
            if extra == 0:  # about the smallest direct budget: a prefix of at most 128 arcs on the device
                extra = L.qw_plan_stream_sizes(pl._plan, 1 << 40, L.QW_STREAM_DIRECT)[1] - 16 * ((g.n_arcs + 3) // 4)
                extra = (extra + 255) // 256 * 256 + 256
            sizes = pl.upload_streamed(walk + extra, mode=mode)
            assert sizes["host_bytes"] == (4 * g.n_arcs if mode == "ring" else 16 * ((g.n_arcs + 3) // 4))
            print(f"[case] streamed {mode} {dtype} graph {gi} n={g.n} tiles={sizes['tiles']} "
                  f"device_arcs={sizes['device_arcs']}", flush=True)
            psi = pl.state(psi0)
            p, norm, pm = pl.evolve(psi, steps, readout=True)
            torch.cuda.synchronize()
            got = psi.cpu().numpy().astype(np.complex128)
            if dtype == "c128":
                assert np.abs(got - ref).max() < 1e-12, (gi, extra)
                assert np.abs(p.cpu().numpy() - pref).max() < 1e-12
                assert abs(float(pm) - pref[params["marked"]].sum()) < 1e-12
            else:
                assert np.linalg.norm(got - ref) < 1e-5, (gi, extra)
            assert abs(float(norm) - float(np.sum(np.abs(got) ** 2))) < 1e-9
            if first is None:
                first = (sizes["tiles"], psi.clone())
                assert first[0] == 1
            else:
                assert torch.equal(psi, first[1]), f"graph {gi}: {mode} {sizes['tiles']} tiles"
            pl.close()


def test_streamed_small_ring_many_tiles_and_rebinding():
    """A budget whose slots hold little more than the largest row (hundreds of tiles per
    stage), K = 1 and zero steps, then a plain upload of the same plan: same results."""
    g = I.erdos_renyi(5000, 12 / 4999, seed=8)
    params = dict(gamma=1 / 12, dt=0.25, taylor_order=16, marked=[4999])
    psi0 = I.random_state(g.n, 9)
    pl = _plan(g, params, "c128")
    walk = pl.info.state_bytes + pl.info.work_bytes
    resident = 4 * (g.n + 1) + 4 * ((g.n + 31) // 32) + 3 * 256 + 256
    sizes = pl.upload_streamed(walk + resident + 3 * 4 * 256, mode="ring")
    print(f"[case] streamed ring tiles={sizes['tiles']}", flush=True)
    assert sizes["tiles"] > 100
    psi = pl.state(psi0)
    pl.evolve(psi, 0)
    torch.cuda.synchronize()
    assert torch.equal(psi, pl.state(psi0))
    pl.evolve(psi, 4)
    ref = oracle.ctqw_evolve(g.row_ptr, g.col, psi0, 4, gamma=params["gamma"], dt=params["dt"], K=16,
                             marked=params["marked"])
    torch.cuda.synchronize()
    assert np.abs(psi.cpu().numpy() - ref).max() < 1e-12
    pl.upload()  # plain binding of the same plan
    x = pl.state(psi0)
    pl.evolve(x, 4)
    torch.cuda.synchronize()
    assert np.abs(x.cpu().numpy() - ref).max() < 1e-12
    pl.close()
    k1 = _plan(g, dict(params, taylor_order=1), "c128")
    k1.upload_streamed(walk + (1 << 20), mode="ring")
    y = k1.state(psi0)
    k1.evolve(y, 3)
    ref1 = oracle.ctqw_evolve(g.row_ptr, g.col, psi0, 3, gamma=params["gamma"], dt=params["dt"], K=1,
                              marked=params["marked"])
    torch.cuda.synchronize()
    assert np.abs(y.cpu().numpy() - ref1).max() < 1e-12
    k1.close()


def test_streamed_plan_cannot_join_a_batch():
    from paper_2406_08186_amd.walk import Batch
    g = I.erdos_renyi(400, 0.02, seed=1)
    pl = _plan(g, dict(gamma=0.2, dt=0.3, taylor_order=8, marked=[1]), "c64")
    pl.upload_streamed(pl.info.state_bytes + pl.info.work_bytes + (1 << 20))
    b = Batch(capacity=2, max_tiles=64, dtype="c64")
    with pytest.raises(L.QwError) as e:
        b.set_slot(0, pl, pl.state(I.uniform(g.n)), 3)
    assert e.value.code == L.QW_EUNSUPPORTED
    b.close()
    pl.close()


@pytest.mark.parametrize("K", [7, 8, 1])
def test_streamed_ring_reuse_across_stages_and_calls(K):
    """Rings that hold every tile (2-3 tiles: nothing is copied after the first stage
    of a call) or part of them (5-13 tiles, alternating tile order), odd and even K
    (the tile order alternates per stage, so across steps too) and K = 1, evolved in
    two calls: bitwise equal to one call on a one-tile ring, and to the oracle."""
    g = I.erdos_renyi(3000, 10 / 2999, seed=12)
    params = dict(gamma=0.1, dt=0.3, taylor_order=K, marked=[5, 2999])
    psi0 = I.random_state(g.n, 13)
    ref = oracle.ctqw_evolve(g.row_ptr, g.col, psi0, 5, gamma=params["gamma"], dt=params["dt"], K=K,
                             marked=params["marked"])
    one = _plan(g, params, "c128")
    assert one.upload_streamed(one.info.state_bytes + one.info.work_bytes + (1 << 30), mode="ring")["tiles"] == 1
    x = one.state(psi0)
    one.evolve(x, 5)
    torch.cuda.synchronize()
    assert np.abs(x.cpu().numpy() - ref).max() < 1e-12
    seen = set()
    for div in (0.6, 0.95, 1.9, 3.5, 8.5):
        pl = _plan(g, params, "c128")
        walk = pl.info.state_bytes + pl.info.work_bytes
        slot = int(4 * g.n_arcs / div / 3)
        sizes = pl.upload_streamed(walk + 8 * g.n + 4096 + 3 * slot, mode="ring")
        seen.add(sizes["tiles"])
        print(f"[case] streamed ring reuse K={K} tiles={sizes['tiles']}", flush=True)
        psi = pl.state(psi0)
        pl.evolve(psi, 3)
        pl.evolve(psi, 2)
        torch.cuda.synchronize()
        assert torch.equal(psi, x), f"{sizes['tiles']} tiles"
        pl.close()
    assert min(seen) <= 3 and max(seen) >= 6, seen
    one.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_direct_mode_long_rows_and_small_many_calls(dtype):
    """Direct mode on a graph with rows longer than a workgroup tile's LDS (a hub of
    degree 12000 and one of 8193: chunked staging, one thread's ordered fold) beside
    short rows whose arc runs start inside 16-byte groups, with the device prefix
    ending inside either hub's row; several calls and zero steps; ring mode: the same
    bits; K = 1 direct and rebound in core against the oracle."""
    n = 21000
    edges = [(0, v) for v in range(1, 12001)] + [(1, v) for v in range(12001, 12001 + 8193)]
    edges += [(v, v + 1) for v in range(2, n - 1)]
    g = I.from_edges(n, edges, name="two_hubs")
    assert int(np.diff(g.row_ptr).max()) > 8192
    params = dict(gamma=4e-5, dt=0.5, taylor_order=9, marked=[0, 7, n - 1])
    psi0 = I.random_state(g.n, 71)
    ref = oracle.ctqw_evolve(g.row_ptr, g.col, psi0, 4, gamma=params["gamma"], dt=params["dt"], K=9,
                             marked=params["marked"])
    out = None
    for mode, extra_arcs in (("direct", 0), ("direct", 5001), ("direct", 12003), ("direct", 1 << 28),
                             ("ring", 1 << 28)):
        pl = _plan(g, params, dtype)
        walk = pl.info.state_bytes + pl.info.work_bytes
        fixed = L.qw_plan_stream_sizes(pl._plan, 1 << 40, L.QW_STREAM_DIRECT)[1] - 16 * ((g.n_arcs + 3) // 4)
        budget = walk + (fixed + 255) // 256 * 256 + 256 + 4 * extra_arcs
        sizes = pl.upload_streamed(budget, mode=mode)
        print(f"[case] direct long rows {dtype} {mode} device_arcs={sizes['device_arcs']}", flush=True)
        if mode == "direct" and extra_arcs < 1 << 20:
            assert sizes["device_arcs"] < g.n_arcs
        psi = pl.state(psi0)
        pl.evolve(psi, 0)
        pl.evolve(psi, 3)
        pl.evolve(psi, 1)
        torch.cuda.synchronize()
        if out is None:
            out = psi.clone()
            got = psi.cpu().numpy().astype(np.complex128)
            if dtype == "c128":
                assert np.abs(got - ref).max() < 1e-12
            else:
                assert np.linalg.norm(got - ref) < 1e-5
        else:
            assert torch.equal(psi, out), (mode, extra_arcs)
        pl.close()
    k1 = _plan(g, dict(params, taylor_order=1), dtype)
    k1.upload_streamed(k1.info.state_bytes + k1.info.work_bytes + (1 << 22))
    y = k1.state(psi0)
    k1.evolve(y, 2)
    r1 = oracle.ctqw_evolve(g.row_ptr, g.col, psi0, 2, gamma=params["gamma"], dt=params["dt"], K=1,
                            marked=params["marked"])
    torch.cuda.synchronize()
    assert np.linalg.norm(y.cpu().numpy().astype(np.complex128) - r1) < (1e-12 if dtype == "c128" else 1e-5)
    k1.upload()
    z = k1.state(psi0)
    k1.evolve(z, 2)
    torch.cuda.synchronize()
    assert np.linalg.norm(z.cpu().numpy().astype(np.complex128) - r1) < (1e-12 if dtype == "c128" else 1e-5)
    k1.close()


def test_direct_mode_refuses_pageable_host_memory():
    g = I.erdos_renyi(500, 0.02, seed=3)
    pl = _plan(g, dict(gamma=0.2, dt=0.3, taylor_order=8, marked=[1]), "c64")
    budget = pl.info.state_bytes + pl.info.work_bytes + (1 << 20)
    host, dev, _, _ = L.qw_plan_stream_sizes(pl._plan, budget, L.QW_STREAM_DIRECT)
    pageable = torch.empty(host, dtype=torch.uint8)  # not pinned
    d = torch.empty(max(dev, 256), dtype=torch.uint8, device="cuda")
    with pytest.raises(L.QwError) as e:
        L.qw_plan_upload_streamed(pl._plan, budget, L.QW_STREAM_DIRECT, pageable.data_ptr(), host, d.data_ptr(),
                                  d.numel(), 0)
    assert e.value.code == L.QW_EINVAL
    pl.close()


@pytest.mark.parametrize("mode", ["direct", "ring"])
def test_streamed_edgeless_graph(mode):
    """No arcs at all (nothing to stage or copy): only the marked vertices' term acts."""
    g = I.Graph(n=300, row_ptr=np.zeros(301, np.int64), col=np.zeros(0, np.int32), name="edgeless")
    params = dict(gamma=0.3, dt=0.4, taylor_order=6, marked=[0, 299])
    psi0 = I.random_state(g.n, 5)
    pl = _plan(g, params, "c128")
    sizes = pl.upload_streamed(pl.info.state_bytes + pl.info.work_bytes + (1 << 20), mode=mode)
    assert sizes["device_arcs"] == 0
    psi = pl.state(psi0)
    pl.evolve(psi, 3)
    ref = oracle.ctqw_evolve(g.row_ptr, g.col, psi0, 3, gamma=params["gamma"], dt=params["dt"], K=6,
                             marked=params["marked"])
    torch.cuda.synchronize()
    assert np.abs(psi.cpu().numpy() - ref).max() < 1e-12
    pl.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_sliced_in_core_stage_and_streamed(dtype):
    """A regular graph whose vector exceeds 7.5 MiB takes the column-sliced ELL stage in
    core; an irregular one the CSR stages in core and out of core (direct mode): every
    walk equals the oracle."""
    from paper_2406_08186_amd.walk import Plan
    cases = [(I.erdos_renyi(300000, 7 / 299999, seed=17), "csr"), (I.random_regular(1000000, 5, seed=18), "structured")]
    for gi, (g, layout) in enumerate(cases):
        n = g.n
        dmax = int(np.diff(g.row_ptr).max())
        params = dict(gamma=0.15, dt=1.0 / (0.15 * dmax + 1.0), taylor_order=10, marked=[3, n - 2])
        psi0 = I.random_state(g.n, 90 + gi)
        ref = oracle.ctqw_evolve(g.row_ptr, g.col, psi0, 2, gamma=params["gamma"], dt=params["dt"], K=10,
                                 marked=params["marked"])

        def check(x):
            got = x.cpu().numpy().astype(np.complex128)
            if dtype == "c128":
                assert np.abs(got - ref).max() < 1e-12
            else:
                assert np.linalg.norm(got - ref) < 1e-5

        core = Plan(g, "ctqw", dtype=dtype, layout=layout, **params)
        assert core.structure == ("general" if layout == "csr" else "ell"), core.structure
        x = core.state(psi0)
        core.evolve(x, 2)
        torch.cuda.synchronize()
        print(f"[case] sliced in core {dtype} {core.structure}", flush=True)
        check(x)
        if layout == "csr":
            st = _plan(g, params, dtype)
            st.upload_streamed(st.info.state_bytes + st.info.work_bytes + 8 * g.n + (1 << 22))
            y = st.state(psi0)
            st.evolve(y, 2)
            torch.cuda.synchronize()
            check(y)
            st.close()
        core.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_sliced_csr_stage(dtype):
    """Irregular graphs whose vector exceeds 7.5 MiB take the column-sliced CSR stage
    (one lane per row for mean degree <= 6, two up to 12, four up to 24, eight up to
    48; rows longer than eight arcs per lane continue from memory).  One lane per row
    adds each row in arc order, as the direct out-of-core stage does: bitwise equal;
    every lane count equals the oracle."""
    from paper_2406_08186_amd.walk import Plan
    n = 1050000
    for gi, dbar in enumerate((5.0, 9.0, 16.0, 30.0)):
        g = I.erdos_renyi(n, dbar / (n - 1), seed=30 + gi)
        dmax = int(np.diff(g.row_ptr).max())
        lanes = 1 if dbar <= 6 else 2 if dbar <= 12 else 4 if dbar <= 24 else 8
        if lanes <= 2:
            assert dmax > 8 * lanes  # some rows take the cursor path
        params = dict(gamma=1.0 / dbar, dt=1.0 / (dmax / dbar + 1.0), taylor_order=9, marked=[11, n - 5])
        psi0 = I.random_state(g.n, 70 + gi)
        ref = oracle.ctqw_evolve(g.row_ptr, g.col, psi0, 2, gamma=params["gamma"], dt=params["dt"], K=9,
                                 marked=params["marked"])
        core = Plan(g, "ctqw", dtype=dtype, layout="csr", **params)
        x = core.state(psi0)
        core.evolve(x, 2)
        torch.cuda.synchronize()
        print(f"[case] sliced csr {dtype} mean degree {dbar}", flush=True)
        got = x.cpu().numpy().astype(np.complex128)
        if dtype == "c128":
            assert np.abs(got - ref).max() < 1e-12
        else:
            assert np.linalg.norm(got - ref) < 1e-5
        if dbar < 6:
            st = _plan(g, params, dtype)
            st.upload_streamed(st.info.state_bytes + st.info.work_bytes + 8 * g.n + (1 << 24))
            y = st.state(psi0)
            st.evolve(y, 2)
            torch.cuda.synchronize()
            assert torch.equal(x, y)
            st.close()
        core.close()
