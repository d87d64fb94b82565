"""Seeded generators: valid simple symmetric graphs with the stated shapes."""
import numpy as np
import pytest

from paper_2406_08186_amd import inputs as I


def _check_simple_symmetric(g):
    rp, col = g.row_ptr, g.col.astype(np.int64)
    tails = np.repeat(np.arange(g.n), np.diff(rp))
    assert np.all(col != tails), "self-loop"
    fwd = set(zip(tails.tolist(), col.tolist()))
    assert len(fwd) == col.size, "repeated arc"
    assert all((w, v) in fwd for v, w in fwd), "not symmetric"


@pytest.mark.parametrize("g", [I.cycle(9), I.cycle_sorted(9), I.torus(4, 5), I.hypercube(5),
                               I.complete(6), I.random_regular(50, 3, 1),
                               I.random_regular(64, 8, 2), I.erdos_renyi(200, 0.03, 3),
                               I.random_mixed(20, 4)])
def test_generated_graphs_are_simple(g):
    _check_simple_symmetric(g)


def test_degrees_and_sizes():
    assert I.hypercube(6).n_arcs == 6 * 64
    assert np.all(I.torus(5, 7).degrees() == 4)
    rr = I.random_regular(101 + 1, 5, seed=3)
    assert np.all(rr.degrees() == 5)
    c = I.cycle(10)
    assert c.row(0).tolist() == [1, 9] and c.row(9).tolist() == [0, 8]


def test_seeded_reproducible():
    a = I.random_regular(300, 6, seed=7)
    b = I.random_regular(300, 6, seed=7)
    assert np.array_equal(a.col, b.col)
    e1 = I.erdos_renyi(500, 0.01, 5)
    e2 = I.erdos_renyi(500, 0.01, 5)
    assert np.array_equal(e1.col, e2.col)


def test_batch_specs():
    specs = I.batch_regular_specs(64, seed=1)
    for s in specs:
        assert 3 <= s["d"] <= 8 and (s["n"] * s["d"]) % 2 == 0
        assert 1000 <= s["n"] <= 200001
        assert 0 <= s["marked"] < s["n"]


# ---- staggered-walk tessellations ------------------------------------------------

def _is_partition(t, n):
    return (t.poly_ptr[0] == 0 and t.poly_ptr[-1] == n and np.all(np.diff(t.poly_ptr) > 0)
            and np.array_equal(np.sort(t.poly_vert), np.arange(n)))


def _polygons_are_cliques(g, t):
    adj = {v: set(int(u) for u in g.row(v)) for v in range(g.n)}
    for p in range(t.n_polygons):
        vs = [int(v) for v in t.poly_vert[t.poly_ptr[p]:t.poly_ptr[p + 1]]]
        if any(b not in adj[a] for a in vs for b in vs if a != b):
            return False
    return True


@pytest.mark.parametrize("l1,l2", [(4, 4), (6, 8), (10, 4), (16, 12)])
def test_stag_lattice_partitions_and_graph(l1, l2):
    g, tess = I.stag_lattice(l1, l2)
    assert g.n == l1 * l2 and set(np.diff(g.row_ptr)) == {6}
    u = I.union_graph(g.n, tess)
    assert np.array_equal(u.row_ptr, g.row_ptr) and np.array_equal(u.col, g.col)
    for k, t in enumerate(tess):
        assert _is_partition(t, g.n) and set(t.sizes()) == {4}
        assert _polygons_are_cliques(g, t)
        first = t.poly_vert[:4]  # corners (r, c), (r, c+1), (r+1, c), (r+1, c+1) of the first square
        assert first[0] // l2 % 2 == k and first[0] % l2 % 2 == k


def test_stag_cycle_and_arcs():
    g, tess = I.stag_cycle(10)
    assert all(_is_partition(t, 10) and set(t.sizes()) == {2} for t in tess)
    assert all(_polygons_are_cliques(g, t) for t in tess)
    h = I.random_mixed(15, seed=4)
    sg, (stars, pairs) = I.stag_arcs(h)
    assert sg.n == h.n_arcs and _is_partition(stars, sg.n) and _is_partition(pairs, sg.n)
    # each pair is an arc and its reverse; each star is one tail's row, in row order
    tails = np.repeat(np.arange(h.n), np.diff(h.row_ptr))
    for a, b in pairs.poly_vert.reshape(-1, 2):
        assert tails[a] == h.col[b] and tails[b] == h.col[a]
    assert np.array_equal(stars.poly_vert, np.arange(h.n_arcs))


def test_stag_random_weighted_is_normalised():
    g, tess = I.stag_random(200, 3, 7, seed=2, weighted=True)
    for t in tess:
        assert _is_partition(t, 200) and t.sizes().max() <= 7
        sq = np.add.reduceat(t.amp ** 2, t.poly_ptr[:-1])
        assert np.abs(sq - 1).max() < 1e-12
        assert _polygons_are_cliques(g, t)
