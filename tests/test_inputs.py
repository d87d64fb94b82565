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
