"""Pins for the oracle's staggered walk, one step psi <- U_T ... U_1 R_M psi
with U_k = 2 P_k - I (reflection form) or exp(i theta_k (2 P_k - I))
(Hamiltonian form), P_k the projector onto tessellation k's polygon vectors
and R_M the phase flip of the marked vertices:

* on the arcs of a graph, the star tessellation (arcs of one tail, uniform)
  followed by the pair tessellation (an arc and its reverse) is the Grover
  coined walk with the flip-flop shift, and with star amplitudes sqrt(P_xy)
  it is Szegedy's walk -- both oracle paths pinned elsewhere;
* on an even cycle tessellated by its two perfect matchings every reflection
  is a swap, so the walk is a permutation: even vertices move +2, odd -2;
* a tessellation of singletons is the identity, a single polygon over all
  vertices fixes the uniform state and negates its orthogonal complement;
* the Hamiltonian form: on one edge, exp(i theta X)|0> = cos(theta)|0> +
  i sin(theta)|1>; theta = pi/2 is i times the reflection; theta and -theta
  cancel and angles of one tessellation add;
* the marked phase flip comes before the tessellations, every marked vertex
  flipped is a global sign, and the walk preserves the norm.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2406_08186_amd import inputs as I


def _evolve(n, tess, psi0, steps, marked=None):
    return oracle.staggered_evolve(n, tess, psi0, steps, marked=marked)


def _graphs():
    return [I.random_mixed(12, seed=3), I.cycle(9), I.complete(5), I.hypercube(4),
            I.erdos_renyi(14, 0.4, seed=2)]


@pytest.mark.parametrize("gi", range(5))
def test_arc_tessellations_are_the_grover_coined_walk(gi):
    g = _graphs()[gi]
    sg, tess = I.stag_arcs(g)
    assert sg.n == g.n_arcs
    psi0 = I.random_state(g.n_arcs, 40 + gi)
    a = _evolve(sg.n, tess, psi0, 13)
    b = oracle.coined_evolve(g.row_ptr, g.col, psi0, 13)
    assert np.abs(a - b).max() < 1e-13


@pytest.mark.parametrize("gi", [0, 2, 4])
def test_weighted_stars_are_szegedy(gi):
    g = _graphs()[gi]
    rng = np.random.default_rng(gi)
    w = {}
    for v in range(g.n):
        for u in g.row(v):
            w.setdefault((min(v, int(u)), max(v, int(u))), rng.uniform(0.2, 2.0))
    p = np.empty(g.n_arcs)
    for v in range(g.n):
        lo, hi = g.row_ptr[v], g.row_ptr[v + 1]
        ww = np.array([w[(min(v, int(u)), max(v, int(u)))] for u in g.col[lo:hi]])
        p[lo:hi] = ww / ww.sum() if ww.size else ww
    sg, tess = I.stag_arcs(g)
    # the star polygons list each tail's arcs in row order, so the amplitude
    # of position i of the star tessellation is sqrt(P) of arc poly_vert[i]
    tess[0].amp = np.sqrt(p[tess[0].poly_vert])
    psi0 = I.random_state(g.n_arcs, 70 + gi)
    a = _evolve(sg.n, tess, psi0, 9)
    b = oracle.szegedy_evolve(g.row_ptr, g.col, psi0, 9, p)
    assert np.abs(a - b).max() < 1e-13


@pytest.mark.parametrize("n,steps", [(4, 3), (10, 7), (64, 41)])
def test_even_cycle_matchings_are_a_permutation(n, steps):
    _, tess = I.stag_cycle(n)
    psi0 = I.random_state(n, n)
    got = _evolve(n, tess, psi0, steps)
    v = np.arange(n)
    want = np.where(v % 2 == 0, psi0[(v - 2 * steps) % n], psi0[(v + 2 * steps) % n])
    assert np.abs(got - want).max() < 1e-14


def test_marked_flip_comes_first():
    n = 12
    _, tess = I.stag_cycle(n)
    # |4> is marked: R_M gives -|4>, the matchings carry it to -|6>
    got = _evolve(n, tess, I.ket_vertex(n, 4), 1, marked=[4])
    assert np.abs(got - (-I.ket_vertex(n, 6))).max() < 1e-15
    # an unmarked start that lands on the marked vertex keeps its sign
    got = _evolve(n, tess, I.ket_vertex(n, 2), 1, marked=[4])
    assert np.abs(got - I.ket_vertex(n, 4)).max() < 1e-15
    # over many steps the walk visits 4 every n/2 steps from 4 on the even ring
    got = _evolve(n, tess, I.ket_vertex(n, 4), n, marked=[4])
    assert np.abs(got - I.ket_vertex(n, 4)).max() < 1e-14  # two visits, two flips


def test_all_marked_is_a_global_sign():
    g, tess = I.stag_random(30, 3, 5, seed=5, weighted=True)
    psi0 = I.random_state(30, 1)
    for steps in (1, 4, 7):
        a = _evolve(30, tess, psi0, steps, marked=list(range(30)))
        b = _evolve(30, tess, psi0, steps)
        assert np.abs(a - (-1) ** steps * b).max() < 1e-14


def test_singletons_are_the_identity_and_marks_flip():
    n = 9
    single = I.tessellation([[v] for v in range(n)])
    psi0 = I.random_state(n, 2)
    assert np.abs(_evolve(n, [single, single], psi0, 5) - psi0).max() < 1e-15
    got = _evolve(n, [single], psi0, 3, marked=[2, 7])
    want = psi0.copy()
    want[[2, 7]] *= -1
    assert np.abs(got - want).max() < 1e-15


def test_one_polygon_reflects_about_the_uniform_state():
    n = 16
    whole = I.tessellation([list(range(n))])
    u = I.uniform(n)
    w = I.random_state(n, 3)
    w -= np.vdot(u, w) * u  # orthogonal to u
    psi0 = 0.6 * u + w
    for s in (1, 2, 5):
        got = _evolve(n, [whole], psi0, s)
        assert np.abs(got - (0.6 * u + (-1) ** s * w)).max() < 1e-14


@pytest.mark.parametrize("theta", [0.3, -1.1, 2.5])
def test_hamiltonian_form_on_one_edge(theta):
    edge = I.tessellation([[0, 1]], theta=theta)
    for s in (1, 3, 8):
        got = _evolve(2, [edge], I.ket_vertex(2, 0), s)
        want = np.array([math.cos(s * theta), 1j * math.sin(s * theta)])
        assert np.abs(got - want).max() < 1e-14


def test_hamiltonian_quarter_turn_is_i_times_the_reflection():
    g, tess = I.stag_random(40, 3, 6, seed=8, weighted=True)
    ham = [I.Tessellation(t.poly_ptr, t.poly_vert, t.amp, math.pi / 2) for t in tess]
    psi0 = I.random_state(40, 4)
    a = _evolve(40, ham, psi0, 5, marked=[3])
    b = _evolve(40, tess, psi0, 5, marked=[3])
    assert np.abs(a - (1j) ** 15 * b).max() < 1e-13


def test_hamiltonian_angles_add_and_cancel():
    g, tess = I.stag_random(35, 2, 4, seed=9, weighted=True)
    t = tess[0]
    psi0 = I.random_state(35, 6)

    def at(theta):
        return I.Tessellation(t.poly_ptr, t.poly_vert, t.amp, theta)

    assert np.abs(_evolve(35, [at(0.7), at(-0.7)], psi0, 3) - psi0).max() < 1e-14
    a = _evolve(35, [at(0.4), at(0.9)], psi0, 4)
    b = _evolve(35, [at(1.3)], psi0, 4)
    assert np.abs(a - b).max() < 1e-13


@pytest.mark.parametrize("seed", [1, 2])
def test_norm_is_preserved(seed):
    g, tess = I.stag_random(200, 4, 9, seed=seed, weighted=True)
    tess[1].theta = 0.37
    psi = _evolve(200, tess, I.random_state(200, seed), 300, marked=[5, 17])
    assert abs(np.linalg.norm(psi) - 1.0) < 1e-12


def test_rejects_a_non_partition():
    t = I.tessellation([[0, 1], [1, 2]])
    with pytest.raises(ValueError):
        _evolve(3, [t], I.uniform(3), 1)
