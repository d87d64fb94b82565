"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: dense
operators built from the definitions, eigendecompositions, closed forms,
invariants and special cases.  ``test_oracle_mutations.py`` plants mistakes
in the oracle and shows these pins catch them.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import closed_forms as cf
from oracle import taylor as ot
from paper_2406_08186_amd import inputs as I
import pins

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def small_graphs():
    return [
        I.cycle(7), I.cycle_sorted(8), I.hypercube(3), I.torus(3, 4),
        I.random_mixed(12, seed=1), I.random_mixed(15, seed=2, p=0.3),
        I.complete(5), I.random_regular(10, 3, seed=3),
    ]


# ---------------------------------------------------------------- coined walk

@pytest.mark.parametrize("gi", range(8))
@pytest.mark.parametrize("steps", [1, 2, 13])
def test_coined_matches_dense_operators(gi, steps):
    """U = S C built densely from the definitions (Sec. 3.2), U^t psi0."""
    g = small_graphs()[gi]
    marked = [] if gi % 2 else [0, g.n - 1]
    psi0 = I.random_state(g.n_arcs, seed=gi)
    u = pins.dense_shift(g) @ pins.dense_coin(g, "grover", marked)
    ref = np.linalg.matrix_power(u, steps) @ psi0
    got = oracle.coined_evolve(g.row_ptr, g.col, psi0, steps, marked=marked)
    assert np.abs(got - ref).max() < 1e-13


@pytest.mark.parametrize("n", [5, 8, 64])
def test_coined_hadamard_matches_dense(n):
    g = I.cycle(n)
    psi0 = I.random_state(g.n_arcs, seed=n)
    u = pins.dense_shift(g) @ pins.dense_coin(g, "hadamard")
    ref = np.linalg.matrix_power(u, 9) @ psi0
    got = oracle.coined_evolve(g.row_ptr, g.col, psi0, 9, coin=oracle.HADAMARD)
    assert np.abs(got - ref).max() < 1e-13


@pytest.mark.parametrize("gi", range(8))
def test_coined_preserves_norm(gi):
    """U is unitary: the norm stays 1 to rounding after many steps."""
    g = small_graphs()[gi]
    psi0 = I.random_state(g.n_arcs, seed=10 + gi)
    psi = oracle.coined_evolve(g.row_ptr, g.col, psi0, 200, marked=[1])
    assert abs(np.linalg.norm(psi) - 1.0) < 1e-13


@pytest.mark.parametrize("gi", [0, 1, 2, 3, 6, 7])
def test_uniform_state_is_fixed_point(gi):
    """Without marks the uniform arc state is a +1 eigenvector of S*Grover."""
    g = small_graphs()[gi]
    u = I.uniform(g.n_arcs)
    psi = oracle.coined_evolve(g.row_ptr, g.col, u, 17)
    assert np.abs(psi - u).max() < 1e-15


def test_uniform_fixed_point_irregular():
    g = I.random_mixed(20, seed=5, n_isolated=0)
    assert len(set(np.diff(g.row_ptr).tolist())) > 2
    u = I.uniform(g.n_arcs)
    psi = oracle.coined_evolve(g.row_ptr, g.col, u, 9)
    assert np.abs(psi - u).max() < 1e-15


def test_grover_on_cycle_is_a_permutation():
    """d = 2 makes the Grover coin the swap, so each step permutes amplitudes."""
    g = I.cycle_sorted(11)
    psi0 = I.random_state(g.n_arcs, seed=4)
    prev = psi0
    for _ in range(5):
        nxt = oracle.coined_evolve(g.row_ptr, g.col, prev, 1)
        assert sorted(map(complex, nxt), key=lambda z: (z.real, z.imag)) == \
            sorted(map(complex, prev), key=lambda z: (z.real, z.imag))
        assert not np.array_equal(nxt, prev)
        prev = nxt


def test_cycle64_hadamard_symmetry_and_parity():
    """(|0,0> + i|0,1>)/sqrt2 on the 64-cycle: mirror-symmetric, even-site support."""
    g, psi0 = I.cycle_hadamard_state(64)
    psi = oracle.coined_evolve(g.row_ptr, g.col, psi0, 100, coin=oracle.HADAMARD)
    p = oracle.coined_prob(g.row_ptr, g.col, psi)
    assert np.abs(p - p[(-np.arange(64)) % 64]).max() < 1e-15
    assert p[1::2].max() == 0.0
    assert abs(p.sum() - 1.0) < 1e-13


def test_cycle64_hadamard_golden():
    """Stored distribution (tests/golden) written by make_golden.py from the oracle."""
    ref = np.loadtxt(_golden("cycle64_hadamard_100.txt"))
    g, psi0 = I.cycle_hadamard_state(64)
    psi = oracle.coined_evolve(g.row_ptr, g.col, psi0, 100, coin=oracle.HADAMARD)
    p = oracle.coined_prob(g.row_ptr, g.col, psi)
    assert np.abs(p - ref).max() < 1e-15
    # and the same numbers from the dense 128x128 operator
    u = pins.dense_shift(g) @ pins.dense_coin(g, "hadamard")
    full = np.linalg.matrix_power(u, 100) @ psi0
    pd = np.add.reduceat(np.abs(full) ** 2, g.row_ptr[:-1])
    assert np.abs(pd - ref).max() < 1e-13


@pytest.mark.parametrize("dim", [4, 6, 9])
def test_hypercube_search_matches_reduced_model(dim):
    """Full coined search on Q_dim equals the 2*dim reduced walk, state by state."""
    g = I.hypercube(dim)
    steps = 3 * dim + 1
    psi = oracle.coined_evolve(g.row_ptr, g.col, I.uniform(g.n_arcs), steps, marked=[0])
    red = cf.hypercube_search_state(dim, steps, g.row_ptr, g.col)
    assert np.abs(psi - red).max() < 1e-14


def test_hypercube_reduced_model_is_unitary_and_peaks():
    """Reduced model: norm 1, and search amplifies p_marked well above 1/N."""
    o, i, hist = cf.hypercube_search_reduced(12, 200, record_marked=True)
    assert abs(np.sum(np.abs(o) ** 2) + np.sum(np.abs(i) ** 2) - 1) < 1e-13
    assert max(hist) > 0.3 and hist[0] == pytest.approx(1 / 4096)


def test_coined_probability_sums_tails():
    """p_v sums arcs whose tail is v (Sec. 3.2): one arc (v,w) puts all mass on v."""
    g = I.random_mixed(12, seed=1)
    v = 3
    w = int(g.row(v)[0])
    psi = I.ket_arc(g, v, w)
    p = oracle.coined_prob(g.row_ptr, g.col, psi)
    assert p[v] == 1.0 and p[w] == 0.0 and p.sum() == 1.0
    x = I.random_state(g.n_arcs, 7)
    p = oracle.coined_prob(g.row_ptr, g.col, x)
    assert abs(p.sum() - 1.0) < 1e-14
    assert p[g.n - 3] >= 0  # isolated vertex index exists
    assert np.all(p[np.diff(g.row_ptr) == 0] == 0.0)


def test_reverse_arcs_and_validation():
    g = I.random_mixed(14, seed=3)
    rev = oracle.reverse_arcs(g.row_ptr, g.col)
    assert np.array_equal(rev[rev], np.arange(g.n_arcs))
    tails = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    assert np.array_equal(g.col[rev], tails)
    with pytest.raises(ValueError):
        oracle.reverse_arcs(np.array([0, 1, 1]), np.array([1], np.int32))
    with pytest.raises(ValueError):
        oracle.reverse_arcs(np.array([0, 1]), np.array([0], np.int32))


def test_hadamard_rejects_wrong_degree():
    g = I.hypercube(3)
    with pytest.raises(ValueError):
        oracle.coined_evolve(g.row_ptr, g.col, I.uniform(g.n_arcs), 1, coin=oracle.HADAMARD)


# ------------------------------------------------------------------------ CTQW

@pytest.mark.parametrize("gi", range(8))
def test_ctqw_matches_eigh(gi):
    """T_20(-iH dt)^n at dt = 0.1 equals exp(-iHt) (dense eigh) to rounding."""
    g = small_graphs()[gi]
    marked = [0] if gi % 2 == 0 else [1, g.n - 1]
    gamma = 0.3 + 0.05 * gi
    psi0 = I.random_state(g.n, seed=20 + gi)
    got = oracle.ctqw_evolve(g.row_ptr, g.col, psi0, 40, gamma=gamma, dt=0.1, K=20, marked=marked)
    ref = pins.expm_eigh(pins.dense_hamiltonian(g, gamma, marked), 4.0, psi0)
    assert np.abs(got - ref).max() < 1e-13


@pytest.mark.parametrize("K", [1, 2, 4, 7])
def test_ctqw_low_order_matches_polynomial(K):
    """At low order the result is exactly the degree-K Taylor polynomial."""
    g = I.random_mixed(13, seed=8)
    h = pins.dense_hamiltonian(g, 0.4, [2])
    psi0 = I.random_state(g.n, seed=K)
    got = oracle.ctqw_evolve(g.row_ptr, g.col, psi0, 6, gamma=0.4, dt=0.35, K=K, marked=[2])
    ref = pins.taylor_eigh(h, 0.35, K, 6, psi0)
    assert np.abs(got - ref).max() < 1e-13
    # and it is NOT the order K-1 or K+1 polynomial
    for kk in (K - 1, K + 1):
        if kk >= 0:
            other = pins.taylor_eigh(h, 0.35, kk, 6, psi0)
            assert np.abs(got - other).max() > 1e-8


def test_ctqw_cycle_bessel_images():
    """Cycle, gamma = 0.25, t = 30: amplitude sum_m i^(x+mN) J_(x+mN)(2 gamma t)."""
    n = 64
    g = I.cycle_sorted(n)
    got = oracle.ctqw_evolve(g.row_ptr, g.col, I.ket_vertex(n, 5), 300, gamma=0.25, dt=0.1, K=20)
    ref = cf.cycle_ctqw(n, 0.25, 30.0, 5)
    assert np.abs(got - ref).max() < 1e-13
    # before wrap-around a single Bessel term suffices
    x = (np.arange(n) - 5) % n
    x = np.where(x > n // 2, x - n, x)
    single = (1j ** np.abs(x)) * __import__("scipy.special", fromlist=["jv"]).jv(np.abs(x), 15.0)
    assert np.abs(got - single).max() < 1e-7


def test_closed_forms_against_eigh():
    """The Bessel-image and torus-product closed forms equal dense eigh."""
    g = I.cycle_sorted(40)
    ref = pins.expm_eigh(pins.dense_hamiltonian(g, 0.25, []), 23.0, I.ket_vertex(40, 7))
    assert np.abs(cf.cycle_ctqw(40, 0.25, 23.0, 7) - ref).max() < 1e-13
    t = I.torus(6, 5)
    ref = pins.expm_eigh(pins.dense_hamiltonian(t, 0.25, []), 7.3, I.ket_vertex(30, 13))
    assert np.abs(cf.torus_ctqw(6, 5, 0.25, 7.3, 13) - ref).max() < 1e-13


def test_ctqw_torus_product_form():
    l1, l2 = 12, 10
    g = I.torus(l1, l2)
    v0 = 5 * l2 + 4
    got = oracle.ctqw_evolve(g.row_ptr, g.col, I.ket_vertex(l1 * l2, v0), 100, gamma=0.25,
                             dt=0.1, K=20)
    ref = cf.torus_ctqw(l1, l2, 0.25, 10.0, v0)
    assert np.abs(got - ref).max() < 1e-13


@pytest.mark.parametrize("n", [16, 64])
def test_ctqw_complete_graph_search(n):
    """K_N, gamma = 1/N, one mark: p_w(t) = sin^2(t/sqrtN) + cos^2(t/sqrtN)/N; 1 at (pi/2)sqrtN."""
    g = I.complete(n)
    t_opt = math.pi / 2 * math.sqrt(n)
    steps = 100
    psi = I.uniform(n)
    for s in range(1, 4):
        psi = oracle.ctqw_evolve(g.row_ptr, g.col, psi, steps, gamma=1.0 / n,
                                 dt=t_opt / (3 * steps), K=24, marked=[3])
        p = abs(psi[3]) ** 2
        assert abs(p - cf.complete_search_prob(n, s * t_opt / 3)) < 1e-12
    assert abs(abs(psi[3]) ** 2 - 1.0) < 1e-12


def test_complete_search_formula_against_eigh():
    n = 16
    g = I.complete(n)
    h = pins.dense_hamiltonian(g, 1.0 / n, [3])
    for t in (0.7, 3.1, 6.2):
        psi = pins.expm_eigh(h, t, I.uniform(n))
        assert abs(abs(psi[3]) ** 2 - cf.complete_search_prob(n, t)) < 1e-13


def test_ctqw_norm_and_vertex_prob():
    g = I.random_regular(30, 4, seed=9)
    psi = oracle.ctqw_evolve(g.row_ptr, g.col, I.random_state(30, 1), 500, gamma=0.25, dt=0.1,
                             K=20, marked=[4])
    p = oracle.vertex_prob(psi)
    assert abs(p.sum() - 1.0) < 1e-13
    assert np.abs(p - np.abs(psi) ** 2).max() < 1e-16


def test_ctqw_isolated_and_empty():
    g = I.from_edges(5, [(0, 1)])
    psi0 = I.random_state(5, 3)
    got = oracle.ctqw_evolve(g.row_ptr, g.col, psi0, 10, gamma=0.5, dt=0.1, K=20, marked=[4])
    ref = pins.expm_eigh(pins.dense_hamiltonian(g, 0.5, [4]), 1.0, psi0)
    assert np.abs(got - ref).max() < 1e-13
    # isolated unmarked vertices keep their amplitude exactly
    assert got[2] == psi0[2] and got[3] == psi0[3]


# ---------------------------------------------------------- Taylor order rule

@pytest.mark.parametrize("rho,steps,tol", [(0.1, 1000, 1e-12), (1.0, 200, 1e-8),
                                           (2.0, 50, 1e-10), (0.5, 10**4, 1e-6)])
def test_taylor_order_is_minimal_and_safe(rho, steps, tol):
    K = ot.taylor_order(rho, steps, tol)
    assert K >= 1
    assert steps * ot.tail_bound(rho, K) <= tol
    if K > 1:
        assert steps * ot.tail_bound(rho, K - 1) > tol
    # the tail bound really bounds the series tail
    exact_tail = sum(rho ** k / math.factorial(k) for k in range(K + 1, K + 60))
    assert exact_tail <= ot.tail_bound(rho, K) * (1 + 1e-12)


def test_taylor_rule_error_within_tolerance():
    """The chosen K keeps the final-state error below tol (against eigh)."""
    g = I.random_regular(40, 5, seed=11)
    gamma, marked = 0.2, [7]
    hb = ot.h_norm_bound(np.diff(g.row_ptr), gamma, marked)
    assert hb == pytest.approx(0.2 * 5 + 1)
    for rho_max, tol in ((1.0, 1e-6), (2.0, 1e-9), (0.5, 1e-12)):
        K, dt, steps = ot.taylor_plan(hb, 15.0, rho_max, tol)
        assert dt * hb <= rho_max + 1e-12
        psi0 = I.random_state(40, 2)
        got = oracle.ctqw_evolve(g.row_ptr, g.col, psi0, steps, gamma=gamma, dt=dt, K=K,
                                 marked=marked)
        ref = pins.expm_eigh(pins.dense_hamiltonian(g, gamma, marked), 15.0, psi0)
        assert np.linalg.norm(got - ref) <= tol + 1e-13


def test_config_grid_taylor_bound():
    """Torus 1024^2 at gamma = 0.25, K = 20, dt = 0.1: per-step tail ~1e-41."""
    hb = ot.h_norm_bound(np.full(4, 4), 0.25, [])
    assert hb == 1.0
    assert ot.tail_bound(0.1, 20) < 1e-40


# ------------------------------------------------------------ helpers/golden

def _golden(name):
    import os
    return os.path.join(os.path.dirname(__file__), "golden", name)


def test_paper_ket_examples():
    """The worked initial states of Sec. 3.1 and Sec. 3.2 are normalised."""
    a = 1 / 2 ** 0.5
    psi = a * (I.ket_vertex(5, 2) + 1j * I.ket_vertex(5, 4))
    assert abs(np.linalg.norm(psi) - 1) < 1e-15
    g = I.complete(4)
    psi = a * I.ket_arc(g, 0, 1) + a * I.ket_arc(g, 0, 2)
    assert abs(np.linalg.norm(psi) - 1) < 1e-15
    with pytest.raises(KeyError):
        I.ket_arc(I.cycle(5), 0, 2)


def test_paper_ctqw_example_golden():
    """Sec. 3.1 example: gamma = 0.35, dt = 0.03, marks {1, 4}, psi0 = (|2> + i|4>)/sqrt2,
    21 states k = 0..20, here on the 101-cycle of Fig. 1.  Stored distributions
    (written from the oracle) checked against dense eigh and the oracle."""
    ref = np.loadtxt(_golden("ctqw_sec31_cycle101.txt"))
    g = I.cycle_sorted(101)
    a = 1 / 2 ** 0.5
    psi = a * (I.ket_vertex(101, 2) + 1j * I.ket_vertex(101, 4))
    h = pins.dense_hamiltonian(g, 0.35, [1, 4])
    for k in range(21):
        pk = np.abs(pins.expm_eigh(h, 0.03 * k, psi)) ** 2
        assert np.abs(pk - ref[k]).max() < 1e-14
    got = psi
    for k in range(1, 21):
        got = oracle.ctqw_evolve(g.row_ptr, g.col, got, 1, gamma=0.35, dt=0.03, K=20,
                                 marked=[1, 4])
        assert np.abs(oracle.vertex_prob(got) - ref[k]).max() < 1e-14
