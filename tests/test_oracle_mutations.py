"""Plant plausible mistakes in the oracle (CPU only) and show the pins catch them.

Each fault is switched on inside the C oracle; the same checks the pin tests
make must then fail.  With no fault, every check passes.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import closed_forms as cf
from paper_2406_08186_amd import inputs as I
import pins


def _coined_dense_ok():
    g = I.random_mixed(12, seed=1)
    psi0 = I.random_state(g.n_arcs, seed=0)
    u = pins.dense_shift(g) @ pins.dense_coin(g, "grover", [0])
    ref = np.linalg.matrix_power(u, 3) @ psi0
    got = oracle.coined_evolve(g.row_ptr, g.col, psi0, 3, marked=[0])
    return np.abs(got - ref).max() < 1e-13


def _coined_norm_ok():
    g = I.random_mixed(12, seed=1)
    psi = oracle.coined_evolve(g.row_ptr, g.col, I.random_state(g.n_arcs, 1), 50, marked=[1])
    return abs(np.linalg.norm(psi) - 1) < 1e-13


def _hadamard_ok():
    g, psi0 = I.cycle_hadamard_state(64)
    psi = oracle.coined_evolve(g.row_ptr, g.col, psi0, 100, coin=oracle.HADAMARD)
    p = oracle.coined_prob(g.row_ptr, g.col, psi)
    import os
    ref = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "cycle64_hadamard_100.txt"))
    return np.abs(p - ref).max() < 1e-15


def _hadamard_dense_ok():
    g = I.cycle(8)
    psi0 = I.random_state(g.n_arcs, seed=8)
    u = pins.dense_shift(g) @ pins.dense_coin(g, "hadamard")
    ref = np.linalg.matrix_power(u, 5) @ psi0
    got = oracle.coined_evolve(g.row_ptr, g.col, psi0, 5, coin=oracle.HADAMARD)
    return np.abs(got - ref).max() < 1e-13


def _hypercube_ok():
    g = I.hypercube(6)
    psi = oracle.coined_evolve(g.row_ptr, g.col, I.uniform(g.n_arcs), 19, marked=[0])
    return np.abs(psi - cf.hypercube_search_state(6, 19, g.row_ptr, g.col)).max() < 1e-14


def _prob_tail_ok():
    g = I.random_mixed(12, seed=1)
    v = 3
    w = int(g.row(v)[0])
    p = oracle.coined_prob(g.row_ptr, g.col, I.ket_arc(g, v, w))
    return p[v] == 1.0 and p[w] == 0.0


def _ctqw_eigh_ok():
    g = I.random_mixed(13, seed=8)
    psi0 = I.random_state(g.n, seed=2)
    got = oracle.ctqw_evolve(g.row_ptr, g.col, psi0, 30, gamma=0.4, dt=0.1, K=20, marked=[2, 5])
    ref = pins.expm_eigh(pins.dense_hamiltonian(g, 0.4, [2, 5]), 3.0, psi0)
    return np.abs(got - ref).max() < 1e-13


def _ctqw_poly_ok():
    g = I.random_mixed(13, seed=8)
    h = pins.dense_hamiltonian(g, 0.4, [2])
    psi0 = I.random_state(g.n, seed=4)
    got = oracle.ctqw_evolve(g.row_ptr, g.col, psi0, 6, gamma=0.4, dt=0.35, K=4, marked=[2])
    return np.abs(got - pins.taylor_eigh(h, 0.35, 4, 6, psi0)).max() < 1e-13


def _complete_search_ok():
    n = 16
    g = I.complete(n)
    t = math.pi / 2 * math.sqrt(n)
    psi = oracle.ctqw_evolve(g.row_ptr, g.col, I.uniform(n), 200, gamma=1 / n, dt=t / 200, K=24,
                             marked=[3])
    return abs(abs(psi[3]) ** 2 - 1) < 1e-12


def _stag_arcs_ok():
    g = I.random_mixed(12, seed=3)
    sg, tess = I.stag_arcs(g)
    psi0 = I.random_state(g.n_arcs, 9)
    a = oracle.staggered_evolve(sg.n, tess, psi0, 5)
    return np.abs(a - oracle.coined_evolve(g.row_ptr, g.col, psi0, 5)).max() < 1e-13


def _stag_mark_order_ok():
    _, tess = I.stag_cycle(12)
    got = oracle.staggered_evolve(12, tess, I.ket_vertex(12, 4), 1, marked=[4])
    return np.abs(got + I.ket_vertex(12, 6)).max() < 1e-15


def _stag_theta_ok():
    edge = I.tessellation([[0, 1]], theta=0.3)
    got = oracle.staggered_evolve(2, [edge], I.ket_vertex(2, 0), 3)
    return np.abs(got - np.array([math.cos(0.9), 1j * math.sin(0.9)])).max() < 1e-14


CHECKS = [_stag_arcs_ok, _stag_mark_order_ok, _stag_theta_ok, _coined_dense_ok, _coined_norm_ok, _hadamard_ok, _hadamard_dense_ok, _hypercube_ok, _prob_tail_ok,
          _ctqw_eigh_ok, _ctqw_poly_ok, _complete_search_ok]


def test_all_checks_pass_without_fault():
    assert all(c() for c in CHECKS)


@pytest.mark.parametrize("name", sorted(oracle.FAULTS))
def test_planted_fault_is_caught(name):
    with oracle.fault(name):
        results = {c.__name__: bool(c()) for c in CHECKS}
    assert not all(results.values()), f"fault {name} slipped through: {results}"
