"""Pins for the oracle's general coins and the persistent shift (Sec. 3.2),
checked against what the definitions and the physics fix, never against the
oracle's own formulas.

* Persistent shift with the identity coin: every walker moves straight on,
  so after t steps the amplitude of arc v -> v+e sits on v+te -> v+(t+1)e
  (a closed-form translation, computed here from coordinates).
* The 2 x 2 Fourier coin is the Hadamard coin, whose path is pinned elsewhere.
* Fourier coins are unitary; with any unitary coin and either shift the norm
  is preserved.
* The uniform arc state is a fixed point of Grover with the persistent shift
  (a permutation of arcs that keeps the uniform state).
* A random unitary coin with the flip-flop shift equals the dense product of
  the shift permutation (built here from arc positions) and the block-diagonal
  coin.
* The 1-D Hadamard walk with the moving shift from (|0,R> + i|0,L>)/sqrt 2 is
  mirror symmetric, lives on even sites after even steps and peaks just
  inside |x| = t / sqrt 2.
"""
import numpy as np
import pytest

import oracle
from paper_2406_08186_amd import inputs as I


def _cycle_coords(n):
    return {v: (v,) for v in range(n)}


@pytest.mark.parametrize("t", [1, 5, 13])
def test_persistent_identity_coin_translates_on_cycle(t):
    n = 11
    g = I.cycle(n)                        # rows v+1, v-1: direction order
    rng = np.random.default_rng(t)
    psi0 = rng.normal(size=g.n_arcs) + 1j * rng.normal(size=g.n_arcs)
    got = oracle.coined_evolve_general(g.row_ptr, g.col, psi0, t, coin=np.eye(2), shift="persistent",
                                       dims=(n,))
    want = np.zeros_like(psi0)
    for v in range(n):
        for e in (+1, -1):
            a0 = I.arc_index(g, v, (v + e) % n)
            a1 = I.arc_index(g, (v + t * e) % n, (v + (t + 1) * e) % n)
            want[a1] = psi0[a0]
    assert np.array_equal(got, want)


def test_persistent_identity_coin_translates_on_grid():
    l1, l2, t = 4, 5, 7
    g = I.torus_directed(l1, l2)
    rng = np.random.default_rng(3)
    psi0 = rng.normal(size=g.n_arcs) + 1j * rng.normal(size=g.n_arcs)
    got = oracle.coined_evolve_general(g.row_ptr, g.col, psi0, t, coin=np.eye(4), shift="persistent",
                                       dims=(l1, l2))
    want = np.zeros_like(psi0)
    for r in range(l1):
        for c in range(l2):
            for dr, dc in ((0, 1), (0, -1), (1, 0), (-1, 0)):
                v = r * l2 + c
                w = ((r + dr) % l1) * l2 + (c + dc) % l2
                x = ((r + t * dr) % l1) * l2 + (c + t * dc) % l2
                y = ((r + (t + 1) * dr) % l1) * l2 + (c + (t + 1) * dc) % l2
                want[I.arc_index(g, x, y)] = psi0[I.arc_index(g, v, w)]
    assert np.array_equal(got, want)
    # back where it started after a full period along each axis
    full = oracle.coined_evolve_general(g.row_ptr, g.col, psi0, l1 * l2, coin=np.eye(4), shift="persistent",
                                        dims=(l1, l2))
    assert np.array_equal(full, psi0)


def test_fourier2_is_hadamard():
    g, psi0 = I.cycle_hadamard_state(64)
    a = oracle.coined_evolve_general(g.row_ptr, g.col, psi0, 100, coin="fourier")
    b = oracle.coined_evolve(g.row_ptr, g.col, psi0, 100, coin=oracle.HADAMARD)
    assert np.abs(a - b).max() < 1e-14


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6])
def test_fourier_coin_is_unitary(d):
    f = oracle.fourier_coin(d)
    assert np.abs(f @ f.conj().T - np.eye(d)).max() < 1e-14
    assert abs(f[0, 0] - 1 / np.sqrt(d)) < 1e-15 and abs(f[1, 1] - np.exp(2j * np.pi / d) / np.sqrt(d)) < 1e-15


@pytest.mark.parametrize("shift", ["flipflop", "persistent"])
@pytest.mark.parametrize("coin", ["fourier", "grover", "random"])
def test_norm_preserved_on_grid(shift, coin):
    g = I.torus_directed(5, 6)
    if coin == "random":
        q, _ = np.linalg.qr(np.random.default_rng(5).normal(size=(4, 4)) +
                            1j * np.random.default_rng(6).normal(size=(4, 4)))
        coin = q
    psi0 = I.random_state(g.n_arcs, 9)
    out = oracle.coined_evolve_general(g.row_ptr, g.col, psi0, 40, coin=coin, shift=shift, dims=(5, 6),
                                       marked=[3, 17])
    assert abs(np.linalg.norm(out) - 1.0) < 1e-13


def test_uniform_fixed_point_persistent_grover():
    g = I.torus_directed(5, 7)
    u = I.uniform(g.n_arcs)
    out = oracle.coined_evolve_general(g.row_ptr, g.col, u, 9, coin="grover", shift="persistent", dims=(5, 7))
    assert np.abs(out - u).max() < 1e-15


def test_random_unitary_coin_matches_dense_flipflop():
    l1, l2 = 3, 4
    g = I.torus_directed(l1, l2)
    q, _ = np.linalg.qr(np.random.default_rng(1).normal(size=(4, 4)) +
                        1j * np.random.default_rng(2).normal(size=(4, 4)))
    na = g.n_arcs
    shift = np.zeros((na, na))
    for v in range(g.n):
        for w in g.col[g.row_ptr[v]:g.row_ptr[v + 1]]:
            shift[I.arc_index(g, int(w), v), I.arc_index(g, v, int(w))] = 1.0   # |v,w> -> |w,v>
    coin = np.kron(np.eye(g.n), q)        # rows are contiguous blocks of 4 arcs in row order
    u = shift @ coin
    psi0 = I.random_state(na, 4)
    want = np.linalg.matrix_power(u, 3) @ psi0
    got = oracle.coined_evolve_general(g.row_ptr, g.col, psi0, 3, coin=q)
    assert np.abs(got - want).max() < 1e-13


def test_hadamard_moving_shift_walk_is_symmetric():
    n, steps = 101, 40
    g = I.cycle(n)
    psi0 = np.zeros(g.n_arcs, dtype=np.complex128)
    psi0[I.arc_index(g, 0, 1)] = 1 / np.sqrt(2)
    psi0[I.arc_index(g, 0, n - 1)] = 1j / np.sqrt(2)
    out = oracle.coined_evolve_general(g.row_ptr, g.col, psi0, steps, coin="hadamard", shift="persistent",
                                       dims=(n,))
    p = oracle.coined_prob(g.row_ptr, g.col, out)
    x = np.arange(n)
    signed = (x + n // 2) % n - n // 2                       # position in [-50, 50]
    assert np.abs(p - p[(-x) % n]).max() < 1e-14            # mirror symmetric
    assert p[signed % 2 == 1].max() == 0.0                   # even sites only after even steps
    assert abs(p.sum() - 1) < 1e-13
    # ballistic spreading: the two peaks sit just inside |x| = t / sqrt 2
    peak = abs(signed[np.argmax(p)])
    assert steps / np.sqrt(2) - 4 <= peak <= steps / np.sqrt(2)
    # on a cycle the flip-flop shift is the moving one followed by a swap of the
    # two coin labels at each vertex: the states differ, the label-summed
    # distribution of this symmetric start does not
    ff = oracle.coined_evolve(g.row_ptr, g.col, psi0, steps, coin=oracle.HADAMARD)
    assert np.abs(ff - out).max() > 1e-3
    assert np.abs(oracle.coined_prob(g.row_ptr, g.col, ff) - p).max() < 1e-14


def test_persistent_successor_rejects_non_lattice():
    g = I.random_regular(20, 3, seed=1)
    with pytest.raises(ValueError):
        oracle.persistent_successor(g.row_ptr, g.col, (20,))
