"""Pins for the oracle's Szegedy walk, U = S (2 Pi - I) with Pi = sum_x
|alpha_x><alpha_x|, alpha_x = sum_y sqrt(P_xy) |x,y>, and S the swap:

* with P the simple random walk (P_xy = 1/d_x) it is the Grover coined walk
  with the flip-flop shift, whose oracle path is pinned elsewhere;
* it equals the dense product of the swap (built here from arc positions)
  and the reflection (built from the alpha_x);
* Szegedy's spectral theorem: for a reversible P, every eigenvalue lambda of
  the discriminant D_xy = sqrt(P_xy P_yx) with |lambda| < 1 gives the pair of
  eigenvalues exp(+-i arccos lambda) of U;
* it preserves the norm for any stochastic P.
"""
import numpy as np
import pytest

import oracle
from paper_2406_08186_amd import inputs as I


def _weights_p(g, seed):
    """A reversible walk: symmetric positive edge weights, P_xy = w_xy / W_x."""
    rng = np.random.default_rng(seed)
    w = {}
    for v in range(g.n):
        for u in g.row(v):
            key = (min(v, int(u)), max(v, int(u)))
            if key not in w:
                w[key] = rng.uniform(0.2, 2.0)
    p = np.empty(g.n_arcs)
    W = np.zeros(g.n)
    for v in range(g.n):
        for a in range(g.row_ptr[v], g.row_ptr[v + 1]):
            u = int(g.col[a])
            W[v] += w[(min(v, u), max(v, u))]
    for v in range(g.n):
        for a in range(g.row_ptr[v], g.row_ptr[v + 1]):
            u = int(g.col[a])
            p[a] = w[(min(v, u), max(v, u))] / W[v]
    return p, w, W


def _graphs():
    return [I.random_mixed(12, seed=3, n_isolated=0), I.cycle(9), I.complete(5), I.erdos_renyi(14, 0.4, seed=2)]


@pytest.mark.parametrize("gi", range(4))
def test_simple_random_walk_is_grover(gi):
    g = _graphs()[gi]
    deg = np.diff(g.row_ptr)
    p = np.repeat(1.0 / np.maximum(deg, 1), deg)
    psi0 = I.random_state(g.n_arcs, gi)
    marked = [1]
    a = oracle.szegedy_evolve(g.row_ptr, g.col, psi0, 17, p, marked=marked)
    b = oracle.coined_evolve(g.row_ptr, g.col, psi0, 17, marked=marked)
    assert np.abs(a - b).max() < 1e-13


@pytest.mark.parametrize("gi", range(4))
def test_matches_dense_operators(gi):
    g = _graphs()[gi]
    p, _, _ = _weights_p(g, gi + 10)
    na = g.n_arcs
    swap = np.zeros((na, na))
    for v in range(g.n):
        for u in g.row(v):
            swap[I.arc_index(g, int(u), v), I.arc_index(g, v, int(u))] = 1.0
    refl = -np.eye(na)
    for v in range(g.n):
        alpha = np.zeros(na)
        for a in range(g.row_ptr[v], g.row_ptr[v + 1]):
            alpha[a] = np.sqrt(p[a])
        refl += 2 * np.outer(alpha, alpha)
    u = swap @ refl
    psi0 = I.random_state(na, 5)
    want = np.linalg.matrix_power(u, 6) @ psi0
    assert np.abs(oracle.szegedy_evolve(g.row_ptr, g.col, psi0, 6, p) - want).max() < 1e-12


@pytest.mark.parametrize("gi", [0, 1, 3])
def test_spectral_theorem(gi):
    g = _graphs()[gi]
    p, w, W = _weights_p(g, gi + 20)
    # U column by column from the oracle (one step on each basis state)
    na = g.n_arcs
    u = np.stack([oracle.szegedy_evolve(g.row_ptr, g.col, np.eye(na)[:, j], 1, p) for j in range(na)], axis=1)
    mu = np.linalg.eigvals(u)
    assert np.abs(np.abs(mu) - 1).max() < 1e-12
    d = np.zeros((g.n, g.n))
    for (x, y), wxy in w.items():
        d[x, y] = d[y, x] = wxy / np.sqrt(W[x] * W[y])       # sqrt(P_xy P_yx)
    lam = np.linalg.eigvalsh(d)
    inner = np.sort(lam[np.abs(lam) < 1 - 1e-9])
    pairs = np.sort(mu.real[np.abs(mu.imag) > 1e-7])
    assert pairs.size == 2 * inner.size
    assert np.abs(pairs - np.sort(np.repeat(inner, 2))).max() < 1e-9


def test_norm_preserved_non_reversible():
    g = I.erdos_renyi(40, 0.2, seed=7)
    rng = np.random.default_rng(8)
    raw = rng.uniform(0.1, 1.0, size=g.n_arcs)
    sums = np.add.reduceat(raw, g.row_ptr[:-1]) if g.n_arcs else raw
    p = raw / np.repeat(sums, np.diff(g.row_ptr))
    out = oracle.szegedy_evolve(g.row_ptr, g.col, I.random_state(g.n_arcs, 2), 50, p, marked=[0, 5])
    assert abs(np.linalg.norm(out) - 1) < 1e-13
