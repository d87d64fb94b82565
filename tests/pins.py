"""Brute-force constructions used to pin the oracle (tests only).

These build the walk operators as dense matrices straight from the
definitions and evolve with dense products or an eigendecomposition, a
route that shares nothing with the oracle's per-element loops.
"""
from __future__ import annotations

import numpy as np


def arcs_of(g):
    """List of (tail, head) in CSR order and a dict arc -> index."""
    tails = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    arcs = list(zip(tails.tolist(), g.col.tolist()))
    return arcs, {a: i for i, a in enumerate(arcs)}


def dense_shift(g):
    """Permutation matrix of S|v,w> = |w,v>: column (v,w) has its 1 in row (w,v)."""
    arcs, index = arcs_of(g)
    m = len(arcs)
    s = np.zeros((m, m))
    for j, (v, w) in enumerate(arcs):
        s[index[(w, v)], j] = 1.0
    return s


def dense_coin(g, coin="grover", marked=()):
    """Block-diagonal coin on the arc basis (blocks = CSR rows, in row order)."""
    m = g.n_arcs
    c = np.zeros((m, m), dtype=np.complex128)
    marked = set(int(x) for x in marked)
    for v in range(g.n):
        lo, hi = int(g.row_ptr[v]), int(g.row_ptr[v + 1])
        d = hi - lo
        if d == 0:
            continue
        if v in marked:
            c[lo:hi, lo:hi] = -np.eye(d)
        elif coin == "hadamard":
            assert d == 2
            c[lo:hi, lo:hi] = np.array([[1, 1], [1, -1]]) / np.sqrt(2)
        else:
            c[lo:hi, lo:hi] = 2.0 / d * np.ones((d, d)) - np.eye(d)
    return c


def dense_adjacency(g):
    a = np.zeros((g.n, g.n))
    for v in range(g.n):
        a[v, g.row(v)] = 1.0
    return a


def dense_hamiltonian(g, gamma, marked=()):
    h = -gamma * dense_adjacency(g)
    for v in marked:
        h[v, v] -= 1.0
    return h


def expm_eigh(h, t, psi0):
    """exp(-iHt) psi0 for real symmetric H by eigendecomposition."""
    w, v = np.linalg.eigh(h)
    return v @ (np.exp(-1j * w * t) * (v.T @ psi0))


def taylor_eigh(h, dt, K, steps, psi0):
    """T_K(-iH dt)^steps psi0 via eigenvalues and numpy's polynomial evaluation."""
    from math import factorial

    w, v = np.linalg.eigh(h)
    coeffs = np.array([1.0 / factorial(k) for k in range(K + 1)])
    scal = np.polynomial.polynomial.polyval(-1j * w * dt, coeffs)
    return v @ (scal ** steps * (v.T @ psi0))
