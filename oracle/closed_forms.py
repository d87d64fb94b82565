"""Exact results the physics fixes, used as pins and full-size checks.

TEST INFRASTRUCTURE ONLY (see the package docstring).

All follow from the paper's definitions (Sec. 3.1: H = -gamma A -
sum_M |v><v|, U(t) = exp(-iHt); Sec. 3.2: U = S C with flip-flop shift and
Grover coin) plus standard special functions:

* CTQW on a cycle, no marks: exp(-iHt) = exp(i gamma t A).  On the infinite
  line the Jacobi-Anger expansion exp(i z cos th) = sum_n i^n J_n(z) e^{i n th}
  gives the amplitude i^x J_x(2 gamma t) at distance x from the start; on a
  cycle of N vertices the images x + mN add up (method of images).
* CTQW on an L1 x L2 torus: A is the Kronecker sum of two cycle adjacencies,
  so the propagator factorises into the product of two cycle propagators.
* CTQW search on the complete graph K_N with gamma = 1/N and one marked
  vertex w, started uniform: in span{|w>, uniform-over-the-rest} the
  Hamiltonian has eigenvalues -(1 +- 1/sqrt N) (up to a global shift), and
  p_w(t) = sin^2(t/sqrt N) + cos^2(t/sqrt N)/N.
* Coined Grover search on the hypercube Q_n with the coin -I at vertex 0,
  started uniform over arcs: the state stays invariant under coordinate
  permutations, so it lives in a 2n-dimensional space indexed by the weight
  k = |v| and the arc direction (out: flips a 0-bit, toward weight k+1; in:
  flips a 1-bit).  See :func:`hypercube_search_reduced`.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import jv


def _line_amplitude(x: np.ndarray, z: float) -> np.ndarray:
    """i^x J_x(z), valid for negative x as well (i^-x J_-x = i^x J_x)."""
    xa = np.abs(x)
    ph = np.exp(1j * (math.pi / 2) * (xa % 4))
    return ph * jv(xa, z)


def cycle_ctqw(n: int, gamma: float, t: float, x0: int = 0, idx=None) -> np.ndarray:
    """exp(-iHt)|x0> on the n-cycle, H = -gamma A, by the method of images."""
    z = 2.0 * gamma * t
    if idx is None:
        idx = np.arange(n)
    idx = np.asarray(idx, dtype=np.int64)
    x = (idx - x0) % n
    x = np.where(x > n // 2, x - n, x)  # nearest representative
    out = np.zeros(idx.shape, dtype=np.complex128)
    # J_m(z) is below 1e-30 once |m| > z + 40 + 10*z^(1/3) (far past the turning point)
    reach = int(z + 60 + 12 * max(z, 1.0) ** (1.0 / 3.0))
    mmax = reach // n + 2
    for m in range(-mmax, mmax + 1):
        out += _line_amplitude(x + m * n, z)
    return out


def torus_ctqw(l1: int, l2: int, gamma: float, t: float, v0: int, idx=None) -> np.ndarray:
    """exp(-iHt)|v0> on the l1 x l2 torus (v = r*l2 + c), H = -gamma A."""
    r0, c0 = divmod(int(v0), l2)
    if idx is None:
        idx = np.arange(l1 * l2)
    idx = np.asarray(idx, dtype=np.int64)
    r, c = idx // l2, idx % l2
    return cycle_ctqw(l1, gamma, t, r0, r) * cycle_ctqw(l2, gamma, t, c0, c)


def complete_search_prob(n: int, t) -> np.ndarray:
    """Success probability of CTQW search on K_n (gamma = 1/n, one mark, uniform start)."""
    s = np.sqrt(n)
    tt = np.asarray(t, dtype=np.float64)
    return np.sin(tt / s) ** 2 + np.cos(tt / s) ** 2 / n


def hypercube_search_reduced(dim: int, steps: int, record_marked: bool = False):
    """Coined Grover search on Q_dim with -I at vertex 0, uniform start.

    Works in the normalised reduced amplitudes
        o_k  (k = 0..dim-1): sqrt(#out-arcs at weight k) * amplitude per out-arc
        i_k  (k = 1..dim)  : sqrt(#in-arcs  at weight k) * amplitude per in-arc
    with #out(k) = C(n,k)(n-k), #in(k) = C(n,k) k.  Grover on a vertex of
    weight k with (n-k) out-arcs sharing one amplitude and k in-arcs sharing
    another acts on (o_k, i_k) as
        [[2(n-k)/n - 1, 2 sqrt(k(n-k))/n], [2 sqrt(k(n-k))/n, 2k/n - 1]],
    the marked vertex (k = 0) gets -1, and the flip-flop shift sends every
    out-arc at weight k to an in-arc at weight k+1 (#out(k) = #in(k+1)):
        i'_{k+1} = phi_out(k),  o'_k = phi_in(k+1).

    Returns (o, i) after `steps` steps (arrays of length dim+1, o[dim] = 0,
    i[0] = 0) and, if record_marked, the list of p_marked = |o_0|^2 for
    steps 0..steps.
    """
    n = dim
    k = np.arange(n + 1, dtype=np.float64)
    binom = np.array([math.comb(n, int(j)) for j in range(n + 1)], dtype=np.float64)
    n_out = binom * (n - k)
    n_in = binom * k
    amp0 = 1.0 / math.sqrt(n * 2.0 ** n)
    o = np.sqrt(n_out) * amp0 + 0j
    i = np.sqrt(n_in) * amp0 + 0j
    a = 2 * (n - k) / n - 1
    b = 2 * np.sqrt(k * (n - k)) / n
    c = 2 * k / n - 1
    hist = [abs(o[0]) ** 2] if record_marked else None
    for _ in range(steps):
        fo = a * o + b * i
        fi = b * o + c * i
        fo[0] = -o[0]
        fi[0] = 0.0
        o_new = np.zeros_like(o)
        i_new = np.zeros_like(i)
        i_new[1:] = fo[:-1]
        o_new[:-1] = fi[1:]
        o, i = o_new, i_new
        if record_marked:
            hist.append(abs(o[0]) ** 2)
    return o, i, hist


def hypercube_search_state(dim: int, steps: int, row_ptr, col, idx=None) -> np.ndarray:
    """Full arc amplitudes (CSR order) of hypercube search from the reduced model.

    Arc (v, w) with w = v xor 2^j is an out-arc when bit j of v is 0.
    """
    o, i, _ = hypercube_search_reduced(dim, steps)
    n = dim
    k = np.arange(n + 1, dtype=np.float64)
    binom = np.array([math.comb(n, int(j)) for j in range(n + 1)], dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        per_out = np.where(k < n, o / np.sqrt(binom * (n - k)), 0)
        per_in = np.where(k > 0, i / np.sqrt(binom * k), 0)
    rp = np.asarray(row_ptr, dtype=np.int64)
    cl = np.asarray(col, dtype=np.int64)
    if idx is None:
        idx = np.arange(cl.size, dtype=np.int64)
    idx = np.asarray(idx, dtype=np.int64)
    tail = np.searchsorted(rp, idx, side="right") - 1
    head = cl[idx]
    weight = np.array([bin(int(v)).count("1") for v in tail], dtype=np.int64) \
        if idx.size < 4096 else _popcount(tail)
    out_arc = head > tail  # flipping a 0-bit increases the label
    return np.where(out_arc, per_out[weight], per_in[weight])


def _popcount(v: np.ndarray) -> np.ndarray:
    v = v.astype(np.uint64)
    c = np.zeros(v.shape, dtype=np.int64)
    while np.any(v):
        c += (v & np.uint64(1)).astype(np.int64)
        v >>= np.uint64(1)
    return c
