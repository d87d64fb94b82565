"""FP64 CPU oracle for the quantum-walk hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the HIP engine and imports nothing from it; the two meet only at
the seeded input generators, which hold none of the walk arithmetic.

Contents
--------
* ``qw_oracle.c`` (loaded here through ctypes): the coined step (Grover,
  Hadamard, Fourier and matrix coins, flip-flop and persistent shifts), the
  Szegedy and staggered walks and the CTQW Taylor step, written out from
  their definitions, plus probabilities.
* :mod:`oracle.taylor`: the truncation-order / step-size rule for the
  Taylor propagator.
* :mod:`oracle.closed_forms`: exact results the physics fixes (Bessel
  images on cycles, Kronecker-product torus, complete-graph search, the
  symmetric-subspace reduction of hypercube search), used as pins and as
  full-size checks.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qw_oracle.c")
_LIB = os.path.join(_HERE, "libqworacle.so")

GROVER = 0
HADAMARD = 1

FAULTS = {
    "coin_delta_sign": 1,
    "no_shift": 2,
    "head_prob": 3,
    "ctqw_no_mark": 4,
    "ctqw_plus_i": 5,
    "taylor_short": 6,
    "hadamard_swap": 7,
    "mark_plus": 8,
    "gamma_on_mark": 9,
    "stag_one_proj": 10,
    "stag_reversed": 11,
    "stag_mark_after": 12,
    "stag_theta_sign": 13,
}


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain IEEE double, no contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    cmd = ["gcc", "-std=gnu11", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = C.CDLL(_LIB)
        i64p = C.POINTER(C.c_int64)
        i32p = C.POINTER(C.c_int32)
        u8p = C.POINTER(C.c_uint8)
        dp = C.POINTER(C.c_double)
        lib.orc_reverse_arcs.argtypes = [C.c_int64, i64p, i32p, i64p]
        lib.orc_reverse_arcs.restype = C.c_int
        lib.orc_coined_evolve.argtypes = [C.c_int64, i64p, i32p, i64p, C.c_int, u8p, dp, C.c_int64]
        lib.orc_coined_evolve.restype = C.c_int
        lib.orc_coined_evolve_general.argtypes = [C.c_int64, i64p, i64p, dp, C.c_int64, u8p, dp, C.c_int64]
        lib.orc_coined_evolve_general.restype = C.c_int
        lib.orc_szegedy_evolve.argtypes = [C.c_int64, i64p, i64p, dp, u8p, dp, C.c_int64]
        lib.orc_szegedy_evolve.restype = C.c_int
        lib.orc_staggered_evolve.argtypes = [C.c_int64, C.c_int32, i64p, i64p, i32p, dp, u8p, i32p, dp, u8p,
                                             dp, C.c_int64]
        lib.orc_staggered_evolve.restype = C.c_int
        lib.orc_coined_prob.argtypes = [C.c_int64, i64p, i32p, dp, dp]
        lib.orc_coined_prob.restype = None
        lib.orc_ctqw_evolve.argtypes = [C.c_int64, i64p, i32p, C.c_double, u8p, C.c_double,
                                        C.c_int32, dp, C.c_int64]
        lib.orc_ctqw_evolve.restype = C.c_int
        lib.orc_vertex_prob.argtypes = [C.c_int64, dp, dp]
        lib.orc_vertex_prob.restype = None
        lib.orc_set_fault.argtypes = [C.c_int]
        lib.orc_set_threads.argtypes = [C.c_int]
        lib.orc_max_threads.restype = C.c_int
        _lib = lib
    return _lib


def _ptr(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def _csr(row_ptr, col):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    return rp, cl


def _marked_bytes(n, marked):
    m = np.zeros(max(n, 1), dtype=np.uint8)
    if marked is not None and len(marked):
        m[np.asarray(marked, dtype=np.int64)] = 1
    return m


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def max_threads() -> int:
    return int(_load().orc_max_threads())


class fault:
    """Context manager that plants one named mistake in the oracle."""

    def __init__(self, name: str):
        self.code = FAULTS[name]

    def __enter__(self):
        _load().orc_set_fault(self.code)
        return self

    def __exit__(self, *exc):
        _load().orc_set_fault(0)
        return False


def reverse_arcs(row_ptr, col) -> np.ndarray:
    """rev[a] = position of the reverse arc; ValueError if the graph is invalid."""
    rp, cl = _csr(row_ptr, col)
    n = rp.size - 1
    rev = np.empty(max(cl.size, 1), dtype=np.int64)
    st = _load().orc_reverse_arcs(n, _ptr(rp, C.c_int64), _ptr(cl, C.c_int32), _ptr(rev, C.c_int64))
    if st == -1:
        raise ValueError("adjacency is not symmetric")
    if st == -2:
        raise ValueError("self-loop")
    return rev[:cl.size]


def coined_evolve(row_ptr, col, psi0, steps: int, coin: int = GROVER, marked=None) -> np.ndarray:
    """(S C)^steps psi0 on the CSR arc basis; returns complex128[n_arcs]."""
    rp, cl = _csr(row_ptr, col)
    n = rp.size - 1
    rev = reverse_arcs(rp, cl)
    if rev.size == 0:
        rev = np.zeros(1, np.int64)
    psi = np.ascontiguousarray(np.array(psi0, dtype=np.complex128, copy=True))
    if psi.size != cl.size:
        raise ValueError("state length must equal the arc count")
    m = _marked_bytes(n, marked)
    buf = psi.view(np.float64) if psi.size else np.zeros(2, np.float64)
    st = _load().orc_coined_evolve(n, _ptr(rp, C.c_int64), _ptr(cl, C.c_int32),
                                   _ptr(rev, C.c_int64), int(coin), _ptr(m, C.c_uint8),
                                   _ptr(buf, C.c_double), int(steps))
    if st == -3:
        raise ValueError("Hadamard coin needs degree 2 at every unmarked vertex")
    if st != 0:
        raise RuntimeError(f"oracle coined evolve failed ({st})")
    return psi


def fourier_coin(d: int) -> np.ndarray:
    """The d x d Fourier coin, F[j][k] = exp(2 pi i j k / d) / sqrt(d) (Sec. 3.2)."""
    j = np.arange(d)
    return np.exp(2j * np.pi * np.outer(j, j) / d) / np.sqrt(d)


def persistent_successor(row_ptr, col, dims) -> np.ndarray:
    """For each arc v -> w of a cycle (dims = (n,)) or a periodic l1 x l2 grid
    (dims = (l1, l2), vertex r*l2 + c), the index of the arc w -> u that keeps
    the direction: u = w + (w - v) in lattice coordinates, taken modulo the
    sides.  The persistent shift sends the amplitude of arc v -> w there."""
    rp, cl = _csr(row_ptr, col)
    n = rp.size - 1
    dims = tuple(int(x) for x in dims)
    if dims == (n,):
        coords = np.arange(n)[:, None]
    elif len(dims) == 2 and dims[0] * dims[1] == n:
        v = np.arange(n)
        coords = np.stack([v // dims[1], v % dims[1]], axis=1)
    else:
        raise ValueError("dims must be (n,) for a cycle or (l1, l2) with l1 * l2 = n")
    side = np.array(dims)
    tails = np.repeat(np.arange(n), np.diff(rp))
    step = (coords[cl] - coords[tails]) % side        # displacement w - v, modulo the sides
    ahead = (coords[cl] + step) % side                # u = w + (w - v)
    u = ahead[:, 0] if len(dims) == 1 else ahead[:, 0] * dims[1] + ahead[:, 1]
    # the arc w -> u: look the key (w, u) up among the keys (tail, head) of all arcs
    key = tails * np.int64(n) + cl
    order = np.argsort(key, kind="stable")
    want = cl.astype(np.int64) * np.int64(n) + u
    pos = np.searchsorted(key[order], want)
    pos = np.minimum(pos, max(cl.size - 1, 0))
    succ = order[pos].astype(np.int64) if cl.size else np.zeros(0, np.int64)
    bad = np.flatnonzero(key[succ] != want) if cl.size else np.zeros(0, np.int64)
    if bad.size:
        a = int(bad[0])
        raise ValueError(f"arc {a}: no arc {int(cl[a])} -> {int(u[a])}")
    if np.unique(succ).size != succ.size:
        raise ValueError("the persistent successor is not a permutation of the arcs")
    return succ


def coined_evolve_general(row_ptr, col, psi0, steps: int, coin="grover", shift: str = "flipflop",
                          dims=None, marked=None) -> np.ndarray:
    """(S C)^steps psi0 with coin "grover", "hadamard", "fourier" or a d x d
    matrix (applied in each row's order, the coin basis; marked vertices take
    -I), and shift "flipflop" (S|v,w> = |w,v>) or "persistent" (the arc
    straight ahead on a cycle or periodic grid given by dims)."""
    rp, cl = _csr(row_ptr, col)
    n = rp.size - 1
    if shift == "flipflop":
        dest = reverse_arcs(rp, cl)
    elif shift == "persistent":
        dest = persistent_successor(rp, cl, dims)
    else:
        raise ValueError("shift is 'flipflop' or 'persistent'")
    if dest.size == 0:
        dest = np.zeros(1, np.int64)
    degs = np.diff(rp)
    d = int(degs.max()) if degs.size else 0
    if isinstance(coin, str) and coin == "grover":
        mat = None
    elif isinstance(coin, str) and coin == "hadamard":
        mat = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2)
    elif isinstance(coin, str) and coin == "fourier":
        mat = fourier_coin(d)
    else:
        mat = np.asarray(coin, dtype=np.complex128)
        if mat.ndim != 2 or mat.shape[0] != mat.shape[1]:
            raise ValueError("coin matrix must be square")
    psi = np.ascontiguousarray(np.array(psi0, dtype=np.complex128, copy=True))
    if psi.size != cl.size:
        raise ValueError("state length must equal the arc count")
    m = _marked_bytes(n, marked)
    buf = psi.view(np.float64) if psi.size else np.zeros(2, np.float64)
    mbuf = None if mat is None else np.ascontiguousarray(mat, dtype=np.complex128).view(np.float64)
    st = _load().orc_coined_evolve_general(n, _ptr(rp, C.c_int64), _ptr(np.ascontiguousarray(dest), C.c_int64),
                                           None if mbuf is None else _ptr(mbuf, C.c_double),
                                           0 if mat is None else mat.shape[0], _ptr(m, C.c_uint8),
                                           _ptr(buf, C.c_double), int(steps))
    if st == -3:
        raise ValueError("the coin matrix's size differs from a vertex degree")
    if st != 0:
        raise RuntimeError(f"oracle coined evolve failed ({st})")
    return psi


def szegedy_evolve(row_ptr, col, psi0, steps: int, p_arc, marked=None) -> np.ndarray:
    """Szegedy walk (S (2 Pi - I))^steps psi0 on the arc basis for the
    transition probabilities p_arc (one per arc in CSR order, P[tail][head];
    each row sums to 1); marked vertices take -I."""
    rp, cl = _csr(row_ptr, col)
    n = rp.size - 1
    p_arc = np.asarray(p_arc, dtype=np.float64)
    if p_arc.size != cl.size or np.any(p_arc < 0):
        raise ValueError("one non-negative transition probability per arc")
    rev = reverse_arcs(rp, cl)
    if rev.size == 0:
        rev = np.zeros(1, np.int64)
    sq = np.ascontiguousarray(np.sqrt(p_arc)) if p_arc.size else np.zeros(1)
    psi = np.ascontiguousarray(np.array(psi0, dtype=np.complex128, copy=True))
    if psi.size != cl.size:
        raise ValueError("state length must equal the arc count")
    m = _marked_bytes(n, marked)
    buf = psi.view(np.float64) if psi.size else np.zeros(2, np.float64)
    st = _load().orc_szegedy_evolve(n, _ptr(rp, C.c_int64), _ptr(rev, C.c_int64), _ptr(sq, C.c_double),
                                    _ptr(m, C.c_uint8), _ptr(buf, C.c_double), int(steps))
    if st != 0:
        raise RuntimeError(f"oracle Szegedy evolve failed ({st})")
    return psi


def staggered_evolve(n: int, tessellations, psi0, steps: int, marked=None) -> np.ndarray:
    """Staggered walk (U_T ... U_1 R_M)^steps psi0 on the vertex basis.

    ``tessellations``: a sequence of objects with ``poly_ptr`` (int64,
    polygons + 1 entries), ``poly_vert`` (int32, n entries: polygon p is
    poly_vert[poly_ptr[p]:poly_ptr[p+1]], every vertex exactly once),
    ``amp`` (None for uniform 1/sqrt|alpha|, else n reals aligned with
    poly_vert, each polygon's squares summing to 1) and ``theta`` (None for
    the reflection 2P - I, else exp(i theta (2P - I))).  Applied in sequence
    order after the phase flip of the marked vertices."""
    n = int(n)
    T = len(tessellations)
    n_poly = np.zeros(max(T, 1), np.int64)
    ptrs, verts, amps = [], [], []
    has_amp = np.zeros(max(T, 1), np.uint8)
    form = np.zeros(max(T, 1), np.int32)
    theta = np.zeros(max(T, 1), np.float64)
    for t, tess in enumerate(tessellations):
        pp = np.ascontiguousarray(tess.poly_ptr, dtype=np.int64)
        vv = np.ascontiguousarray(tess.poly_vert, dtype=np.int32)
        if vv.size != n or pp[0] != 0 or pp[-1] != n or np.any(np.diff(pp) <= 0):
            raise ValueError("a tessellation must split the n vertices into non-empty polygons")
        if not np.array_equal(np.sort(vv), np.arange(n)):
            raise ValueError("a tessellation must hold every vertex exactly once")
        n_poly[t] = pp.size - 1
        ptrs.append(pp)
        verts.append(vv)
        if tess.amp is not None:
            has_amp[t] = 1
            amps.append(np.ascontiguousarray(tess.amp, dtype=np.float64))
        else:
            amps.append(np.zeros(n, np.float64))
        if tess.theta is not None:
            form[t] = 1
            theta[t] = float(tess.theta)
    pp_all = np.concatenate(ptrs) if ptrs else np.zeros(1, np.int64)
    vv_all = np.concatenate(verts) if verts and n else np.zeros(1, np.int32)
    aa_all = np.concatenate(amps) if amps and n else np.zeros(1, np.float64)
    psi = np.ascontiguousarray(np.array(psi0, dtype=np.complex128, copy=True))
    if psi.size != n:
        raise ValueError("state length must equal the vertex count")
    m = _marked_bytes(n, marked)
    buf = psi.view(np.float64) if psi.size else np.zeros(2, np.float64)
    st = _load().orc_staggered_evolve(n, T, _ptr(n_poly, C.c_int64), _ptr(pp_all, C.c_int64),
                                      _ptr(vv_all, C.c_int32), _ptr(aa_all, C.c_double), _ptr(has_amp, C.c_uint8),
                                      _ptr(form, C.c_int32), _ptr(theta, C.c_double), _ptr(m, C.c_uint8),
                                      _ptr(buf, C.c_double), int(steps))
    if st != 0:
        raise RuntimeError(f"oracle staggered evolve failed ({st})")
    return psi


def coined_prob(row_ptr, col, psi) -> np.ndarray:
    rp, cl = _csr(row_ptr, col)
    n = rp.size - 1
    x = np.ascontiguousarray(psi, dtype=np.complex128)
    p = np.empty(max(n, 1), dtype=np.float64)
    buf = x.view(np.float64) if x.size else np.zeros(2)
    _load().orc_coined_prob(n, _ptr(rp, C.c_int64), _ptr(cl, C.c_int32), _ptr(buf, C.c_double),
                            _ptr(p, C.c_double))
    return p[:n]


def ctqw_evolve(row_ptr, col, psi0, steps: int, gamma: float, dt: float, K: int,
                marked=None) -> np.ndarray:
    """T_K(-i H dt)^steps psi0 with H = -gamma A - sum_M |v><v| (power form)."""
    rp, cl = _csr(row_ptr, col)
    n = rp.size - 1
    psi = np.ascontiguousarray(np.array(psi0, dtype=np.complex128, copy=True))
    if psi.size != n:
        raise ValueError("state length must equal the vertex count")
    m = _marked_bytes(n, marked)
    cl2 = cl if cl.size else np.zeros(1, np.int32)
    st = _load().orc_ctqw_evolve(n, _ptr(rp, C.c_int64), _ptr(cl2, C.c_int32), float(gamma),
                                 _ptr(m, C.c_uint8), float(dt), int(K),
                                 _ptr(psi.view(np.float64), C.c_double), int(steps))
    if st != 0:
        raise RuntimeError(f"oracle ctqw evolve failed ({st})")
    return psi


def vertex_prob(psi) -> np.ndarray:
    x = np.ascontiguousarray(psi, dtype=np.complex128)
    p = np.empty(max(x.size, 1), dtype=np.float64)
    buf = x.view(np.float64) if x.size else np.zeros(2)
    _load().orc_vertex_prob(x.size, _ptr(buf, C.c_double), _ptr(p, C.c_double))
    return p[:x.size]


from . import closed_forms, taylor  # noqa: E402,F401
