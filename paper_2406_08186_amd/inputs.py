"""Seeded synthetic inputs: graph families and initial states.

This module is shared by the HIP path's tests and bench and by the CPU
oracle's tests.  It draws graphs, states and staggered-walk tessellations
(vertex partitions) and does nothing else: no coin, no shift, no
Hamiltonian, no reflection, no probability -- none of the walk arithmetic.

Graphs are returned as a symmetric 0/1 adjacency pattern in CSR form
(``row_ptr`` int64[n+1], ``col`` int32[nnz]).  Row ``v`` lists the heads of
the arcs whose tail is ``v``; with the paper's arc basis (Sec. 3.2: arcs
ordered tail-major, then by head label) a row is sorted ascending, which
every generator here emits except :func:`cycle`, whose rows are in direction
order (+1 neighbour first, then -1) so that position-coin labels |v,0>, |v,1>
are "step right" and "step left" on every vertex.

The graph families follow the ones the paper names (cycle, two-dimensional
grid, hypercube, arbitrary adjacency; Sec. 3.1) plus the random families
the benchmark workloads use (random d-regular, Erdos-Renyi).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Graph:
    """Symmetric adjacency pattern in CSR form (host arrays)."""

    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col: np.ndarray  # int32[nnz]
    name: str = "graph"

    @property
    def n_arcs(self) -> int:
        return int(self.row_ptr[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def row(self, v: int) -> np.ndarray:
        return self.col[self.row_ptr[v]:self.row_ptr[v + 1]]


def _from_rows(n: int, heads: np.ndarray, tails: np.ndarray, name: str,
               sort_rows: bool = True) -> Graph:
    """Build CSR from arc lists (tail -> head); rows sorted by head when asked."""
    tails = np.asarray(tails, dtype=np.int64)
    heads = np.asarray(heads, dtype=np.int64)
    if sort_rows:
        keys = tails * np.int64(max(n, 1)) + heads
        keys.sort()
        t, h = np.divmod(keys, np.int64(max(n, 1)))
    else:
        order = np.argsort(tails, kind="stable")
        t = tails[order]
        h = heads[order]
    counts = np.bincount(t, minlength=n).astype(np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Graph(n=n, row_ptr=row_ptr, col=h.astype(np.int32), name=name)


def from_edges(n: int, edges, name: str = "graph") -> Graph:
    """Undirected simple edge list -> symmetric CSR with sorted rows."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if e.size == 0:
        return Graph(n=n, row_ptr=np.zeros(n + 1, np.int64),
                     col=np.zeros(0, np.int32), name=name)
    tails = np.concatenate([e[:, 0], e[:, 1]])
    heads = np.concatenate([e[:, 1], e[:, 0]])
    return _from_rows(n, heads, tails, name)


def cycle(n: int) -> Graph:
    """Cycle C_n in direction order: row v = [v+1 mod n, v-1 mod n]."""
    if n < 3:
        raise ValueError("a cycle needs at least 3 vertices")
    v = np.arange(n, dtype=np.int64)
    col = np.empty(2 * n, dtype=np.int32)
    col[0::2] = (v + 1) % n
    col[1::2] = (v - 1) % n
    row_ptr = np.arange(0, 2 * n + 1, 2, dtype=np.int64)
    return Graph(n=n, row_ptr=row_ptr, col=col, name=f"cycle{n}")


def cycle_sorted(n: int) -> Graph:
    """Cycle C_n with rows sorted by head label (the paper's default basis)."""
    v = np.arange(n, dtype=np.int64)
    return from_edges(n, np.stack([v, (v + 1) % n], 1), name=f"cycle{n}s")


def torus(l1: int, l2: int) -> Graph:
    """Periodic l1 x l2 grid, vertex v = r*l2 + c, rows sorted."""
    if l1 < 3 or l2 < 3:
        raise ValueError("torus sides must be >= 3")
    n = l1 * l2
    v = np.arange(n, dtype=np.int64)
    r, c = v // l2, v % l2
    nb = np.stack([((r + 1) % l1) * l2 + c, ((r - 1) % l1) * l2 + c,
                   r * l2 + (c + 1) % l2, r * l2 + (c - 1) % l2], 1)
    nb.sort(axis=1)
    row_ptr = np.arange(0, 4 * n + 1, 4, dtype=np.int64)
    return Graph(n=n, row_ptr=row_ptr, col=nb.reshape(-1).astype(np.int32),
                 name=f"torus{l1}x{l2}")


def torus_directed(l1: int, l2: int) -> Graph:
    """Periodic l1 x l2 grid (vertex r*l2 + c) with every row in direction
    order: c+1, c-1, r+1, r-1 (wrapping) -- the coin basis of position-coin
    notation on a grid."""
    if l1 < 3 or l2 < 3:
        raise ValueError("sides must be at least 3")
    v = np.arange(l1 * l2, dtype=np.int64)
    r, c = v // l2, v % l2
    heads = np.stack([r * l2 + (c + 1) % l2, r * l2 + (c - 1) % l2,
                      ((r + 1) % l1) * l2 + c, ((r - 1) % l1) * l2 + c], axis=1)
    row_ptr = np.arange(0, 4 * l1 * l2 + 1, 4, dtype=np.int64)
    return Graph(n=l1 * l2, row_ptr=row_ptr, col=heads.reshape(-1).astype(np.int32),
                 name=f"torus{l1}x{l2}d")


def hypercube(dim: int) -> Graph:
    """Hypercube Q_dim: v ~ v xor 2^j, rows sorted."""
    if dim < 1:
        raise ValueError("dim >= 1")
    n = 1 << dim
    v = np.arange(n, dtype=np.int64)[:, None]
    nb = v ^ (np.int64(1) << np.arange(dim, dtype=np.int64))[None, :]
    nb.sort(axis=1)
    row_ptr = np.arange(0, dim * n + 1, dim, dtype=np.int64)
    return Graph(n=n, row_ptr=row_ptr, col=nb.reshape(-1).astype(np.int32),
                 name=f"hypercube{dim}")


def complete(n: int) -> Graph:
    """Complete graph K_n, rows sorted."""
    if n < 2:
        return Graph(n=n, row_ptr=np.zeros(n + 1, np.int64), col=np.zeros(0, np.int32),
                     name=f"complete{n}")
    tails = np.repeat(np.arange(n, dtype=np.int64), n - 1)
    heads = np.tile(np.arange(n - 1, dtype=np.int64), n)
    heads += heads >= tails  # skip the diagonal: row v lists 0..v-1, v+1..n-1
    row_ptr = np.arange(0, n * (n - 1) + 1, n - 1, dtype=np.int64)
    return Graph(n=n, row_ptr=row_ptr, col=heads.astype(np.int32), name=f"complete{n}")


def random_regular(n: int, d: int, seed: int) -> Graph:
    """Uniform-ish random simple d-regular graph.

    Configuration (pairing) model followed by random edge switchings that
    remove loops and repeated edges; resampled until connected.
    """
    if (n * d) % 2:
        raise ValueError("n*d must be even")
    if d >= n:
        raise ValueError("need d < n")
    rng = np.random.default_rng(seed)
    for _attempt in range(50):
        pts = np.repeat(np.arange(n, dtype=np.int64), d)
        rng.shuffle(pts)
        e = pts.reshape(-1, 2).copy()
        e.sort(axis=1)
        e = _switch_to_simple(e, rng)
        g = from_edges(n, e, name=f"rr{n}d{d}s{seed}")
        if _connected(g):
            return g
    raise RuntimeError("could not draw a connected random regular graph")


def _switch_to_simple(e: np.ndarray, rng) -> np.ndarray:
    """Remove loops and repeated edges by degree-preserving switches.

    A bad edge (a, b) and a random edge (c, d) become (a, c), (b, d) (or
    (a, d), (b, c)) when neither new edge is a loop or already present.
    """
    m = e.shape[0]
    n_hint = np.int64(int(e.max()) + 1)
    for _sweep in range(1000):
        keys = e[:, 0] * n_hint + e[:, 1]
        order = np.argsort(keys, kind="stable")
        sk = keys[order]
        dup = np.zeros(m, dtype=bool)
        dup[order[1:][sk[1:] == sk[:-1]]] = True
        bad = np.flatnonzero((e[:, 0] == e[:, 1]) | dup)
        if bad.size == 0:
            return e
        extra = set()   # keys created during this sweep
        removed = set()

        def present(k):
            if k in extra:
                return True
            if k in removed:
                return False
            i = np.searchsorted(sk, k)
            return i < sk.size and sk[i] == k

        for i in bad.tolist():
            for _try in range(100):
                j = int(rng.integers(m))
                if j == i:
                    continue
                a, b = int(e[i, 0]), int(e[i, 1])
                c, dd = int(e[j, 0]), int(e[j, 1])
                if rng.integers(2):
                    c, dd = dd, c
                n1 = (min(a, c), max(a, c))
                n2 = (min(b, dd), max(b, dd))
                if n1[0] == n1[1] or n2[0] == n2[1] or n1 == n2:
                    continue
                k1 = n1[0] * int(n_hint) + n1[1]
                k2 = n2[0] * int(n_hint) + n2[1]
                if present(k1) or present(k2):
                    continue
                for k_old in (a * int(n_hint) + b if a <= b else b * int(n_hint) + a,
                              min(c, dd) * int(n_hint) + max(c, dd)):
                    extra.discard(k_old)
                    removed.add(k_old)
                extra.add(k1)
                extra.add(k2)
                removed.discard(k1)
                removed.discard(k2)
                e[i] = n1
                e[j] = n2
                break
    raise RuntimeError("edge switching did not converge")


def _connected(g: Graph) -> bool:
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    a = csr_matrix((np.ones(g.n_arcs, np.int8), g.col, g.row_ptr), shape=(g.n, g.n))
    k, _ = connected_components(a, directed=False)
    return k == 1


def erdos_renyi(n: int, p: float, seed: int) -> Graph:
    """G(n, p): each of the n(n-1)/2 pairs is an edge independently with prob. p.

    Isolated vertices are kept.  The edge count is drawn from the binomial
    distribution and that many distinct pairs are drawn uniformly.
    """
    rng = np.random.default_rng(seed)
    total = n * (n - 1) // 2
    m = int(rng.binomial(total, p))
    keys = np.empty(0, dtype=np.int64)
    while keys.size < m:
        need = m - keys.size
        u = rng.integers(0, n, size=int(need * 1.1) + 16, dtype=np.int64)
        w = rng.integers(0, n, size=u.size, dtype=np.int64)
        ok = u != w
        a = np.minimum(u[ok], w[ok])
        b = np.maximum(u[ok], w[ok])
        keys = np.unique(np.concatenate([keys, a * n + b]))
    if keys.size > m:
        keys = rng.choice(keys, size=m, replace=False)
    e = np.stack([keys // n, keys % n], 1)
    return from_edges(n, e, name=f"er{n}p{p:.3g}s{seed}")


def random_mixed(n: int, seed: int, p: float = 0.15, n_isolated: int = 1,
                 n_leaves: int = 2, hub: bool = True) -> Graph:
    """Small irregular test graph: isolated vertices, degree-1 leaves, a hub."""
    rng = np.random.default_rng(seed)
    core = n - n_isolated - n_leaves
    edges = set()
    for u in range(core):
        for w in range(u + 1, core):
            if rng.random() < p:
                edges.add((u, w))
    for u in range(core - 1):  # keep the core connected
        edges.add((u, u + 1))
    if hub and core > 4:
        for w in range(1, core):
            edges.add((0, w))
    for i in range(n_leaves):
        leaf = core + i
        edges.add((int(rng.integers(core)), leaf))
    return from_edges(n, sorted(edges), name=f"mixed{n}s{seed}")


# ---------------------------------------------------------------------------
# Staggered-walk tessellations
# ---------------------------------------------------------------------------

@dataclass
class Tessellation:
    """A partition of the vertices into polygons (cliques of the walk's
    graph): polygon p is ``poly_vert[poly_ptr[p]:poly_ptr[p+1]]``.  ``amp``
    holds one real amplitude per position of ``poly_vert`` (None = uniform);
    ``theta`` None asks for the reflection form, a number for the
    Hamiltonian form with that angle."""

    poly_ptr: np.ndarray  # int64[polygons + 1]
    poly_vert: np.ndarray  # int32[n]
    amp: np.ndarray | None = None
    theta: float | None = None

    @property
    def n_polygons(self) -> int:
        return int(self.poly_ptr.size - 1)

    def sizes(self) -> np.ndarray:
        return np.diff(self.poly_ptr)


def tessellation(polygons, amp=None, theta=None) -> Tessellation:
    """Tessellation from a list of vertex lists (one per polygon)."""
    sizes = np.array([len(p) for p in polygons], dtype=np.int64)
    ptr = np.zeros(sizes.size + 1, np.int64)
    np.cumsum(sizes, out=ptr[1:])
    vert = np.concatenate([np.asarray(p, dtype=np.int64) for p in polygons]) if polygons else np.zeros(0)
    return Tessellation(ptr, vert.astype(np.int32), amp, theta)


def _uniform_tessellation(vert_by_poly: np.ndarray) -> Tessellation:
    """Polygons of one size: row p of ``vert_by_poly`` lists polygon p."""
    npoly, size = vert_by_poly.shape
    ptr = np.arange(0, npoly * size + 1, size, dtype=np.int64)
    return Tessellation(ptr, vert_by_poly.reshape(-1).astype(np.int32))


def union_graph(n: int, tessellations, name: str = "staggered") -> Graph:
    """The graph whose edges are the pairs of vertices sharing a polygon of
    some tessellation (every polygon a clique of it)."""
    edges = []
    for t in tessellations:
        sizes = t.sizes()
        for size in np.unique(sizes):
            if size < 2:
                continue
            idx = np.flatnonzero(sizes == size)
            members = t.poly_vert[t.poly_ptr[idx][:, None] + np.arange(size)[None, :]].astype(np.int64)
            iu, ju = np.triu_indices(int(size), 1)
            edges.append(np.stack([members[:, iu].reshape(-1), members[:, ju].reshape(-1)], 1))
    if not edges:
        return from_edges(n, [], name)
    e = np.concatenate(edges)
    keys = np.unique(np.minimum(e[:, 0], e[:, 1]) * np.int64(n) + np.maximum(e[:, 0], e[:, 1]))
    lo, hi = np.divmod(keys, np.int64(n))
    return from_edges(n, np.stack([lo, hi], 1), name)


def stag_cycle(n: int) -> tuple[Graph, list[Tessellation]]:
    """Even cycle C_n, two tessellations by its edges: {2i, 2i+1} and
    {2i+1, 2i+2 mod n}."""
    if n < 4 or n % 2:
        raise ValueError("an even cycle of at least 4 vertices")
    v = np.arange(0, n, 2, dtype=np.int64)
    a = _uniform_tessellation(np.stack([v, v + 1], 1))
    b = _uniform_tessellation(np.stack([v + 1, (v + 2) % n], 1))
    return cycle_sorted(n), [a, b]


def stag_lattice(l1: int, l2: int | None = None) -> tuple[Graph, list[Tessellation]]:
    """Periodic l1 x l2 lattice (vertex r*l2 + c) covered by 2 x 2 squares:
    tessellation alpha holds the squares with top-left corner (2i, 2j), beta
    those with corner (2i+1, 2j+1); each square lists its corners in the
    order (r, c), (r, c+1), (r+1, c), (r+1, c+1).  The graph is the union of
    the squares as cliques (degree 6)."""
    l2 = l1 if l2 is None else l2
    if l1 < 4 or l2 < 4 or l1 % 2 or l2 % 2:
        raise ValueError("even sides of at least 4")
    tess = []
    for off in (0, 1):
        r = (np.arange(0, l1, 2, dtype=np.int64) + off)[:, None]
        c = (np.arange(0, l2, 2, dtype=np.int64) + off)[None, :]
        r1, c1 = (r + 1) % l1, (c + 1) % l2
        corners = np.stack([np.broadcast_to(x, (l1 // 2, l2 // 2)) for x in
                            (r * l2 + c, r * l2 + c1, r1 * l2 + c, r1 * l2 + c1)], axis=-1)
        tess.append(_uniform_tessellation(corners.reshape(-1, 4)))
    # every vertex is a corner of one square per tessellation: its six
    # neighbours are the other corners of its two squares
    n = l1 * l2
    nb = np.empty((n, 6), dtype=np.int64)
    for k, t in enumerate(tess):
        sq = t.poly_vert.reshape(-1, 4).astype(np.int64)
        for i in range(4):
            nb[sq[:, i], 3 * k:3 * k + 3] = sq[:, [j for j in range(4) if j != i]]
    nb.sort(axis=1)
    row_ptr = np.arange(0, 6 * n + 1, 6, dtype=np.int64)
    g = Graph(n=n, row_ptr=row_ptr, col=nb.reshape(-1).astype(np.int32), name=f"stag_lattice{l1}x{l2}")
    return g, tess


def stag_arcs(g: Graph) -> tuple[Graph, list[Tessellation]]:
    """Staggered walk on the arcs of ``g`` (staggered vertex = arc position in
    CSR order): tessellation 1 puts the arcs of each tail in one polygon (in
    row order), tessellation 2 pairs every arc with its reverse."""
    stars = [list(range(int(g.row_ptr[v]), int(g.row_ptr[v + 1]))) for v in range(g.n)
             if g.row_ptr[v + 1] > g.row_ptr[v]]
    tails = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    heads = g.col.astype(np.int64)
    key = tails * g.n + heads
    order = np.argsort(key)
    rkey = heads * g.n + tails
    rev = order[np.searchsorted(key[order], rkey)]
    a = np.arange(g.n_arcs, dtype=np.int64)
    first = a < rev
    pairs = np.stack([a[first], rev[first]], 1)
    tess = [tessellation(stars), _uniform_tessellation(pairs)]
    return union_graph(g.n_arcs, tess, name=f"{g.name}_arcs"), tess


def stag_random(n: int, n_tess: int, max_size: int, seed: int,
                weighted: bool = False) -> tuple[Graph, list[Tessellation]]:
    """``n_tess`` random tessellations of n vertices, polygon sizes uniform in
    1..max_size (the last polygon takes what is left), vertices shuffled;
    weighted: random real amplitudes scaled to unit length per polygon."""
    rng = np.random.default_rng(seed)
    tess = []
    for _ in range(n_tess):
        perm = rng.permutation(n)
        sizes = []
        left = n
        while left > 0:
            s = int(min(left, rng.integers(1, max_size + 1)))
            sizes.append(s)
            left -= s
        ptr = np.zeros(len(sizes) + 1, np.int64)
        np.cumsum(sizes, out=ptr[1:])
        t = Tessellation(ptr, perm.astype(np.int32))
        if weighted:
            amp = rng.uniform(-1.0, 1.0, n)
            for p in range(len(sizes)):
                seg = slice(ptr[p], ptr[p + 1])
                amp[seg] /= np.linalg.norm(amp[seg])
            t.amp = amp
        tess.append(t)
    return union_graph(n, tess, name=f"stag_random{n}"), tess


# ---------------------------------------------------------------------------
# Initial states (interleaved or complex numpy arrays, complex128)
# ---------------------------------------------------------------------------

def arc_index(g: Graph, v: int, w: int) -> int:
    """Position of arc (v, w) in the CSR arc order; KeyError if absent."""
    r = g.row(v)
    hit = np.flatnonzero(r == w)
    if hit.size != 1:
        raise KeyError(f"arc ({v},{w}) not in graph")
    return int(g.row_ptr[v] + hit[0])


def ket_arc(g: Graph, v: int, w: int) -> np.ndarray:
    psi = np.zeros(g.n_arcs, dtype=np.complex128)
    psi[arc_index(g, v, w)] = 1.0
    return psi


def ket_vertex(n: int, v: int) -> np.ndarray:
    psi = np.zeros(n, dtype=np.complex128)
    psi[v] = 1.0
    return psi


def uniform(size: int) -> np.ndarray:
    return np.full(size, 1.0 / math.sqrt(size), dtype=np.complex128)


def random_state(size: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(size) + 1j * rng.standard_normal(size)
    return (z / np.linalg.norm(z)).astype(np.complex128)


# ---------------------------------------------------------------------------
# Workload recipes
# ---------------------------------------------------------------------------

def cycle_hadamard_state(n: int = 64) -> tuple[Graph, np.ndarray]:
    """Cycle in direction order with (|0,0> + i|0,1>)/sqrt2 at vertex 0."""
    g = cycle(n)
    psi = np.zeros(g.n_arcs, dtype=np.complex128)
    psi[0] = 1 / math.sqrt(2)
    psi[1] = 1j / math.sqrt(2)
    return g, psi


def batch_regular_specs(count: int, seed: int, n_min: float = 1e3,
                        n_max: float = 2e5) -> list[dict]:
    """Sizes/degrees/marks of a batch of CTQW searches on random regular graphs.

    N log-uniform in [n_min, n_max], d uniform in 3..8 (N bumped by one when
    N*d is odd), gamma = 1/d, one uniformly drawn marked vertex, t_f = 2 sqrt(N).
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        nn = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        d = int(rng.integers(3, 9))
        if (nn * d) % 2:
            nn += 1
        out.append(dict(n=nn, d=d, gamma=1.0 / d, marked=int(rng.integers(nn)),
                        t_final=2.0 * math.sqrt(nn), graph_seed=int(rng.integers(2**31))))
    return out
