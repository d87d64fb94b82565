// Host runtime of the quantum-walk step engine: the C ABI declared in
// include/qwalk.h.  Plan creation validates the adjacency, builds the device
// tables (reverse arcs for the flip-flop shift, LDS tiles, structure maps,
// marked-vertex bitmap) into one host image, and fixes the Taylor order; the
// device-side calls only enqueue kernels on the caller's stream.

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "qw_internal.h"
#include "qw_plan.h"
#include "qwalk.h"

using namespace qwk;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int ok() {
  g_err.clear();
  return QW_OK;
}

int dev_fail(hipError_t e, const char *what) {
  return fail(QW_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// ---- Taylor remainder bound -------------------------------------------------
double tail_bound(double rho, int K) {
  if (rho <= 0.0) return 0.0;
  if (rho >= K + 2) return std::numeric_limits<double>::infinity();
  const double lead = std::exp((K + 1) * std::log(rho) - std::lgamma(K + 2.0));
  return lead * (K + 2) / (K + 2 - rho);
}

int taylor_order(double rho, int64_t steps, double tol) {
  for (int K = 1; K <= 64; ++K)
    if (static_cast<double>(steps) * tail_bound(rho, K) <= tol) return K;
  return -1;
}

// ---- structure recognition ---------------------------------------------------
int ctz32(uint32_t x) { return __builtin_ctz(x); }

bool is_hypercube(int64_t n, const std::vector<int64_t> &rp, const int32_t *col, int32_t *dim_out) {
  if (n < 2 || (n & (n - 1)) != 0) return false;
  const int dim = ctz32(static_cast<uint32_t>(n));
  if (dim > kMaxHypercubeDim) return false;
  for (int64_t v = 0; v < n; ++v) {
    if (rp[v + 1] - rp[v] != dim) return false;
    for (int64_t a = rp[v]; a < rp[v + 1]; ++a) {
      const uint32_t x = static_cast<uint32_t>(v) ^ static_cast<uint32_t>(col[a]);
      if (x == 0 || (x & (x - 1)) != 0) return false;
    }
  }
  *dim_out = dim;
  return true;
}

bool is_cycle(int64_t n, const std::vector<int64_t> &rp, const int32_t *col, bool ordered) {
  if (n < 3) return false;
  for (int64_t v = 0; v < n; ++v) {
    if (rp[v + 1] - rp[v] != 2) return false;
    const int64_t up = (v + 1) % n, dn = (v + n - 1) % n;
    const int64_t h0 = col[rp[v]], h1 = col[rp[v] + 1];
    const bool fwd = (h0 == up && h1 == dn), bwd = (h0 == dn && h1 == up);
    if (!(fwd || (!ordered && bwd))) return false;
  }
  return true;
}

bool is_torus(int64_t n, const std::vector<int64_t> &rp, const int32_t *col, int32_t *l1o, int32_t *l2o,
              bool ordered = false) {
  if (n < 9 || rp[1] - rp[0] != 4) return false;
  int64_t s[4];
  for (int i = 0; i < 4; ++i) s[i] = col[rp[0] + i];
  std::sort(s, s + 4);
  const int64_t l2 = s[2];
  if (s[0] != 1 || s[1] != l2 - 1 || l2 < 3 || n % l2 != 0) return false;
  const int64_t l1 = n / l2;
  if (l1 < 3 || s[3] != n - l2) return false;
  for (int64_t v = 0; v < n; ++v) {
    if (rp[v + 1] - rp[v] != 4) return false;
    const int64_t r = v / l2, c = v % l2;
    int64_t want[4] = {r * l2 + (c + 1) % l2, r * l2 + (c + l2 - 1) % l2, ((r + 1) % l1) * l2 + c,
                       ((r + l1 - 1) % l1) * l2 + c};
    int64_t got[4];
    for (int i = 0; i < 4; ++i) got[i] = col[rp[v] + i];
    if (!ordered) {  // any order; else exactly c+1, c-1, r+1, r-1
      std::sort(want, want + 4);
      std::sort(got, got + 4);
    }
    if (!std::equal(want, want + 4, got)) return false;
  }
  *l1o = static_cast<int32_t>(l1);
  *l2o = static_cast<int32_t>(l2);
  return true;
}

// slot of arc (v, w) in the slot-major structured layouts
int slot_of(int structure, int64_t v, int64_t w, int64_t n, int32_t l2) {
  if (structure == kCycle) return w == (v + 1) % n ? 0 : 1;
  if (structure == kTorus) {
    const int64_t l1 = n / l2;
    const int64_t r = v / l2, c = v % l2, rw = w / l2, cw = w % l2;
    if (rw == r) return cw == (c + 1) % l2 ? 0 : 1;
    (void)l1;
    return rw == (r + 1) % l1 ? 2 : 3;
  }
  return ctz32(static_cast<uint32_t>(v ^ w));
}

template <typename X>
void put(std::vector<unsigned char> &img, size_t off, const X *src, size_t count) {
  if (count) std::memcpy(img.data() + off, src, count * sizeof(X));
}

// Host tables of one staggered tessellation before they go into the image.
struct StagHost {
  std::vector<int32_t> vert, ptr, bptr, bvert;
  std::vector<double> amp, bamp;
  std::vector<StagChunk> chunks;
};

// Validate the tessellations (partitions of the vertices into cliques of the
// graph with unit polygon vectors) and split each into thread-path polygons
// (at most kStagThreadMax vertices; one size -> column-major table) and big
// polygons cut into chunks of kStagChunk positions.
int build_tessellations(const qw_walk_desc *w, int64_t n, const std::vector<int64_t> &rp, const int32_t *col,
                        std::vector<StagHost> &out, qw_plan *p) {
  const int32_t T = w->n_tessellations;
  if (T < 1 || T > kStagMaxTess) return fail(QW_EINVAL, "a staggered walk needs 1..%d tessellations, got %d", kStagMaxTess, T);
  if (!w->tessellations) return fail(QW_EINVAL, "null tessellation array");
  out.assign(static_cast<size_t>(T), StagHost());
  p->stag.assign(static_cast<size_t>(T), StagTess());
  std::vector<int32_t> seen(static_cast<size_t>(n), -1);
  std::vector<int64_t> owner(static_cast<size_t>(n), -1);
  int64_t poly_id = 0;
  for (int32_t k = 0; k < T; ++k) {
    const qw_tessellation &q = w->tessellations[k];
    const int64_t np = q.n_polygons;
    if (np < (n > 0 ? 1 : 0) || np > n) return fail(QW_EINVAL, "tessellation %d: %lld polygons for %lld vertices", k, (long long)np, (long long)n);
    if (n > 0 && (!q.poly_ptr || !q.poly_vert)) return fail(QW_EINVAL, "tessellation %d: null polygon arrays", k);
    if (q.form != QW_REFLECTION && q.form != QW_HAMILTONIAN) return fail(QW_EINVAL, "tessellation %d: bad form %d", k, q.form);
    if (q.form == QW_HAMILTONIAN && !std::isfinite(q.theta)) return fail(QW_EINVAL, "tessellation %d: theta not finite", k);
    if (n == 0) continue;
    const int64_t *pp = q.poly_ptr;
    if (pp[0] != 0 || pp[np] != n) return fail(QW_EINVAL, "tessellation %d: poly_ptr must run from 0 to n", k);
    for (int64_t i = 0; i < np; ++i)
      if (pp[i + 1] <= pp[i]) return fail(QW_EINVAL, "tessellation %d: polygon %lld is empty", k, (long long)i);
    for (int64_t i = 0; i < n; ++i) {
      const int32_t v = q.poly_vert[i];
      if (v < 0 || v >= n) return fail(QW_EINVAL, "tessellation %d: vertex %d out of range", k, v);
      if (seen[v] == k) return fail(QW_EINVAL, "tessellation %d: vertex %d in two polygons", k, v);
      seen[v] = k;
    }
    for (int64_t i = 0; i < np; ++i) {
      const int64_t lo = pp[i], hi = pp[i + 1], sz = hi - lo;
      // clique: every member has the other sz - 1 members among its neighbours
      for (int64_t j = lo; j < hi; ++j) owner[q.poly_vert[j]] = poly_id;
      for (int64_t j = lo; j < hi; ++j) {
        const int32_t u = q.poly_vert[j];
        int64_t cnt = 0;
        for (int64_t a = rp[u]; a < rp[u + 1]; ++a) cnt += owner[col[a]] == poly_id;
        if (cnt != sz - 1)
          return fail(QW_EGRAPH, "tessellation %d: polygon %lld is not a clique of the graph (vertex %d)", k, (long long)i, u);
      }
      ++poly_id;
      if (q.amp) {
        double ss = 0.0;
        for (int64_t j = lo; j < hi; ++j) {
          if (!std::isfinite(q.amp[j])) return fail(QW_EINVAL, "tessellation %d: amplitude %lld not finite", k, (long long)j);
          ss += q.amp[j] * q.amp[j];
        }
        if (std::fabs(ss - 1.0) > 1e-12)
          return fail(QW_EINVAL, "tessellation %d: polygon %lld has squared amplitudes summing to %.17g", k, (long long)i, ss);
      }
    }
    // split into thread-path and big polygons
    StagHost &h = out[static_cast<size_t>(k)];
    StagTess &t = p->stag[static_cast<size_t>(k)];
    int64_t n_small = 0, small_size = -1, max_small = 0, small_pos = 0;
    for (int64_t i = 0; i < np; ++i) {
      const int64_t sz = pp[i + 1] - pp[i];
      if (sz > kStagThreadMax) continue;
      ++n_small;
      small_pos += sz;
      max_small = std::max(max_small, sz);
      small_size = (small_size < 0 || small_size == sz) ? sz : 0;
    }
    t.n_small = static_cast<int32_t>(n_small);
    t.max_small = static_cast<int32_t>(max_small);
    t.small_size = static_cast<int32_t>(std::max<int64_t>(small_size, 0));
    if (n_small > 0) {
      h.vert.resize(static_cast<size_t>(small_pos));
      if (q.amp) h.amp.resize(static_cast<size_t>(small_pos));
      if (t.small_size == 0) h.ptr.reserve(static_cast<size_t>(n_small) + 1);
      int64_t ps = 0, at = 0;
      for (int64_t i = 0; i < np; ++i) {
        const int64_t lo = pp[i], sz = pp[i + 1] - lo;
        if (sz > kStagThreadMax) continue;
        if (t.small_size == 0) h.ptr.push_back(static_cast<int32_t>(at));
        for (int64_t j = 0; j < sz; ++j) {
          const size_t dst = t.small_size > 0 ? static_cast<size_t>(j * n_small + ps) : static_cast<size_t>(at + j);
          h.vert[dst] = q.poly_vert[lo + j];
          if (q.amp) h.amp[dst] = q.amp[lo + j];
        }
        at += sz;
        ++ps;
      }
      if (t.small_size == 0) h.ptr.push_back(static_cast<int32_t>(at));
    }
    h.bptr.push_back(0);
    for (int64_t i = 0; i < np; ++i) {
      const int64_t lo = pp[i], sz = pp[i + 1] - lo;
      if (sz <= kStagThreadMax) continue;
      const int32_t begin = static_cast<int32_t>(h.bvert.size());
      const int32_t first = static_cast<int32_t>(h.chunks.size());
      const int32_t count = static_cast<int32_t>((sz + kStagChunk - 1) / kStagChunk);
      for (int64_t j = 0; j < sz; ++j) {
        h.bvert.push_back(q.poly_vert[lo + j]);
        if (q.amp) h.bamp.push_back(q.amp[lo + j]);
      }
      for (int32_t c = 0; c < count; ++c) {
        StagChunk ch{};
        ch.begin = begin + c * kStagChunk;
        ch.end = static_cast<int32_t>(std::min<int64_t>(begin + sz, int64_t{begin} + int64_t{c + 1} * kStagChunk));
        ch.first = first;
        ch.count = count;
        ch.size = static_cast<int32_t>(sz);
        h.chunks.push_back(ch);
      }
      h.bptr.push_back(static_cast<int32_t>(h.bvert.size()));
    }
    t.n_big = static_cast<int32_t>(h.bptr.size()) - 1;
    t.n_chunks = static_cast<int32_t>(h.chunks.size());
    if (t.n_big == 0) h.bptr.clear();
    if (q.form == QW_HAMILTONIAN) {
      t.c0[0] = std::cos(q.theta);
      t.c0[1] = 0.0;
      t.c1[0] = 0.0;
      t.c1[1] = std::sin(q.theta);
    }
  }
  return QW_OK;
}

// Two tessellations that are the 2 x 2 squares of a periodic l1 x l2 lattice
// (vertex r*l2 + c, l1, l2 even >= 4): the first with top-left corners at even
// coordinates, the second at odd ones, uniform amplitudes.  Polygon order and
// the order of the corners inside a polygon are free.
bool stag_square_lattice(const qw_walk_desc *w, int64_t n, int32_t *l1o, int32_t *l2o) {
  if (w->n_tessellations != 2 || n < 16) return false;
  const qw_tessellation *tess = w->tessellations;
  if (tess[0].amp || tess[1].amp || tess[0].n_polygons * 4 != n || tess[1].n_polygons * 4 != n) return false;
  if (tess[0].poly_ptr[1] - tess[0].poly_ptr[0] != 4) return false;
  int64_t f[4];
  for (int i = 0; i < 4; ++i) f[i] = tess[0].poly_vert[tess[0].poly_ptr[0] + i];
  std::sort(f, f + 4);
  if (f[1] != f[0] + 1 || f[3] != f[2] + 1) return false;
  const int64_t l2 = f[2] - f[0];
  if (l2 < 4 || l2 % 2 != 0 || n % l2 != 0) return false;
  const int64_t l1 = n / l2;
  if (l1 < 4 || l1 % 2 != 0 || l1 >= (int64_t{1} << 31)) return false;
  for (int k = 0; k < 2; ++k) {
    const qw_tessellation &t = tess[k];
    for (int64_t q = 0; q < t.n_polygons; ++q) {
      const int64_t lo = t.poly_ptr[q];
      if (t.poly_ptr[q + 1] - lo != 4) return false;
      int64_t got[4], corner = -1;
      for (int i = 0; i < 4; ++i) {
        got[i] = t.poly_vert[lo + i];
        if ((got[i] / l2) % 2 == k && (got[i] % l2) % 2 == k) corner = got[i];
      }
      if (corner < 0) return false;
      const int64_t r = corner / l2, c = corner % l2, r1 = (r + 1) % l1, c1 = (c + 1) % l2;
      int64_t want[4] = {r * l2 + c, r * l2 + c1, r1 * l2 + c, r1 * l2 + c1};
      std::sort(got, got + 4);
      std::sort(want, want + 4);
      if (!std::equal(got, got + 4, want)) return false;
    }
  }
  *l1o = static_cast<int32_t>(l1);
  *l2o = static_cast<int32_t>(l2);
  return true;
}

int build_plan(const qw_csr *g, const qw_walk_desc *w, qw_plan *p) {
  if (!g || !w) return fail(QW_EINVAL, "null graph or walk descriptor");
  const int64_t n = g->n;
  if (n < 0 || n >= (int64_t{1} << 31)) return fail(QW_EINVAL, "vertex count %lld out of range", (long long)n);
  if (w->kind != QW_COINED && w->kind != QW_CTQW && w->kind != QW_STAGGERED)
    return fail(QW_EINVAL, "bad walk kind %d", w->kind);
  if (w->dtype != QW_C64 && w->dtype != QW_C128) return fail(QW_EINVAL, "bad dtype %d", w->dtype);
  if (w->layout < QW_LAYOUT_AUTO || w->layout > QW_LAYOUT_DENSE)
    return fail(QW_EINVAL, "bad layout %d", w->layout);
  if (w->layout == QW_LAYOUT_DENSE) {
    if (w->kind != QW_CTQW) return fail(QW_EUNSUPPORTED, "the dense layout is for continuous-time walks");
    if (w->columns < 0 || w->columns > kMaxDenseColumns)
      return fail(QW_EINVAL, "columns %d out of range (1..%d)", w->columns, kMaxDenseColumns);
  } else if (w->columns > 1 || w->columns < 0) {
    return fail(QW_EINVAL, "columns > 1 needs the dense layout");
  }
  if (w->kind == QW_COINED && (w->coin < QW_GROVER || w->coin > QW_SZEGEDY))
    return fail(QW_EINVAL, "bad coin %d", w->coin);
  if (w->kind == QW_COINED && w->shift != QW_FLIPFLOP && w->shift != QW_PERSISTENT)
    return fail(QW_EINVAL, "bad shift %d", w->shift);
  if (w->kind == QW_COINED && w->coin == QW_MATRIX && (!w->coin_matrix || w->coin_dim < 1))
    return fail(QW_EINVAL, "the matrix coin needs coin_matrix and coin_dim >= 1");
  if (w->kind == QW_COINED && w->coin == QW_SZEGEDY && w->shift != QW_FLIPFLOP)
    return fail(QW_EUNSUPPORTED, "the Szegedy coin takes the flip-flop shift");
  if (w->n_marked < 0 || (w->n_marked > 0 && !w->marked)) return fail(QW_EINVAL, "bad marked list");
  if (n > 0 && (!g->row_ptr)) return fail(QW_EINVAL, "null row_ptr");
  p->kind = w->kind;
  p->coin = w->kind == QW_COINED ? w->coin : QW_GROVER;
  p->shift = w->kind == QW_COINED ? w->shift : QW_FLIPFLOP;
  p->dtype = w->dtype;
  p->layout = w->layout;
  p->n = n;

  // ---- CSR validation
  std::vector<int64_t> rp(static_cast<size_t>(n) + 1, 0);
  if (n > 0) std::memcpy(rp.data(), g->row_ptr, sizeof(int64_t) * (n + 1));
  if (rp[0] != 0) return fail(QW_EGRAPH, "row_ptr[0] must be 0");
  for (int64_t v = 0; v < n; ++v)
    if (rp[v + 1] < rp[v]) return fail(QW_EGRAPH, "row_ptr decreases at row %lld", (long long)v);
  const int64_t na = rp[n];
  if (na >= (int64_t{1} << 31)) return fail(QW_EUNSUPPORTED, "%lld arcs: the engine indexes arcs with int32", (long long)na);
  if (na > 0 && !g->col) return fail(QW_EINVAL, "null col");
  p->n_arcs = na;
  const int32_t *col = g->col;
  int32_t maxd = 0;
  for (int64_t v = 0; v < n; ++v) {
    maxd = std::max<int32_t>(maxd, static_cast<int32_t>(rp[v + 1] - rp[v]));
    for (int64_t a = rp[v]; a < rp[v + 1]; ++a) {
      if (col[a] < 0 || col[a] >= n) return fail(QW_EGRAPH, "head %d out of range in row %lld", col[a], (long long)v);
      if (col[a] == v) return fail(QW_EGRAPH, "self-loop at vertex %lld", (long long)v);
    }
  }
  p->max_degree = maxd;
  // rows sorted by head (positions), duplicates, reverse arcs
  std::vector<int32_t> order(static_cast<size_t>(na));
  for (int64_t v = 0; v < n; ++v) {
    int32_t *o = order.data() + rp[v];
    const int64_t d = rp[v + 1] - rp[v];
    for (int64_t i = 0; i < d; ++i) o[i] = static_cast<int32_t>(rp[v] + i);
    std::sort(o, o + d, [&](int32_t x, int32_t y) { return col[x] < col[y]; });
    for (int64_t i = 1; i < d; ++i)
      if (col[o[i]] == col[o[i - 1]]) return fail(QW_EGRAPH, "repeated arc (%lld,%d)", (long long)v, col[o[i]]);
  }
  std::vector<int32_t> rev(static_cast<size_t>(na));
  for (int64_t v = 0; v < n; ++v) {
    for (int64_t a = rp[v]; a < rp[v + 1]; ++a) {
      const int64_t u = col[a];
      const int32_t *lo = order.data() + rp[u], *hi = order.data() + rp[u + 1];
      const int32_t *it = std::lower_bound(lo, hi, v, [&](int32_t x, int64_t key) { return col[x] < key; });
      if (it == hi || col[*it] != v)
        return fail(QW_EGRAPH, "adjacency not symmetric: arc (%lld,%lld) has no reverse", (long long)v, (long long)u);
      rev[a] = *it;
    }
  }
  std::vector<int32_t>().swap(order);

  // ---- marked set
  std::vector<uint32_t> bits(static_cast<size_t>((n + 31) / 32) + 1, 0u);
  std::vector<int32_t> mlist(static_cast<size_t>(w->n_marked));
  for (int64_t i = 0; i < w->n_marked; ++i) {
    const int32_t m = w->marked[i];
    if (m < 0 || m >= n) return fail(QW_EINVAL, "marked vertex %d out of range", m);
    if ((bits[m >> 5] >> (m & 31)) & 1u) return fail(QW_EINVAL, "marked vertex %d repeated", m);
    bits[m >> 5] |= 1u << (m & 31);
    mlist[i] = m;
  }
  p->n_marked = static_cast<int32_t>(w->n_marked);

  // ---- Szegedy transition probabilities
  if (p->kind == QW_COINED && p->coin == QW_SZEGEDY) {
    if (na > 0 && !w->transition) return fail(QW_EINVAL, "the Szegedy coin needs transition probabilities");
    p->sqrt_p.resize(static_cast<size_t>(na));
    for (int64_t v = 0; v < n; ++v) {
      double row = 0.0;
      for (int64_t a = rp[v]; a < rp[v + 1]; ++a) {
        const double x = w->transition[a];
        if (!(x >= 0.0) || !std::isfinite(x)) return fail(QW_EINVAL, "transition probability of arc %lld is not >= 0", (long long)a);
        row += x;
        p->sqrt_p[static_cast<size_t>(a)] = std::sqrt(x);
      }
      if (rp[v + 1] > rp[v] && std::fabs(row - 1.0) > 1e-12)
        return fail(QW_EINVAL, "transition probabilities of vertex %lld sum to %.17g", (long long)v, row);
    }
  }

  // ---- staggered tessellations
  std::vector<StagHost> tess;
  if (p->kind == QW_STAGGERED) {
    const int st = build_tessellations(w, n, rp, col, tess, p);
    if (st != QW_OK) return st;
  }

  // ---- walk parameters
  if (p->kind == QW_COINED && p->coin == QW_HADAMARD) {
    for (int64_t v = 0; v < n; ++v) {
      const int64_t d = rp[v + 1] - rp[v];
      const bool mk = (bits[v >> 5] >> (v & 31)) & 1u;
      if (!mk && d != 0 && d != 2)
        return fail(QW_EUNSUPPORTED, "Hadamard coin needs degree 2, vertex %lld has %lld", (long long)v, (long long)d);
    }
  }
  if (p->kind == QW_CTQW) {
    if (!(w->gamma > 0.0) || !std::isfinite(w->gamma)) return fail(QW_EINVAL, "gamma must be positive");
    if (!(w->dt > 0.0) || !std::isfinite(w->dt)) return fail(QW_EINVAL, "dt must be positive");
    p->gamma = w->gamma;
    p->dt = w->dt;
    double h = 0.0;
    for (int64_t v = 0; v < n; ++v) {
      const bool mk = (bits[v >> 5] >> (v & 31)) & 1u;
      h = std::max(h, w->gamma * static_cast<double>(rp[v + 1] - rp[v]) + (mk ? 1.0 : 0.0));
    }
    p->h_bound = h;
    if (w->taylor_order > 0) {
      if (w->taylor_order > 64) return fail(QW_EINVAL, "taylor_order above 64");
      p->K = w->taylor_order;
    } else {
      if (!(w->trunc_tol > 0.0) || w->horizon_steps < 1)
        return fail(QW_EINVAL, "automatic Taylor order needs trunc_tol > 0 and horizon_steps >= 1");
      const int K = taylor_order(w->dt * h, w->horizon_steps, w->trunc_tol);
      if (K < 0) return fail(QW_EUNSUPPORTED, "no Taylor order <= 64 meets the tolerance at rho = %g", w->dt * h);
      p->K = K;
    }
    p->trunc_bound = tail_bound(w->dt * h, p->K);
  }

  // ---- path choice: small (one workgroup), structured, or general CSR
  const bool c128 = p->dtype == QW_C128;
  int structure = kGeneral;
  const bool small_fits = p->kind == QW_COINED
                              ? coined_small_lds(c128, static_cast<int>(n), static_cast<int>(na)) <= kSmallLdsBytes
                              : ctqw_small_lds(c128, static_cast<int>(n), static_cast<int>(na)) <= kSmallLdsBytes;
  if (p->kind == QW_STAGGERED) {
    const bool fits = stag_small_lds(c128, static_cast<int>(n)) <= kSmallLdsBytes;
    int32_t a = 0, b = 0;
    if (p->layout == QW_LAYOUT_AUTO && fits && n > 0) {
      structure = kSmall;
    } else if ((p->layout == QW_LAYOUT_AUTO || p->layout == QW_LAYOUT_STRUCTURED) &&
               stag_square_lattice(w, n, &a, &b)) {
      structure = kStagLattice;
      p->dims[0] = a;
      p->dims[1] = b;
    } else {
      structure = kGeneral;
    }
  } else if (p->layout == QW_LAYOUT_DENSE) {
    structure = kDense;
    p->columns = std::max(1, w->columns);
    p->ld = static_cast<int32_t>((n + kDenseK - 1) / kDenseK * kDenseK);
    p->rows_pad = static_cast<size_t>((n + kDenseRows - 1) / kDenseRows * kDenseRows);
    p->dense_bytes = p->rows_pad * static_cast<size_t>(p->ld) * (c128 ? 8 : 4);
  } else if (p->lattice()) {
    // Fourier / matrix coins and the persistent shift: lattice kernels only,
    // rows in direction order unless the coin is Grover (order-invariant)
    if (p->layout != QW_LAYOUT_AUTO && p->layout != QW_LAYOUT_STRUCTURED)
      return fail(QW_EUNSUPPORTED, "Fourier and matrix coins and the persistent shift need the structured layout");
    int32_t a = 0, b = 0;
    const bool ordered = p->coin != QW_GROVER;
    if (n > 0 && is_cycle(n, rp, col, ordered)) {
      structure = kCycle;
      p->dims[0] = static_cast<int32_t>(n);
    } else if (n > 0 && is_torus(n, rp, col, &a, &b, ordered)) {
      structure = kTorus;
      p->dims[0] = a;
      p->dims[1] = b;
    } else {
      return fail(QW_EUNSUPPORTED, "Fourier and matrix coins and the persistent shift need a cycle (rows v+1, v-1) "
                                   "or a periodic grid (rows c+1, c-1, r+1, r-1)");
    }
    const int d = structure == kCycle ? 2 : 4;
    if (p->coin == QW_MATRIX) {
      if (w->coin_dim != d)
        return fail(QW_EUNSUPPORTED, "matrix coin of size %d on a lattice of degree %d", w->coin_dim, d);
      p->coin_mat.assign(w->coin_matrix, w->coin_matrix + 2 * d * d);
    } else if (p->coin == QW_FOURIER) {
      p->coin_mat.resize(static_cast<size_t>(2 * d * d));
      const double pi = 3.14159265358979323846;
      for (int j = 0; j < d; ++j)
        for (int k = 0; k < d; ++k) {
          const int m = (j * k) % d;  // exact phase index
          p->coin_mat[2 * (j * d + k)] = std::cos(2 * pi * m / d) / std::sqrt(static_cast<double>(d));
          p->coin_mat[2 * (j * d + k) + 1] = std::sin(2 * pi * m / d) / std::sqrt(static_cast<double>(d));
        }
    }
  } else if (p->layout == QW_LAYOUT_AUTO && small_fits && n > 0) {
    structure = kSmall;
  } else if (p->layout != QW_LAYOUT_CSR && n > 0 && !(p->kind == QW_COINED && p->coin == QW_SZEGEDY)) {
    int32_t a = 0, b = 0;
    const bool ordered = p->kind == QW_COINED && p->coin == QW_HADAMARD;
    if (!ordered && is_hypercube(n, rp, col, &a)) {
      structure = kHypercube;
      p->dims[0] = a;
    } else if (is_cycle(n, rp, col, ordered)) {
      structure = kCycle;
      p->dims[0] = static_cast<int32_t>(n);
    } else if (!ordered && is_torus(n, rp, col, &a, &b)) {
      structure = kTorus;
      p->dims[0] = a;
      p->dims[1] = b;
    } else if (p->kind == QW_CTQW && maxd >= 1 && maxd <= kMaxEllDegree && na == static_cast<int64_t>(maxd) * n) {
      structure = kEll;  // every vertex has degree maxd
      p->dims[0] = maxd;
    }
  }
  p->structure = structure;

  // ---- device tables
  const bool coined = p->kind == QW_COINED;
  p->has_rev = coined && (structure == kGeneral || structure == kSmall);
  p->has_tiles = coined && structure == kGeneral;
  p->has_perm = coined && (structure == kCycle || structure == kTorus || structure == kHypercube);
  const bool ctqw = p->kind == QW_CTQW;
  p->has_col = ctqw && (structure == kGeneral || structure == kSmall || structure == kEll || structure == kDense);

  std::vector<int32_t> tiles;
  if (p->has_tiles) {
    tiles.push_back(0);
    int64_t arcs = 0, verts = 0;
    for (int64_t v = 0; v < n; ++v) {
      const int64_t d = rp[v + 1] - rp[v];
      if (verts > 0 && (arcs + d > kTileArcs || verts == kTileMaxVerts)) {
        tiles.push_back(static_cast<int32_t>(v));
        arcs = verts = 0;
      }
      arcs += d;
      ++verts;
      if (d > kTileArcs) {
        tiles.push_back(static_cast<int32_t>(v + 1));
        arcs = verts = 0;
      }
    }
    if (tiles.back() != n) tiles.push_back(static_cast<int32_t>(n));
    p->n_tiles = static_cast<int32_t>(tiles.size()) - 1;
  }
  std::vector<int32_t> perm;
  if (p->has_perm) {
    perm.assign(static_cast<size_t>(na), -1);
    for (int64_t v = 0; v < n; ++v)
      for (int64_t a = rp[v]; a < rp[v + 1]; ++a) {
        const int j = slot_of(structure, v, col[a], n, p->dims[1]);
        const size_t slot = static_cast<size_t>(j) * n + v;
        if (j < 0 || slot >= perm.size() || perm[slot] != -1)
          return fail(QW_EINVAL, "internal: structured slot map is not a bijection at vertex %lld", (long long)v);
        perm[slot] = static_cast<int32_t>(a);
      }
    for (int32_t x : perm)
      if (x < 0) return fail(QW_EINVAL, "internal: structured slot map has a hole");
  }
  if (ctqw && structure == kGeneral) {
    const double avg = n > 0 ? static_cast<double>(na) / n : 0.0;
    p->group = avg <= 6 ? 1 : avg <= 12 ? 2 : avg <= 24 ? 4 : avg <= 48 ? 8 : avg <= 96 ? 16 : avg <= 192 ? 32 : 64;
    p->sorted_rows = 1;
    for (int64_t v = 0; v < n && p->sorted_rows; ++v)
      for (int64_t a = rp[v] + 1; a < rp[v + 1]; ++a)
        if (col[a] <= col[a - 1]) {
          p->sorted_rows = 0;
          break;
        }
  }

  // grid CTQW: stages per launch and, per strip of the blocked kernel, whether
  // a marked vertex lies in its window (halo included)
  std::vector<uint8_t> tmark;
  if (ctqw && structure == kTorus) {
    GraphView tv;
    tv.structure = structure;
    tv.dims[0] = p->dims[0];
    tv.dims[1] = p->dims[1];
    p->block_depth = torus_block_depth(c128, tv, p->K);
    if (p->block_depth > 1) {
      const StripGrid sg = torus_strips(c128, p->dims[0], p->dims[1], p->block_depth);
      const int l1 = p->dims[0], l2 = p->dims[1], S = sg.halo;
      p->strip_rows = sg.rows;
      tmark.assign(static_cast<size_t>(sg.count()), 0);
      const double cost = static_cast<double>(mlist.size()) * (sg.tiles_r + sg.tiles_c);
      if (cost > 5e7) {
        std::fill(tmark.begin(), tmark.end(), 1);  // dense marked set: every strip takes the marked path
      } else {
        std::vector<int> rows_hit, cols_hit;
        for (int32_t v : mlist) {
          const int gr = v / l2, gc = v % l2;
          rows_hit.clear();
          cols_hit.clear();
          for (int t = 0; t < sg.tiles_r; ++t) {
            const int lo = ((std::min(t * sg.rows, l1 - sg.rows) - S) % l1 + l1) % l1;
            if ((gr - lo + l1) % l1 < sg.rows + 2 * S) rows_hit.push_back(t);
          }
          for (int t = 0; t < sg.tiles_c; ++t) {
            const int lo = ((std::min(t * sg.core, l2 - sg.core) - S) % l2 + l2) % l2;
            if ((gc - lo + l2) % l2 < sg.width) cols_hit.push_back(t);
          }
          for (int a : rows_hit)
            for (int b : cols_hit) tmark[static_cast<size_t>(a) * sg.tiles_c + b] = 1;
        }
      }
      p->has_tmark = true;
    }
  }

  size_t off = 0;
  auto section = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + std::max<size_t>(bytes, 4));
    return o;
  };
  p->off_rp = section(sizeof(int32_t) * (n + 1));
  if (p->has_col) p->off_col = section(sizeof(int32_t) * na);
  if (p->has_rev) p->off_rev = section(sizeof(int32_t) * na);
  if (p->has_tiles) p->off_tiles = section(sizeof(int32_t) * tiles.size());
  if (p->has_perm) p->off_perm = section(sizeof(int32_t) * na);
  p->off_bits = section(sizeof(uint32_t) * bits.size());
  p->off_mlist = section(sizeof(int32_t) * std::max<size_t>(mlist.size(), 1));
  if (p->has_tmark) p->off_tmark = section(tmark.size());
  p->has_coin = !p->coin_mat.empty();
  if (p->has_coin) p->off_coin = section(sizeof(double) * p->coin_mat.size());
  p->has_sqrtp = p->kind == QW_COINED && p->coin == QW_SZEGEDY;
  // Degree-2 graphs of at most 64 vertices on the one-workgroup path keep
  // their amplitudes in one wavefront's registers; cycles in direction order
  // move them by lane shifts.
  if (p->kind == QW_COINED && p->structure == kSmall && !p->has_sqrtp && !p->lattice() && n >= 3 && n <= 64 &&
      na == 2 * n) {
    bool deg2 = true, ring = true;
    for (int64_t v = 0; v < n && deg2; ++v) {
      deg2 = rp[v + 1] - rp[v] == 2;
      ring = ring && deg2 && rev[2 * v] == 2 * ((v + 1) % n) + 1 && rev[2 * v + 1] == 2 * ((v + n - 1) % n);
    }
    p->two_reg = deg2 ? (ring ? 2 : 1) : 0;
  }
  if (p->has_sqrtp) p->off_sqrtp = section(sizeof(double) * p->sqrt_p.size());
  for (size_t k = 0; k < tess.size(); ++k) {
    StagHost &h = tess[k];
    StagTess &t = p->stag[k];
    if (!h.vert.empty()) t.off_vert = static_cast<int64_t>(section(sizeof(int32_t) * h.vert.size()));
    if (!h.amp.empty()) t.off_amp = static_cast<int64_t>(section(sizeof(double) * h.amp.size()));
    if (!h.ptr.empty()) t.off_ptr = static_cast<int64_t>(section(sizeof(int32_t) * h.ptr.size()));
    if (!h.bvert.empty()) {
      t.off_bptr = static_cast<int64_t>(section(sizeof(int32_t) * h.bptr.size()));
      t.off_bvert = static_cast<int64_t>(section(sizeof(int32_t) * h.bvert.size()));
      if (!h.bamp.empty()) t.off_bamp = static_cast<int64_t>(section(sizeof(double) * h.bamp.size()));
      t.off_chunk = static_cast<int64_t>(section(sizeof(StagChunk) * h.chunks.size()));
    }
  }
  if (!tess.empty()) p->off_stag = section(sizeof(StagTess) * p->stag.size());
  p->image.assign(off, 0);
  if (structure == kDense) p->off_dense = align256(off);
  std::vector<int32_t> rp32(static_cast<size_t>(n) + 1);
  for (int64_t v = 0; v <= n; ++v) rp32[v] = static_cast<int32_t>(rp[v]);
  put(p->image, p->off_rp, rp32.data(), rp32.size());
  if (p->has_col && structure == kEll) {
    // column-major: entry (j, v) = j-th smallest neighbour of v.  Sorted rows
    // let the LDS-staged batch kernel, which visits the vector in blocks of
    // increasing index, add a row's neighbours in the same order as the
    // gather kernels.
    std::vector<int32_t> colT(static_cast<size_t>(na));
    const int64_t d = p->dims[0];
    std::vector<int32_t> row(static_cast<size_t>(d));
    for (int64_t v = 0; v < n; ++v) {
      std::copy(col + rp[v], col + rp[v] + d, row.begin());
      std::sort(row.begin(), row.end());
      for (int64_t j = 0; j < d; ++j) colT[static_cast<size_t>(j) * n + v] = row[j];
    }
    put(p->image, p->off_col, colT.data(), colT.size());
  } else if (p->has_col) {
    put(p->image, p->off_col, col, static_cast<size_t>(na));
  }
  if (p->has_rev) put(p->image, p->off_rev, rev.data(), rev.size());
  if (p->has_tiles) put(p->image, p->off_tiles, tiles.data(), tiles.size());
  if (p->has_perm) put(p->image, p->off_perm, perm.data(), perm.size());
  put(p->image, p->off_bits, bits.data(), bits.size());
  put(p->image, p->off_mlist, mlist.data(), mlist.size());
  if (p->has_tmark) put(p->image, p->off_tmark, tmark.data(), tmark.size());
  if (p->has_coin) put(p->image, p->off_coin, p->coin_mat.data(), p->coin_mat.size());
  if (p->has_sqrtp) put(p->image, p->off_sqrtp, p->sqrt_p.data(), p->sqrt_p.size());
  int64_t max_chunks = 0;
  for (size_t k = 0; k < tess.size(); ++k) {
    const StagHost &h = tess[k];
    const StagTess &t = p->stag[k];
    if (t.off_vert >= 0) put(p->image, static_cast<size_t>(t.off_vert), h.vert.data(), h.vert.size());
    if (t.off_amp >= 0) put(p->image, static_cast<size_t>(t.off_amp), h.amp.data(), h.amp.size());
    if (t.off_ptr >= 0) put(p->image, static_cast<size_t>(t.off_ptr), h.ptr.data(), h.ptr.size());
    if (t.off_bptr >= 0) put(p->image, static_cast<size_t>(t.off_bptr), h.bptr.data(), h.bptr.size());
    if (t.off_bvert >= 0) put(p->image, static_cast<size_t>(t.off_bvert), h.bvert.data(), h.bvert.size());
    if (t.off_bamp >= 0) put(p->image, static_cast<size_t>(t.off_bamp), h.bamp.data(), h.bamp.size());
    if (t.off_chunk >= 0) put(p->image, static_cast<size_t>(t.off_chunk), h.chunks.data(), h.chunks.size());
    max_chunks = std::max<int64_t>(max_chunks, t.n_chunks);
  }
  if (!tess.empty()) put(p->image, p->off_stag, p->stag.data(), p->stag.size());
  std::vector<StagHost>().swap(tess);

  // ---- workspace
  const size_t es = c128 ? 16 : 8;
  const int64_t len = coined ? na : n * p->columns;
  p->state_bytes = es * static_cast<size_t>(len);
  GraphView probe;
  probe.n = static_cast<int32_t>(n);
  probe.structure = structure;
  probe.group = p->group;
  probe.columns = p->columns;
  const size_t partials = static_cast<size_t>(std::max(readout_partials(probe), ctqw_stage_partials(probe))) + 1;
  size_t w_off = 0;
  auto wsec = [&](size_t bytes) {
    const size_t o = w_off;
    w_off = align256(w_off + std::max<size_t>(bytes, 8));
    return o;
  };
  if (p->kind == QW_STAGGERED) {
    // in place on the caller's state: only the big-polygon partial sums; the
    // square-lattice kernel writes every step to the other of two buffers
    if (structure == kStagLattice) p->off_w1 = wsec(p->state_bytes);
    if (max_chunks > 0) p->off_stagpart = wsec(2 * sizeof(double) * static_cast<size_t>(max_chunks));
  } else {
    wsec(p->state_bytes);                  // buffer 0 at offset 0
    p->off_w1 = wsec(p->state_bytes);      // buffer 1
  }
  if (p->block_depth > 1) p->off_w2 = wsec(p->state_bytes);  // buffer 2: the other psi
  p->off_pscratch = wsec(sizeof(double) * static_cast<size_t>(n) * p->columns);
  p->off_partials = wsec(sizeof(double) * partials);
  if (structure == kDense) {
    GraphView dv;
    dv.n = static_cast<int32_t>(n);
    dv.columns = p->columns;
    const int sp = dense_splits(dv);
    if (sp > 1) p->off_dpartial = wsec(sizeof(double) * static_cast<size_t>(sp) * n * 2 * p->columns);
  }
  p->work_bytes = w_off;
  return ok();
}

int check_bound(const qw_plan *p) {
  if (!p) return fail(QW_EINVAL, "null plan");
  if (!p->d_graph) return fail(QW_ESTATE, "plan not uploaded (call qw_plan_upload first)");
  return QW_OK;
}

Readout make_readout(const qw_plan *p, unsigned char *work, double *d_p, double *d_norm, double *d_pm) {
  Readout r;
  r.p = d_p;
  r.norm = d_norm;
  r.pmarked = d_pm;
  r.pscratch = reinterpret_cast<double *>(work + p->off_pscratch);
  r.partials = reinterpret_cast<double *>(work + p->off_partials);
  return r;
}

#define QW_TRY(expr, what)                   \
  do {                                       \
    hipError_t e_ = (expr);                  \
    if (e_ != hipSuccess) return dev_fail(e_, what); \
  } while (0)

int readout_only(const qw_plan *p, const void *psi, const Readout &ro, hipStream_t s) {
  const bool c128 = p->dtype == QW_C128;
  const GraphView &g = p->view;
  if (!ro.any()) return QW_OK;
  if (p->kind == QW_COINED) {
    QW_TRY(coined_prob_csr(c128, g, psi, ro, s), "coined probability kernel");
  } else {
    QW_TRY(vertex_prob(c128, g, psi, ro, s), "vertex probability kernel");
  }
  QW_TRY(finish_readout(g, readout_partials(g), ro, s), "readout reduction kernel");
  return QW_OK;
}

int evolve_coined(const qw_plan *p, void *psi, unsigned char *work, int64_t steps, const Readout &ro,
                  hipStream_t s) {
  const bool c128 = p->dtype == QW_C128;
  const GraphView &g = p->view;
  const int had = p->coin == QW_HADAMARD;
  void *w0 = work, *w1 = work + p->off_w1;
  if (p->structure == kSmall) {
    QW_TRY(coined_small(c128, g, psi, had, steps, ro, s), "coined small-graph kernel");
    return QW_OK;
  }
  if (steps == 0) return readout_only(p, psi, ro, s);
  if (p->structure == kGeneral) {
    void *cur = psi, *oth = w0;
    for (int64_t i = 0; i < steps; ++i) {
      QW_TRY(coined_tile_step(c128, g, cur, oth, had, s), "coined step kernel");
      std::swap(cur, oth);
    }
    if (cur != psi) QW_TRY(copy_state(c128, p->n_arcs, cur, psi, s), "state copy kernel");
    return readout_only(p, psi, ro, s);
  }
  QW_TRY(coined_perm_in(c128, g, psi, w0, s), "layout permutation kernel");
  void *cur = w0, *oth = w1;
  for (int64_t i = 0; i < steps; ++i) {
    QW_TRY(coined_struct_step(c128, g, cur, oth, had, s), "coined structured step kernel");
    std::swap(cur, oth);
  }
  QW_TRY(coined_perm_out(c128, g, cur, psi, ro, s), "layout permutation kernel");
  if (ro.any()) QW_TRY(finish_readout(g, readout_partials(g), ro, s), "readout reduction kernel");
  return QW_OK;
}

int evolve_staggered(const qw_plan *p, void *psi, unsigned char *work, int64_t steps, const Readout &ro,
                     hipStream_t s) {
  const bool c128 = p->dtype == QW_C128;
  const GraphView &g = p->view;
  if (p->structure == kSmall) {
    QW_TRY(stag_small(c128, g, psi, steps, ro, s), "staggered small-graph kernel");
    return QW_OK;
  }
  if (p->structure == kStagLattice) {
    void *cur = psi, *oth = work + p->off_w1;
    for (int64_t i = 0; i < steps;) {
      const int k = steps - i >= 2 ? 2 : 1;  // two steps per launch, an odd last one alone
      QW_TRY(stag_lattice_step(c128, g, p->stag[0], p->stag[1], k, cur, oth, s), "staggered lattice kernel");
      std::swap(cur, oth);
      i += k;
    }
    if (cur != psi) QW_TRY(copy_state(c128, p->n, cur, psi, s), "state copy kernel");
    return readout_only(p, psi, ro, s);
  }
  auto *partials = reinterpret_cast<double *>(work + p->off_stagpart);
  for (int64_t i = 0; i < steps && p->n > 0; ++i)
    for (size_t k = 0; k < p->stag.size(); ++k)
      QW_TRY(stag_tess(c128, g, p->stag[k], psi, k == 0 && p->n_marked > 0, partials, s),
             "staggered tessellation kernels");
  return readout_only(p, psi, ro, s);
}

int evolve_ctqw(const qw_plan *p, void *psi, unsigned char *work, int64_t steps, const Readout &ro,
                hipStream_t s) {
  const bool c128 = p->dtype == QW_C128;
  const GraphView &g = p->view;
  const int K = p->K;
  std::vector<double> alpha(K), beta(K);
  for (int k = 1; k <= K; ++k) {
    beta[k - 1] = p->dt / k;
    alpha[k - 1] = p->gamma * p->dt / k;
  }
  if (p->structure == kSmall) {
    QW_TRY(ctqw_small(c128, g, psi, alpha.data(), beta.data(), K, steps, ro, s), "CTQW small-graph kernel");
    return QW_OK;
  }
  if (steps == 0) return readout_only(p, psi, ro, s);
  void *w0 = work, *w1 = work + p->off_w1;
  if (p->block_depth > 1) {
    // temporal blocking: K/S launches per step, each S stages in registers;
    // psi alternates between the caller's buffer and buffer 2, y between 0 and 1
    std::vector<double> a64(64, 0.0), b64(64, 0.0);
    for (int k = 0; k < K; ++k) {
      a64[k] = alpha[k];
      b64[k] = beta[k];
    }
    const int S = p->block_depth, per = K / S;
    void *pc = psi, *pa = work + p->off_w2;
    void *ybuf[2] = {w0, w1};
    for (int64_t i = 0; i < steps; ++i) {
      for (int j = 0; j < per; ++j) {
        const void *yin = (j == 0) ? pc : ybuf[(j - 1) & 1];
        void *out = (j == per - 1) ? pa : ybuf[j & 1];
        QW_TRY(torus_block_stages(c128, g, S, pc, yin, out, K - j * S, a64.data(), b64.data(), s),
               "grid CTQW blocked stages kernel");
      }
      std::swap(pc, pa);
    }
    if (pc != psi) QW_TRY(copy_state(c128, p->n, pc, psi, s), "state copy kernel");
    return readout_only(p, psi, ro, s);
  }
  if (p->structure == kDense) {
    GraphView gd = g;
    gd.dense_partial = p->off_dpartial ? reinterpret_cast<double *>(work + p->off_dpartial) : nullptr;
    for (int64_t i = 0; i < steps; ++i) {
      const void *yin = psi;
      for (int k = K; k >= 1; --k) {
        void *yout = (k == 1) ? (K == 1 ? w0 : psi) : (((K - k) & 1) ? w1 : w0);
        QW_TRY(dense_stage(c128, gd, yin, psi, yout, beta[k - 1], s), "dense Horner stage kernel");
        yin = yout;
      }
      if (K == 1) QW_TRY(copy_state(c128, p->n * p->columns, w0, psi, s), "state copy kernel");
    }
    return readout_only(p, psi, ro, s);
  }
  bool fused_done = false;
  for (int64_t i = 0; i < steps; ++i) {
    const void *yin = psi;
    for (int k = K; k >= 1; --k) {
      void *yout = (k == 1) ? (K == 1 ? w0 : psi) : (((K - k) & 1) ? w1 : w0);
      const bool fuse = ro.any() && k == 1 && K >= 2 && i == steps - 1;
      StageCoef c{alpha[k - 1], beta[k - 1]};
      QW_TRY(ctqw_stage(c128, g, yin, psi, yout, c, fuse ? &ro : nullptr, s), "CTQW Horner stage kernel");
      fused_done |= fuse;
      yin = yout;
    }
    if (K == 1) QW_TRY(copy_state(c128, p->n, w0, psi, s), "state copy kernel");
  }
  if (!ro.any()) return QW_OK;
  if (!fused_done) return readout_only(p, psi, ro, s);
  QW_TRY(finish_readout(g, ctqw_stage_partials(g), ro, s), "readout reduction kernel");
  return QW_OK;
}

}  // namespace

namespace qwk {

int set_error(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int clear_error() { return ok(); }

int plan_readout(const qw_plan *p, const void *psi, unsigned char *work, double *d_p, double *d_norm,
                 double *d_pmarked, hipStream_t s) {
  const Readout ro = make_readout(p, work, d_p, d_norm, d_pmarked);
  return readout_only(p, psi, ro, s);
}

int plan_struct_out(const qw_plan *p, const void *internal, void *psi, unsigned char *work, double *d_p,
                    double *d_norm, double *d_pmarked, hipStream_t s) {
  const Readout ro = make_readout(p, work, d_p, d_norm, d_pmarked);
  QW_TRY(coined_perm_out(p->dtype == QW_C128, p->view, internal, psi, ro, s), "layout permutation kernel");
  if (ro.any()) QW_TRY(finish_readout(p->view, readout_partials(p->view), ro, s), "readout reduction kernel");
  return QW_OK;
}

}  // namespace qwk

// =============================== C ABI =======================================

extern "C" {

int qw_plan_create(const qw_csr *graph, const qw_walk_desc *walk, qw_plan **out) {
  if (!out) return fail(QW_EINVAL, "null output pointer");
  *out = nullptr;
  qw_plan *p = nullptr;
  try {
    p = new qw_plan();
    const int st = build_plan(graph, walk, p);
    if (st != QW_OK) {
      delete p;
      return st;
    }
  } catch (const std::bad_alloc &) {
    delete p;
    return fail(QW_ENOMEM, "host allocation failed");
  } catch (...) {
    delete p;
    return fail(QW_EINVAL, "unexpected host exception");
  }
  *out = p;
  return ok();
}

int qw_plan_destroy(qw_plan *plan) {
  delete plan;
  return ok();
}

int qw_plan_get_info(const qw_plan *p, qw_plan_info *info) {
  if (!p || !info) return fail(QW_EINVAL, "null argument");
  std::memset(info, 0, sizeof *info);
  info->n = p->n;
  info->n_arcs = p->n_arcs;
  info->state_len = p->kind == QW_COINED ? p->n_arcs : p->n;
  info->kind = p->kind;
  info->coin = p->coin;
  info->dtype = p->dtype;
  info->structure = p->structure;
  info->dims[0] = p->dims[0];
  info->dims[1] = p->dims[1];
  info->max_degree = p->max_degree;
  info->taylor_order = p->K;
  info->dt = p->dt;
  info->h_norm_bound = p->h_bound;
  info->trunc_bound = p->trunc_bound;
  info->graph_bytes = p->image.size();
  info->state_bytes = p->state_bytes;
  info->work_bytes = p->work_bytes;
  info->columns = p->columns;
  info->block_depth = p->block_depth;
  info->state_len = p->kind == QW_COINED ? p->n_arcs : p->n * p->columns;
  if (p->structure == kDense) info->graph_bytes = p->off_dense + p->dense_bytes;
  return ok();
}

int qw_plan_upload(qw_plan *p, void *d_graph, size_t graph_bytes, void *stream) {
  if (!p || !d_graph) return fail(QW_EINVAL, "null plan or graph buffer");
  const size_t need = p->structure == kDense ? p->off_dense + p->dense_bytes : p->image.size();
  if (graph_bytes < need)
    return fail(QW_ENOMEM, "graph buffer of %zu bytes, plan needs %zu", graph_bytes, need);
  if (reinterpret_cast<uintptr_t>(d_graph) % 256 != 0) return fail(QW_EINVAL, "graph buffer not 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  release_streamed(p);  // a plain upload ends an out-of-core binding
  QW_TRY(hipMemcpyAsync(d_graph, p->image.data(), p->image.size(), hipMemcpyHostToDevice, s), "graph upload");
  auto *base = static_cast<unsigned char *>(d_graph);
  p->d_graph = base;
  GraphView &g = p->view;
  g = GraphView();
  g.n = static_cast<int32_t>(p->n);
  g.n_arcs = static_cast<int32_t>(p->n_arcs);
  g.structure = p->structure;
  g.dims[0] = p->dims[0];
  g.dims[1] = p->dims[1];
  g.n_marked = p->n_marked;
  g.n_tiles = p->n_tiles;
  g.group = p->group;
  g.sorted_rows = p->sorted_rows;
  g.rp = reinterpret_cast<const int32_t *>(base + p->off_rp);
  if (p->has_col) g.col = reinterpret_cast<const int32_t *>(base + p->off_col);
  if (p->structure == kEll) g.ell_d = p->dims[0];
  if (p->has_rev) g.rev = reinterpret_cast<const int32_t *>(base + p->off_rev);
  if (p->has_tiles) g.tiles = reinterpret_cast<const int32_t *>(base + p->off_tiles);
  if (p->has_perm) g.perm = reinterpret_cast<const int32_t *>(base + p->off_perm);
  g.markbits = reinterpret_cast<const uint32_t *>(base + p->off_bits);
  g.marklist = reinterpret_cast<const int32_t *>(base + p->off_mlist);
  if (p->has_tmark) g.tmark = reinterpret_cast<const uint8_t *>(base + p->off_tmark);
  g.strip_rows = p->strip_rows;
  g.two_reg = p->two_reg;
  g.persistent = p->shift == QW_PERSISTENT;
  if (p->has_coin) g.coin = reinterpret_cast<const double *>(base + p->off_coin);
  if (p->has_sqrtp) g.sqrtp = reinterpret_cast<const double *>(base + p->off_sqrtp);
  g.columns = p->columns;
  g.base = base;
  if (!p->stag.empty()) {
    g.stag = reinterpret_cast<const StagTess *>(base + p->off_stag);
    g.n_tess = static_cast<int32_t>(p->stag.size());
  }
  if (p->structure == kDense) {
    g.ld = p->ld;
    g.dense = base + p->off_dense;
    QW_TRY(dense_fill(p->dtype == QW_C128, g, p->gamma, p->rows_pad, s), "dense H fill kernels");
  }
  return ok();
}

int qw_evolve(const qw_plan *p, void *d_psi, void *d_work, size_t work_bytes, int64_t steps, double *d_p,
              double *d_norm, double *d_pmarked, void *stream) {
  int st = check_bound(p);
  if (st != QW_OK) return st;
  if (steps < 0) return fail(QW_EINVAL, "negative step count");
  if (!d_psi && p->state_bytes) return fail(QW_EINVAL, "null state");
  if (!d_work) return fail(QW_EINVAL, "null workspace");
  if (work_bytes < p->work_bytes) return fail(QW_ENOMEM, "workspace of %zu bytes, plan needs %zu", work_bytes, p->work_bytes);
  auto *work = static_cast<unsigned char *>(d_work);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (p->streamed) {
    st = evolve_streamed(p, d_psi, work, steps, d_p, d_norm, d_pmarked, s);
    return st == QW_OK ? ok() : st;
  }
  const Readout ro = make_readout(p, work, d_p, d_norm, d_pmarked);
  st = p->kind == QW_COINED     ? evolve_coined(p, d_psi, work, steps, ro, s)
       : p->kind == QW_STAGGERED ? evolve_staggered(p, d_psi, work, steps, ro, s)
                                 : evolve_ctqw(p, d_psi, work, steps, ro, s);
  return st == QW_OK ? ok() : st;
}

int qw_probabilities(const qw_plan *p, const void *d_psi, double *d_p, double *d_norm, double *d_pmarked,
                     void *d_work, size_t work_bytes, void *stream) {
  int st = check_bound(p);
  if (st != QW_OK) return st;
  if (!d_psi && p->state_bytes) return fail(QW_EINVAL, "null state");
  if (!d_work) return fail(QW_EINVAL, "null workspace");
  if (work_bytes < p->work_bytes) return fail(QW_ENOMEM, "workspace of %zu bytes, plan needs %zu", work_bytes, p->work_bytes);
  auto *work = static_cast<unsigned char *>(d_work);
  const Readout ro = make_readout(p, work, d_p, d_norm, d_pmarked);
  st = readout_only(p, d_psi, ro, static_cast<hipStream_t>(stream));
  return st == QW_OK ? ok() : st;
}

int qw_copy_to_host(void *h_dst, const void *d_src, size_t bytes, void *stream) {
  if (bytes == 0) return ok();
  if (!h_dst || !d_src) return fail(QW_EINVAL, "null buffer");
  if ((reinterpret_cast<uintptr_t>(h_dst) | reinterpret_cast<uintptr_t>(d_src)) & 15)
    return fail(QW_EINVAL, "buffers must be 16-byte aligned");
  hipPointerAttribute_t attr{};
  if (hipPointerGetAttributes(&attr, d_src) != hipSuccess || attr.type != hipMemoryTypeDevice) {
    (void)hipGetLastError();
    return fail(QW_EINVAL, "source is not device memory");
  }
  void *base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(reinterpret_cast<hipDeviceptr_t *>(&base), &size, const_cast<void *>(d_src)) !=
          hipSuccess ||
      static_cast<const char *>(d_src) + bytes > static_cast<const char *>(base) + size) {
    (void)hipGetLastError();
    return fail(QW_EINVAL, "source allocation holds fewer than %zu bytes", bytes);
  }
  void *dp = nullptr;
  if (hipHostGetDevicePointer(&dp, h_dst, 0) != hipSuccess || !dp || (reinterpret_cast<uintptr_t>(dp) & 15)) {
    (void)hipGetLastError();
    return fail(QW_EINVAL, "destination is not pinned host memory the device can write (hipHostMalloc)");
  }
  const hipError_t e = copy_link(dp, d_src, bytes, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(QW_EDEVICE, "copy launch: %s", hipGetErrorString(e));
  return ok();
}

size_t qw_small_many_desc_bytes(int32_t count) {
  return count > 0 ? sizeof(SmallWalk) * static_cast<size_t>(count) : 0;
}

int qw_small_many(const qw_plan *const *plans, void *const *d_psi, const int64_t *steps, int32_t count,
                  void *d_desc, size_t desc_bytes, void *stream) {
  if (count < 0) return fail(QW_EINVAL, "negative walk count");
  if (count == 0) return ok();
  if (!plans || !d_psi || !steps) return fail(QW_EINVAL, "null walk arrays");
  if (!d_desc) return fail(QW_EINVAL, "null descriptor buffer");
  if (desc_bytes < qw_small_many_desc_bytes(count))
    return fail(QW_ENOMEM, "descriptor buffer of %zu bytes, %d walks need %zu", desc_bytes, count,
                qw_small_many_desc_bytes(count));
  std::vector<SmallWalk> walks;
  try {
    walks.resize(static_cast<size_t>(count));
  } catch (const std::bad_alloc &) {
    return fail(QW_ENOMEM, "host allocation");
  }
  const int dtype = plans[0] ? plans[0]->dtype : QW_C64;
  size_t lds = 0;
  int threads = 64;
  for (int32_t i = 0; i < count; ++i) {
    const qw_plan *p = plans[i];
    int st = check_bound(p);
    if (st != QW_OK) return st;
    if (p->dtype != dtype) return fail(QW_EINVAL, "walk %d: all walks must share one dtype", i);
    if (p->structure != kSmall) return fail(QW_EINVAL, "walk %d: plan is not on the one-workgroup path", i);
    if (steps[i] < 0) return fail(QW_EINVAL, "walk %d: negative step count", i);
    if (!d_psi[i] && p->state_bytes) return fail(QW_EINVAL, "walk %d: null state", i);
    const bool c128 = p->dtype == QW_C128, coined = p->kind == QW_COINED;
    const int n = static_cast<int>(p->n), na = static_cast<int>(p->n_arcs);
    lds = std::max(lds, coined                      ? coined_small_lds(c128, n, na)
                        : p->kind == QW_STAGGERED ? stag_small_lds(c128, n)
                                                  : ctqw_small_lds(c128, n, na));
    const int want = coined ? na : n;
    while (threads < 1024 && threads < want) threads *= 2;
    SmallWalk &w = walks[static_cast<size_t>(i)];
    w.g = p->view;
    w.psi = d_psi[i];
    w.coined = coined;
    w.staggered = p->kind == QW_STAGGERED;
    w.hadamard = p->coin == QW_HADAMARD;
    w.K = p->K;
    w.steps = steps[i];
    for (int k = 1; k <= p->K && p->kind == QW_CTQW; ++k) {
      w.beta[k - 1] = p->dt / k;
      w.alpha[k - 1] = p->gamma * p->dt / k;
    }
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t bytes = qw_small_many_desc_bytes(count);
  hipError_t e = hipMemcpyAsync(d_desc, walks.data(), bytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return fail(QW_EDEVICE, "descriptor copy: %s", hipGetErrorString(e));
  e = small_many(dtype == QW_C128, static_cast<const SmallWalk *>(d_desc), count, lds, threads, s);
  if (e != hipSuccess) return fail(QW_EDEVICE, "many-small-walks kernel: %s", hipGetErrorString(e));
  return ok();
}

int qw_taylor_order(double rho, int64_t steps, double tol, int32_t *K) {
  if (!K) return fail(QW_EINVAL, "null output");
  if (!(rho >= 0.0) || !std::isfinite(rho) || steps < 1 || !(tol > 0.0))
    return fail(QW_EINVAL, "rho >= 0, steps >= 1 and tol > 0 required");
  const int k = taylor_order(rho, steps, tol);
  if (k < 0) return fail(QW_EUNSUPPORTED, "no order <= 64 meets the tolerance");
  *K = k;
  return ok();
}

int qw_taylor_plan(double h_bound, double t_total, double rho_max, double tol, int32_t *K, double *dt,
                   int64_t *steps) {
  if (!K || !dt || !steps) return fail(QW_EINVAL, "null output");
  if (!(h_bound >= 0.0) || !(t_total > 0.0) || !(rho_max > 0.0) || !(tol > 0.0) || !std::isfinite(t_total))
    return fail(QW_EINVAL, "h_bound >= 0, t_total > 0, rho_max > 0 and tol > 0 required");
  int64_t n = h_bound > 0.0 ? static_cast<int64_t>(std::ceil(t_total * h_bound / rho_max)) : 1;
  if (n < 1) n = 1;
  const double d = t_total / static_cast<double>(n);
  const int k = taylor_order(d * h_bound, n, tol);
  if (k < 0) return fail(QW_EUNSUPPORTED, "no order <= 64 meets the tolerance");
  *K = k;
  *dt = d;
  *steps = n;
  return ok();
}

double qw_taylor_tail_bound(double rho, int32_t K) { return tail_bound(rho, K); }

const char *qw_last_error(void) { return g_err.c_str(); }

const char *qw_version(void) { return "qwalk-mi355x 0.1 (gfx950)"; }

}  // extern "C"
