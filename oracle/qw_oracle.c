/*
 * FP64 CPU oracle for the quantum-walk time-evolution step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the engine's product path may link,
 * load or call this file; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header or table with the HIP path.
 *
 * Every routine is the plain definition from the paper (Hiperwalk, arXiv
 * 2406.08186) written out in complex double precision, one output element
 * at a time, with a fixed summation order per element, so the result does
 * not depend on the number of OpenMP threads.
 *
 *   Coined walk (Sec. 3.2):  U = S C with the flip-flop shift S|v,w> = |w,v>
 *     and the Grover coin  C|v,w> = sum_{v' in N(v)} (2/d(v) - delta_{w,v'}) |v,v'>.
 *     The arc basis is CSR order: row v lists the heads of the arcs with tail v.
 *     Extensions used by the benchmark workloads (not in the paper): the
 *     Hadamard coin (1/sqrt2)[[1,1],[1,-1]] on a degree-2 vertex's two arcs in
 *     row order, and the coin -I at marked vertices for spatial search.
 *   Coined probability (Sec. 3.2):  p_v = sum over arcs with tail v of |psi_a|^2.
 *   CTQW (Sec. 3.1, Hamiltonian H = -gamma A - sum_{v in M} |v><v|):
 *     psi(t+dt) = T_K(-i H dt) psi(t), the Taylor series of exp(-iH dt) cut
 *     after the term k = K, evaluated in POWER form
 *       term_0 = psi,  term_k = (-i dt / k) H term_{k-1},  psi' = sum_k term_k.
 *   CTQW probability (Sec. 3.1):  p_v = |psi_v|^2.
 *   Szegedy and staggered walks (named as future work in Sec. 5): see their
 *     routines below.
 *
 * Arrays of complex numbers are interleaved (re, im) doubles.
 *
 * Fault injection (orc_set_fault) exists only so the tests can plant a
 * plausible mistake in the oracle and show that a pin catches it.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double _Complex cplx;

enum { ORC_GROVER = 0, ORC_HADAMARD = 1 };

/* Planted-mistake codes for the mutation tests (0 = none). */
enum {
  ORC_FAULT_NONE = 0,
  ORC_FAULT_COIN_DELTA_SIGN = 1,   /* +delta instead of -delta in the Grover coin */
  ORC_FAULT_NO_SHIFT = 2,          /* psi'_a = phi_a (shift dropped)              */
  ORC_FAULT_HEAD_PROB = 3,         /* coined p summed over heads, not tails       */
  ORC_FAULT_CTQW_NO_MARK = 4,      /* marked term of H dropped                    */
  ORC_FAULT_CTQW_PLUS_I = 5,       /* exp(+iHt) instead of exp(-iHt)              */
  ORC_FAULT_TAYLOR_SHORT = 6,      /* last Taylor term dropped                    */
  ORC_FAULT_HADAMARD_SWAP = 7,     /* Hadamard rows swapped                       */
  ORC_FAULT_MARK_PLUS = 8,         /* marked coin +I instead of -I                */
  ORC_FAULT_GAMMA_ON_MARK = 9,     /* marked term scaled by gamma                 */
  ORC_FAULT_STAG_ONE_PROJ = 10,    /* staggered: P - I instead of 2P - I          */
  ORC_FAULT_STAG_REVERSED = 11,    /* staggered: tessellations in reverse order   */
  ORC_FAULT_STAG_MARK_AFTER = 12,  /* staggered: marked phase after the product   */
  ORC_FAULT_STAG_THETA_SIGN = 13   /* staggered: exp(-i theta H) for exp(i theta H)*/
};

static int g_fault = ORC_FAULT_NONE;
static int g_threads = 0;

void orc_set_fault(int code) { g_fault = code; }
void orc_set_threads(int n) { g_threads = n; }

int orc_max_threads(void) {
#ifdef _OPENMP
  return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
  return 1;
#endif
}

/*
 * Reverse-arc index.  For arc a = (v, w) at position a of the CSR arrays,
 * rev[a] is the position of arc (w, v).  Found by scanning row w.
 * Returns 0, or -1 if some arc has no reverse (adjacency not symmetric),
 * or -2 if some arc is a self-loop.
 */
int orc_reverse_arcs(int64_t n, const int64_t *row_ptr, const int32_t *col, int64_t *rev) {
  int status = 0;
#pragma omp parallel for schedule(dynamic, 256) num_threads(orc_max_threads())
  for (int64_t v = 0; v < n; ++v) {
    for (int64_t a = row_ptr[v]; a < row_ptr[v + 1]; ++a) {
      int64_t w = col[a];
      int64_t found = -1;
      if (w == v) {
#pragma omp atomic write
        status = -2;
      }
      for (int64_t b = row_ptr[w]; b < row_ptr[w + 1]; ++b) {
        if (col[b] == v) { found = b; break; }
      }
      if (found < 0) {
#pragma omp atomic write
        status = -1;
      }
      rev[a] = found;
    }
  }
  return status;
}

/*
 * Coin on vertex v's block of arcs [lo, hi): phi = C_v psi, written as the
 * matrix-vector product with the coin's matrix elements.
 */
static void coin_block(int coin, int marked, int64_t lo, int64_t hi,
                       const cplx *psi, cplx *phi) {
  int64_t d = hi - lo;
  if (d == 0) return;
  if (marked) {
    double sign = (g_fault == ORC_FAULT_MARK_PLUS) ? 1.0 : -1.0;
    for (int64_t a = lo; a < hi; ++a) phi[a] = sign * psi[a];
    return;
  }
  if (coin == ORC_HADAMARD) {
    const double h = 1.0 / sqrt(2.0);
    cplx x0 = psi[lo], x1 = psi[lo + 1];
    if (g_fault == ORC_FAULT_HADAMARD_SWAP) {
      phi[lo] = h * (x0 - x1);
      phi[lo + 1] = h * (x0 + x1);
    } else {
      phi[lo] = h * (x0 + x1);
      phi[lo + 1] = h * (x0 - x1);
    }
    return;
  }
  /* Grover: <v,v'| C |v,w> = 2/d - delta_{w,v'} */
  double delta_sign = (g_fault == ORC_FAULT_COIN_DELTA_SIGN) ? 1.0 : -1.0;
  for (int64_t out = lo; out < hi; ++out) {
    cplx acc = 0.0;
    for (int64_t in = lo; in < hi; ++in) {
      double c = 2.0 / (double)d + (in == out ? delta_sign : 0.0);
      acc += c * psi[in];
    }
    phi[out] = acc;
  }
}

/*
 * Coined evolution: psi <- (S C)^steps psi, in place.
 * coin: 0 Grover, 1 Hadamard (requires degree 2 at every unmarked vertex
 * with arcs).  marked: byte per vertex (may be NULL).  rev from
 * orc_reverse_arcs.  Returns 0, or -3 if the Hadamard coin meets a vertex
 * whose degree is not 2, -4 on allocation failure.
 */
int orc_coined_evolve(int64_t n, const int64_t *row_ptr, const int32_t *col,
                      const int64_t *rev, int coin, const uint8_t *marked,
                      double *psi_io, int64_t steps) {
  (void)col;
  int64_t n_arcs = row_ptr[n];
  if (coin == ORC_HADAMARD) {
    for (int64_t v = 0; v < n; ++v) {
      int64_t d = row_ptr[v + 1] - row_ptr[v];
      int mk = marked ? marked[v] : 0;
      if (!mk && d != 0 && d != 2) return -3;
    }
  }
  cplx *psi = (cplx *)psi_io;
  cplx *phi = (cplx *)malloc(sizeof(cplx) * (size_t)(n_arcs > 0 ? n_arcs : 1));
  if (!phi) return -4;
  for (int64_t s = 0; s < steps; ++s) {
#pragma omp parallel for schedule(dynamic, 1024) num_threads(orc_max_threads())
    for (int64_t v = 0; v < n; ++v)
      coin_block(coin, marked ? marked[v] : 0, row_ptr[v], row_ptr[v + 1], psi, phi);
    /* flip-flop: S|w,v> = |v,w>, so the amplitude at (v,w) comes from (w,v) */
#pragma omp parallel for schedule(static) num_threads(orc_max_threads())
    for (int64_t a = 0; a < n_arcs; ++a)
      psi[a] = (g_fault == ORC_FAULT_NO_SHIFT) ? phi[a] : phi[rev[a]];
  }
  free(phi);
  return 0;
}

/*
 * Coined evolution with any coin and shift (Sec. 3.2): psi <- (S C)^steps psi,
 * in place.  coin_mat: NULL for the Grover coin, else an interleaved complex
 * d x d matrix (row-major) applied to every unmarked vertex of degree
 * coin_dim, in the order of its row (the coin basis); marked vertices take
 * -I.  dest[a]: the arc that receives phi_a -- the reverse arc for the
 * flip-flop shift, the arc straight ahead for the persistent shift; it must
 * be a permutation of the arcs.  Returns 0, -3 if a vertex with arcs, not
 * marked, has a degree other than coin_dim, -4 on allocation failure.
 */
int orc_coined_evolve_general(int64_t n, const int64_t *row_ptr, const int64_t *dest,
                              const double *coin_mat, int64_t coin_dim, const uint8_t *marked,
                              double *psi_io, int64_t steps) {
  int64_t n_arcs = row_ptr[n];
  if (coin_mat) {
    for (int64_t v = 0; v < n; ++v) {
      int64_t d = row_ptr[v + 1] - row_ptr[v];
      int mk = marked ? marked[v] : 0;
      if (!mk && d != 0 && d != coin_dim) return -3;
    }
  }
  const cplx *cm = (const cplx *)coin_mat;
  cplx *psi = (cplx *)psi_io;
  cplx *phi = (cplx *)malloc(sizeof(cplx) * (size_t)(n_arcs > 0 ? n_arcs : 1));
  if (!phi) return -4;
  for (int64_t s = 0; s < steps; ++s) {
#pragma omp parallel for schedule(dynamic, 1024) num_threads(orc_max_threads())
    for (int64_t v = 0; v < n; ++v) {
      int64_t lo = row_ptr[v], hi = row_ptr[v + 1];
      int mk = marked ? marked[v] : 0;
      if (!cm || mk) {
        coin_block(ORC_GROVER, mk, lo, hi, psi, phi);
        continue;
      }
      /* phi_j = sum_k C[j][k] psi_k over the vertex's arcs in row order */
      for (int64_t j = 0; j < hi - lo; ++j) {
        cplx acc = 0.0;
        for (int64_t k = 0; k < hi - lo; ++k) acc += cm[j * coin_dim + k] * psi[lo + k];
        phi[lo + j] = acc;
      }
    }
#pragma omp parallel for schedule(static) num_threads(orc_max_threads())
    for (int64_t a = 0; a < n_arcs; ++a) psi[dest[a]] = phi[a];
  }
  free(phi);
  return 0;
}

/*
 * Szegedy walk (the paper's frontend future work, Sec. 5), on the arc basis:
 * psi <- (S (2 Pi - I))^steps psi with Pi = sum_x |alpha_x><alpha_x|,
 * alpha_x = sum_y sqrt(P_xy) |x,y>, and S the flip-flop swap.  The
 * reflection is written as its matrix elements, <a| 2 Pi - I |b> =
 * 2 sqrt(P_a) sqrt(P_b) - delta_ab for arcs a, b of the same tail.  sqrt_p:
 * double per arc (CSR order).  Marked vertices take -I.
 */
int orc_szegedy_evolve(int64_t n, const int64_t *row_ptr, const int64_t *rev, const double *sqrt_p,
                       const uint8_t *marked, double *psi_io, int64_t steps) {
  int64_t n_arcs = row_ptr[n];
  cplx *psi = (cplx *)psi_io;
  cplx *phi = (cplx *)malloc(sizeof(cplx) * (size_t)(n_arcs > 0 ? n_arcs : 1));
  if (!phi) return -4;
  for (int64_t s = 0; s < steps; ++s) {
#pragma omp parallel for schedule(dynamic, 1024) num_threads(orc_max_threads())
    for (int64_t v = 0; v < n; ++v) {
      int64_t lo = row_ptr[v], hi = row_ptr[v + 1];
      if (marked && marked[v]) {
        for (int64_t a = lo; a < hi; ++a) phi[a] = -psi[a];
        continue;
      }
      for (int64_t out = lo; out < hi; ++out) {
        cplx acc = 0.0;
        for (int64_t in = lo; in < hi; ++in)
          acc += (2.0 * sqrt_p[out] * sqrt_p[in] - (in == out ? 1.0 : 0.0)) * psi[in];
        phi[out] = acc;
      }
    }
#pragma omp parallel for schedule(static) num_threads(orc_max_threads())
    for (int64_t a = 0; a < n_arcs; ++a) psi[a] = phi[rev[a]];
  }
  free(phi);
  return 0;
}

/*
 * Staggered walk (the paper's frontend future work, Sec. 5; the model of
 * Portugal, Santos, Fernandes and Goncalves, 2016), on the vertex basis.  A
 * tessellation k is a partition of the vertices into polygons alpha, each
 * with a real unit vector |alpha> = sum_{v in alpha} a_v |v> (uniform:
 * a_v = 1/sqrt|alpha|), and P_k = sum_alpha |alpha><alpha| is the projector
 * onto their span.  With H_k = 2 P_k - I (a reflection, H_k^2 = I) one step is
 *   psi <- U_T ... U_2 U_1 R_M psi,
 * R_M = I - 2 sum_{m in M} |m><m| (the marked vertices' phase flip, applied
 * first), and U_k = H_k (form 0, the reflection) or U_k = exp(i theta_k H_k)
 * = cos(theta_k) I + i sin(theta_k) H_k (form 1, the staggered model with
 * Hamiltonians).  The projection is formed in a vector of its own, then
 * psi <- c0 psi + c1 (2 P psi - psi) with (c0, c1) = (0, 1) or
 * (cos theta, i sin theta).
 *
 * Tessellation t's polygons are n_poly[t] ranges of its vertex list: its
 * pointer array (n_poly[t] + 1 entries) is the t-th block of poly_ptr (blocks
 * back to back), its vertex list (n entries) the t-th block of n entries of
 * vert, its amplitudes the t-th block of amp when has_amp[t] (else uniform).
 * Returns 0, or -4 on allocation failure.
 */
int orc_staggered_evolve(int64_t n, int32_t n_tess, const int64_t *n_poly, const int64_t *poly_ptr,
                         const int32_t *vert, const double *amp, const uint8_t *has_amp, const int32_t *form,
                         const double *theta, const uint8_t *marked, double *psi_io, int64_t steps) {
  cplx *psi = (cplx *)psi_io;
  cplx *proj = (cplx *)malloc(sizeof(cplx) * (size_t)(n > 0 ? n : 1));
  int64_t *ptr_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_tess > 0 ? n_tess : 1));
  if (!proj || !ptr_off) {
    free(proj);
    free(ptr_off);
    return -4;
  }
  int64_t off = 0;
  for (int32_t t = 0; t < n_tess; ++t) {
    ptr_off[t] = off;
    off += n_poly[t] + 1;
  }
  for (int64_t s = 0; s < steps; ++s) {
    if (marked && g_fault != ORC_FAULT_STAG_MARK_AFTER)
      for (int64_t v = 0; v < n; ++v)
        if (marked[v]) psi[v] = -psi[v];
    for (int32_t k = 0; k < n_tess; ++k) {
      int32_t t = (g_fault == ORC_FAULT_STAG_REVERSED) ? n_tess - 1 - k : k;
      const int64_t *pp = poly_ptr + ptr_off[t];
      const int32_t *vv = vert + (size_t)t * (size_t)n;
      const double *aa = has_amp[t] ? amp + (size_t)t * (size_t)n : NULL;
      /* proj = P_t psi, polygon by polygon: <alpha|psi> |alpha> */
#pragma omp parallel for schedule(dynamic, 1024) num_threads(orc_max_threads())
      for (int64_t p = 0; p < n_poly[t]; ++p) {
        int64_t lo = pp[p], hi = pp[p + 1];
        double uni = 1.0 / sqrt((double)(hi - lo));
        cplx inner = 0.0;
        for (int64_t i = lo; i < hi; ++i) inner += (aa ? aa[i] : uni) * psi[vv[i]];
        for (int64_t i = lo; i < hi; ++i) proj[vv[i]] = (aa ? aa[i] : uni) * inner;
      }
      cplx c0 = 0.0, c1 = 1.0;
      if (form[t] == 1) {
        double th = (g_fault == ORC_FAULT_STAG_THETA_SIGN) ? -theta[t] : theta[t];
        c0 = cos(th);
        c1 = I * sin(th);
      }
      double two = (g_fault == ORC_FAULT_STAG_ONE_PROJ) ? 1.0 : 2.0;
#pragma omp parallel for schedule(static) num_threads(orc_max_threads())
      for (int64_t v = 0; v < n; ++v) psi[v] = c0 * psi[v] + c1 * (two * proj[v] - psi[v]);
    }
    if (marked && g_fault == ORC_FAULT_STAG_MARK_AFTER)
      for (int64_t v = 0; v < n; ++v)
        if (marked[v]) psi[v] = -psi[v];
  }
  free(proj);
  free(ptr_off);
  return 0;
}

/* Coined vertex probability p_v = sum over arcs with tail v of |psi_a|^2. */
void orc_coined_prob(int64_t n, const int64_t *row_ptr, const int32_t *col,
                     const double *psi_in, double *p) {
  const cplx *psi = (const cplx *)psi_in;
  if (g_fault == ORC_FAULT_HEAD_PROB) {
    for (int64_t v = 0; v < n; ++v) p[v] = 0.0;
    for (int64_t v = 0; v < n; ++v)
      for (int64_t a = row_ptr[v]; a < row_ptr[v + 1]; ++a) {
        double re = creal(psi[a]), im = cimag(psi[a]);
        p[col[a]] += re * re + im * im;
      }
    return;
  }
#pragma omp parallel for schedule(static) num_threads(orc_max_threads())
  for (int64_t v = 0; v < n; ++v) {
    double acc = 0.0;
    for (int64_t a = row_ptr[v]; a < row_ptr[v + 1]; ++a) {
      double re = creal(psi[a]), im = cimag(psi[a]);
      acc += re * re + im * im;
    }
    p[v] = acc;
  }
}

/* (H x)_v = -gamma sum_{u in N(v)} x_u - [v in M] x_v */
static void apply_h(int64_t n, const int64_t *row_ptr, const int32_t *col, double gamma,
                    const uint8_t *marked, const cplx *x, cplx *y) {
#pragma omp parallel for schedule(static) num_threads(orc_max_threads())
  for (int64_t v = 0; v < n; ++v) {
    cplx acc = 0.0;
    for (int64_t a = row_ptr[v]; a < row_ptr[v + 1]; ++a) acc += x[col[a]];
    cplx hv = -gamma * acc;
    if (marked && marked[v] && g_fault != ORC_FAULT_CTQW_NO_MARK)
      hv -= (g_fault == ORC_FAULT_GAMMA_ON_MARK ? gamma : 1.0) * x[v];
    y[v] = hv;
  }
}

/*
 * CTQW evolution with the order-K Taylor propagator in power form,
 * psi <- T_K(-i H dt)^steps psi, in place.  Returns 0, or -4 on allocation
 * failure.
 */
int orc_ctqw_evolve(int64_t n, const int64_t *row_ptr, const int32_t *col, double gamma,
                    const uint8_t *marked, double dt, int32_t K, double *psi_io,
                    int64_t steps) {
  cplx *psi = (cplx *)psi_io;
  size_t bytes = sizeof(cplx) * (size_t)(n > 0 ? n : 1);
  cplx *term = (cplx *)malloc(bytes);
  cplx *next = (cplx *)malloc(bytes);
  cplx *acc = (cplx *)malloc(bytes);
  if (!term || !next || !acc) { free(term); free(next); free(acc); return -4; }
  const cplx minus_i = (g_fault == ORC_FAULT_CTQW_PLUS_I) ? I : -I;
  int32_t kmax = (g_fault == ORC_FAULT_TAYLOR_SHORT) ? K - 1 : K;
  for (int64_t s = 0; s < steps; ++s) {
    memcpy(term, psi, bytes);
    memcpy(acc, psi, bytes);
    for (int32_t k = 1; k <= kmax; ++k) {
      apply_h(n, row_ptr, col, gamma, marked, term, next);
      cplx coef = minus_i * (dt / (double)k);
#pragma omp parallel for schedule(static) num_threads(orc_max_threads())
      for (int64_t v = 0; v < n; ++v) {
        term[v] = coef * next[v];
        acc[v] += term[v];
      }
    }
    memcpy(psi, acc, bytes);
  }
  free(term); free(next); free(acc);
  return 0;
}

/* CTQW vertex probability p_v = |psi_v|^2. */
void orc_vertex_prob(int64_t n, const double *psi_in, double *p) {
  const cplx *psi = (const cplx *)psi_in;
#pragma omp parallel for schedule(static) num_threads(orc_max_threads())
  for (int64_t v = 0; v < n; ++v) {
    double re = creal(psi[v]), im = cimag(psi[v]);
    p[v] = re * re + im * im;
  }
}
