// HIP kernels of the quantum-walk step engine (gfx950 / CDNA4, wave64).
//
// State storage is T = float2 (complex64) or double2 (complex128).  Every
// kernel loads T, does its arithmetic in FP64 registers and rounds once when
// it stores, so a complex64 walk differs from the FP64 one only by one
// rounding of each stored amplitude per kernel (no systematically biased
// coefficient such as a rounded 2/d).  The one exception is the blocked grid
// sweep, which computes complex64 in FP32 with every coefficient split into
// two floats (still no rounded coefficient).  All reductions are FP64 with a
// fixed order, so results are bitwise reproducible.
//
// Coined step (Hiperwalk Sec. 3.2): psi' = S C psi with the flip-flop shift
// S|v,w> = |w,v> and, per vertex block, the Grover coin
// (C psi)_{v,v'} = (2/d) sum_w psi_{v,w} - psi_{v,v'}, the Hadamard coin on a
// degree-2 block, or -I at marked vertices.
// CTQW Horner stage (Sec. 3.1 Hamiltonian): y_out = psi + (-i dt/k) H y_in with
// (H y)_v = -gamma sum_{u ~ v} y_u - [v in M] y_v, i.e.
// y_out = psi + i (alpha sum_u y_u + beta [v in M] y_v), alpha = gamma dt/k,
// beta = dt/k.

#include <algorithm>
#include <type_traits>

#include "qw_internal.h"

namespace qwk {
namespace {

constexpr double kInvSqrt2 = 0.70710678118654752440;

typedef int i32x4 __attribute__((ext_vector_type(4)));  // 16-byte vector for the non-temporal builtin

inline int blocks_for(int64_t n, int per) { return static_cast<int>((n + per - 1) / per); }

// ---- storage <-> FP64 -------------------------------------------------------
__device__ __forceinline__ double2 ld(const float2 *p, int64_t i) {
  float2 v = p[i];
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ double2 ld(const double2 *p, int64_t i) { return p[i]; }
__device__ __forceinline__ double2 cvt(float2 v) { return make_double2(v.x, v.y); }
__device__ __forceinline__ double2 cvt(double2 v) { return v; }
__device__ __forceinline__ void st(float2 *p, int64_t i, double2 v) {
  p[i] = make_float2(static_cast<float>(v.x), static_cast<float>(v.y));
}
__device__ __forceinline__ void st(double2 *p, int64_t i, double2 v) { p[i] = v; }
template <typename T> __device__ __forceinline__ T pack(double2 v);
template <> __device__ __forceinline__ float2 pack<float2>(double2 v) {
  return make_float2(static_cast<float>(v.x), static_cast<float>(v.y));
}
template <> __device__ __forceinline__ double2 pack<double2>(double2 v) { return v; }

__device__ __forceinline__ double2 add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 scale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double abs2(double2 a) { return a.x * a.x + a.y * a.y; }

__device__ __forceinline__ bool marked(const uint32_t *bits, int v) {
  return (bits[v >> 5] >> (v & 31)) & 1u;
}

// Global-address-space views of pointers that kernels read from tables in
// memory (the batch's slot table).  The compiler cannot tell where such a
// pointer points and would address through flat instructions, which count
// against the LDS wait counter too; through these views it emits global
// loads and stores.
#define QW_GLOBAL __attribute__((address_space(1)))
template <typename T> using gptr = const QW_GLOBAL T *;
template <typename T> using gmut = QW_GLOBAL T *;
template <typename T> __device__ __forceinline__ gptr<T> as_global(const T *p) { return (gptr<T>)p; }
template <typename T> __device__ __forceinline__ gmut<T> as_global_mut(T *p) { return (gmut<T>)p; }
// Complex elements through such views are moved as the compiler's own
// two-element vectors (one 8- or 16-byte access each).
typedef float qw_f2v __attribute__((ext_vector_type(2)));
typedef double qw_d2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 gld(gptr<float2> p, int64_t i) {
  const qw_f2v v = reinterpret_cast<const QW_GLOBAL qw_f2v *>(p)[i];
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ double2 gld(gptr<double2> p, int64_t i) {
  const qw_d2v v = reinterpret_cast<const QW_GLOBAL qw_d2v *>(p)[i];
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void gst(gmut<float2> p, int64_t i, float2 v) {
  reinterpret_cast<QW_GLOBAL qw_f2v *>(p)[i] = qw_f2v{v.x, v.y};
}
__device__ __forceinline__ void gst(gmut<double2> p, int64_t i, double2 v) {
  reinterpret_cast<QW_GLOBAL qw_d2v *>(p)[i] = qw_d2v{v.x, v.y};
}

// The value x holds in lane `src` of the wavefront (a cross-lane permute).
__device__ __forceinline__ float2 lane_pull(float2 x, int src) {
  return make_float2(__shfl(x.x, src, 64), __shfl(x.y, src, 64));
}
__device__ __forceinline__ double2 lane_pull(double2 x, int src) {
  return make_double2(__shfl(x.x, src, 64), __shfl(x.y, src, 64));
}

constexpr int kFromLower = 0x138;  // DPP wave_shr:1, lane i receives lane i-1 (lane 0 receives 0)
constexpr int kFromUpper = 0x130;  // DPP wave_shl:1, lane i receives lane i+1 (lane 63 receives 0)

constexpr int kRotFromUpper = 0x134;  // DPP wave_rol:1, lane i receives lane (i+1) mod 64
constexpr int kRotFromLower = 0x13C;  // DPP wave_ror:1, lane i receives lane (i-1) mod 64

// Lane v of the first wavefront receives lane (v + 1) mod n of x (UP) or lane
// (v - 1) mod n (down), for n <= 64.  FULL (n = 64): one DPP rotation of the
// wavefront.  Otherwise a one-lane DPP shift, and the lane that wraps reads
// its source lane directly.
template <bool UP, bool FULL> __device__ __forceinline__ int ring_pull(int x, int n) {
  if (FULL) return __builtin_amdgcn_update_dpp(0, x, UP ? kRotFromUpper : kRotFromLower, 0xf, 0xf, false);
  const int shifted = __builtin_amdgcn_update_dpp(0, x, UP ? kFromUpper : kFromLower, 0xf, 0xf, true);
  const int wrapped = __builtin_amdgcn_readlane(x, UP ? 0 : n - 1);
  return static_cast<int>(threadIdx.x) == (UP ? n - 1 : 0) ? wrapped : shifted;
}
template <bool UP, bool FULL> __device__ __forceinline__ float ring_pull(float x, int n) {
  return __int_as_float(ring_pull<UP, FULL>(__float_as_int(x), n));
}
template <bool UP, bool FULL> __device__ __forceinline__ double ring_pull(double x, int n) {
  const long long b = __double_as_longlong(x);
  const int lo = ring_pull<UP, FULL>(static_cast<int>(b), n);
  const int hi = ring_pull<UP, FULL>(static_cast<int>(b >> 32), n);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
template <bool UP, bool FULL> __device__ __forceinline__ float2 ring_pull(float2 v, int n) {
  return make_float2(ring_pull<UP, FULL>(v.x, n), ring_pull<UP, FULL>(v.y, n));
}
template <bool UP, bool FULL> __device__ __forceinline__ double2 ring_pull(double2 v, int n) {
  return make_double2(ring_pull<UP, FULL>(v.x, n), ring_pull<UP, FULL>(v.y, n));
}

// Workgroup b is dispatched to XCD b % 8 (round-robin over the 8 XCDs).  This
// remap gives XCD x one contiguous range of logical blocks, so neighbouring
// rows of a stencil are read through the same L2.  It is a bijection on
// [0, nb) for any nb.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

// Grover on one block given its sum s: phi = 2 s/d - psi.  The mean is the
// correctly rounded FP64 quotient; doubling it is exact.
__device__ __forceinline__ double2 grover_mean(double2 s, int d) {
  double inv = 1.0 / static_cast<double>(d);
  return make_double2(s.x * inv, s.y * inv);
}

// ---- deterministic FP64 block reduction ---------------------------------------
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Sum of x over the block (blockDim.x a multiple of 64, <= 1024); result valid
// in every thread.  Uses `red` (>= 16 doubles of LDS).
__device__ double block_sum(double x, double *red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  x = wave_sum(x);
  __syncthreads();
  if (lane == 0) red[wave] = x;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += red[i];
  return t;
}

// ---- readout tail: partial norms ---------------------------------------------
__global__ __launch_bounds__(256) void k_finish(const double *partials, int count, const double *p,
                                                const int32_t *marklist, int n_marked, int columns,
                                                double *norm, double *pmarked) {
  __shared__ double red[16];
  double acc = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) acc += partials[i];
  double tot = block_sum(acc, red);
  double pm = 0.0;
  for (int i = threadIdx.x; i < n_marked; i += blockDim.x)
    for (int b = 0; b < columns; ++b) pm += p[static_cast<int64_t>(marklist[i]) * columns + b];
  double ptot = block_sum(pm, red);
  if (threadIdx.x == 0) {
    if (norm) *norm = tot;
    if (pmarked) *pmarked = ptot;
  }
}

// ---- coined: whole walk in one workgroup (its LDS, or one wavefront's registers)
// Steps of a graph whose vertices all have degree 2, at most 64 of them, held
// in the first wavefront's registers: lane v has the amplitudes x0, x1 of arcs
// 2v, 2v + 1, whose reverse arcs are r0, r1; mk marks vertex v.  HAD picks the
// Hadamard coin (else Grover), MARKS says some vertex is marked, RING that the
// graph is a cycle in direction order (1: one-lane shifts instead of
// permutes; 2: 64 vertices, wavefront rotations).  The loop body has no
// branch; arithmetic and rounding are those of the LDS loops of
// coined_small_walk.
template <typename T, bool HAD, bool MARKS, int RING>
__device__ void two_reg_steps(T &x0, T &x1, int r0, int r1, bool mk, int n, int64_t steps) {
  for (int64_t s = 0; s < steps; ++s) {
    const double2 y0 = cvt(x0), y1 = cvt(x1);
    double2 f0, f1;
    if (HAD) {
      f0 = scale(add(y0, y1), kInvSqrt2);
      f1 = scale(sub(y0, y1), kInvSqrt2);
    } else {
      const double2 m = grover_mean(add(add(make_double2(0.0, 0.0), y0), y1), 2);
      f0 = sub(add(m, m), y0);
      f1 = sub(add(m, m), y1);
    }
    if (MARKS) {
      f0 = mk ? scale(y0, -1.0) : f0;
      f1 = mk ? scale(y1, -1.0) : f1;
    }
    const T q0 = pack<T>(f0), q1 = pack<T>(f1);
    if (RING) {
      x0 = ring_pull<true, RING == 2>(q1, n);
      x1 = ring_pull<false, RING == 2>(q0, n);
    } else {
      const T u0 = lane_pull(q0, r0 >> 1), w0 = lane_pull(q1, r0 >> 1);
      const T u1 = lane_pull(q0, r1 >> 1), w1 = lane_pull(q1, r1 >> 1);
      x0 = (r0 & 1) ? w0 : u0;
      x1 = (r1 & 1) ? w1 : u1;
    }
  }
}

template <typename T>
__device__ void coined_small_walk(const GraphView &g, T *psi, int hadamard, int64_t steps, const Readout &ro,
                                  unsigned char *smem, double *red) {
  const int n = g.n, na = g.n_arcs;
  if (g.two_reg) {
    // Every vertex has degree 2 and there are at most 64 (cycles, unions of
    // cycles; the plan checked): lane v of the first wavefront keeps vertex
    // v's two amplitudes (arcs 2v, 2v + 1) in registers from the first load
    // to the last store and takes the shifted ones from the lanes that own
    // the reverse arcs, so the walk needs no LDS and no barrier.  Arithmetic,
    // rounding and the readout's summation order are those of the LDS path.
    if (threadIdx.x < 64) {
      const bool live = static_cast<int>(threadIdx.x) < n;
      const int v = live ? static_cast<int>(threadIdx.x) : 0;
      T x0 = psi[2 * v], x1 = psi[2 * v + 1];
      // new amplitude of arc 2v + k = coin output at arc rev[2v + k], held by
      // lane rev >> 1 in its slot rev & 1
      const int r0 = g.rev[2 * v], r1 = g.rev[2 * v + 1];
      const bool mk = marked(g.markbits, v);
      const int rk = g.two_reg == 2 ? (n == 64 ? 2 : 1) : 0;
      switch ((hadamard ? 6 : 0) + (g.n_marked > 0 ? 3 : 0) + rk) {
        case 0: two_reg_steps<T, false, false, 0>(x0, x1, r0, r1, mk, n, steps); break;
        case 1: two_reg_steps<T, false, false, 1>(x0, x1, r0, r1, mk, n, steps); break;
        case 2: two_reg_steps<T, false, false, 2>(x0, x1, r0, r1, mk, n, steps); break;
        case 3: two_reg_steps<T, false, true, 0>(x0, x1, r0, r1, mk, n, steps); break;
        case 4: two_reg_steps<T, false, true, 1>(x0, x1, r0, r1, mk, n, steps); break;
        case 5: two_reg_steps<T, false, true, 2>(x0, x1, r0, r1, mk, n, steps); break;
        case 6: two_reg_steps<T, true, false, 0>(x0, x1, r0, r1, mk, n, steps); break;
        case 7: two_reg_steps<T, true, false, 1>(x0, x1, r0, r1, mk, n, steps); break;
        case 8: two_reg_steps<T, true, false, 2>(x0, x1, r0, r1, mk, n, steps); break;
        case 9: two_reg_steps<T, true, true, 0>(x0, x1, r0, r1, mk, n, steps); break;
        case 10: two_reg_steps<T, true, true, 1>(x0, x1, r0, r1, mk, n, steps); break;
        default: two_reg_steps<T, true, true, 2>(x0, x1, r0, r1, mk, n, steps); break;
      }
      if (live) {
        psi[2 * v] = x0;
        psi[2 * v + 1] = x1;
      }
      // p_v, the norm and p_M in the summation order of the LDS readout below
      // (one vertex per thread there; the other wavefronts add exact zeros)
      const double pv = live ? (0.0 + abs2(cvt(x0))) + abs2(cvt(x1)) : 0.0;
      if (ro.p && live) ro.p[v] = pv;
      const double tot = wave_sum(0.0 + pv);
      const double ptot = wave_sum(live && mk ? 0.0 + pv : 0.0);
      if (threadIdx.x == 0) {
        if (ro.norm) *ro.norm = tot;
        if (ro.pmarked) *ro.pmarked = ptot;
      }
    }
    return;  // two_reg is the same in every thread
  }
  T *a = reinterpret_cast<T *>(smem);
  T *b = a + na;
  int32_t *srp = reinterpret_cast<int32_t *>(b + na);
  int32_t *srev = srp + n + 1;
  uint32_t *smark = reinterpret_cast<uint32_t *>(srev + na);  // the marked bitmap, read every step
  const int n_words = (n + 31) / 32;
  {
    // each thread's first element of every table: the loads go out together
    const int t = threadIdx.x;
    T v0{};
    int32_t r0 = 0, p0 = 0;
    uint32_t m0 = 0;
    if (t < na) {
      v0 = psi[t];
      r0 = g.rev[t];
    }
    if (t <= n) p0 = g.rp[t];
    if (t < n_words) m0 = g.markbits[t];
    if (t < na) {
      a[t] = v0;
      srev[t] = r0;
    }
    if (t <= n) srp[t] = p0;
    if (t < n_words) smark[t] = m0;
  }
  for (int i = threadIdx.x + blockDim.x; i < na; i += blockDim.x) {
    a[i] = psi[i];
    srev[i] = g.rev[i];
  }
  for (int i = threadIdx.x + blockDim.x; i <= n; i += blockDim.x) srp[i] = g.rp[i];
  for (int i = threadIdx.x + blockDim.x; i < n_words; i += blockDim.x) smark[i] = g.markbits[i];
  __syncthreads();
  // One step per pass: each vertex's coin output goes straight to the
  // reverse arcs' slots of the other buffer (the flip-flop shift), so a step
  // is one LDS pass and one barrier.  When every vertex has a thread of its
  // own and degree <= 4 (cycles, grids), the thread keeps its vertex's arc
  // range, reverse-arc slots and mark in registers across the steps.
  constexpr int kRegDeg = 4;
  int own_ok = n <= static_cast<int>(blockDim.x) ? 1 : 0;
  int rlo = 0, rd = 0, rmk = 0, rrev[kRegDeg] = {0, 0, 0, 0};
  if (own_ok && threadIdx.x < n) {
    rlo = srp[threadIdx.x];
    rd = srp[threadIdx.x + 1] - rlo;
    rmk = marked(smark, threadIdx.x) ? 1 : 0;
#pragma unroll
    for (int k = 0; k < kRegDeg; ++k) rrev[k] = k < rd ? srev[rlo + k] : 0;
  }
  own_ok = __syncthreads_and(own_ok && (threadIdx.x >= n || rd <= kRegDeg) && !g.sqrtp);
  for (int64_t s = 0; s < steps && own_ok; ++s) {
    if (threadIdx.x < n && rd > 0) {
      double2 x[kRegDeg];
#pragma unroll
      for (int k = 0; k < kRegDeg; ++k) x[k] = k < rd ? cvt(a[rlo + k]) : make_double2(0.0, 0.0);
      if (rmk) {
#pragma unroll
        for (int k = 0; k < kRegDeg; ++k)
          if (k < rd) b[rrev[k]] = pack<T>(scale(x[k], -1.0));
      } else if (hadamard) {
        b[rrev[0]] = pack<T>(scale(add(x[0], x[1]), kInvSqrt2));
        b[rrev[1]] = pack<T>(scale(sub(x[0], x[1]), kInvSqrt2));
      } else {
        double2 sum = make_double2(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < kRegDeg; ++k)
          if (k < rd) sum = add(sum, x[k]);
        const double2 m = grover_mean(sum, rd);
#pragma unroll
        for (int k = 0; k < kRegDeg; ++k)
          if (k < rd) b[rrev[k]] = pack<T>(sub(add(m, m), x[k]));
      }
    }
    __syncthreads();
    T *t = a;
    a = b;
    b = t;
  }
  for (int64_t s = 0; s < steps && !own_ok; ++s) {
    for (int v = threadIdx.x; v < n; v += blockDim.x) {
      const int lo = srp[v], hi = srp[v + 1], d = hi - lo;
      if (d == 0) continue;
      if (marked(smark, v)) {
        for (int i = lo; i < hi; ++i) b[srev[i]] = pack<T>(scale(cvt(a[i]), -1.0));
      } else if (hadamard) {
        double2 x0 = cvt(a[lo]), x1 = cvt(a[lo + 1]);
        b[srev[lo]] = pack<T>(scale(add(x0, x1), kInvSqrt2));
        b[srev[lo + 1]] = pack<T>(scale(sub(x0, x1), kInvSqrt2));
      } else if (g.sqrtp) {
        const double *wt = g.sqrtp + g.rp[v];  // Szegedy: 2 w_a <w, x> - x_a
        double2 sum = make_double2(0.0, 0.0);
        for (int i = lo; i < hi; ++i) sum = add(sum, scale(cvt(a[i]), wt[i - lo]));
        for (int i = lo; i < hi; ++i) b[srev[i]] = pack<T>(sub(scale(sum, 2.0 * wt[i - lo]), cvt(a[i])));
      } else {
        double2 sum = make_double2(0.0, 0.0);
        for (int i = lo; i < hi; ++i) sum = add(sum, cvt(a[i]));
        double2 m = grover_mean(sum, d);
        for (int i = lo; i < hi; ++i) b[srev[i]] = pack<T>(sub(add(m, m), cvt(a[i])));
      }
    }
    __syncthreads();
    T *t = a;
    a = b;
    b = t;
  }
  for (int i = threadIdx.x; i < na; i += blockDim.x) psi[i] = a[i];
  if (ro.p || ro.norm || ro.pmarked) {
    // p_v from the LDS copy; p_M adds the marked vertices' p_v as they pass
    double acc = 0.0, pm = 0.0;
    for (int v = threadIdx.x; v < n; v += blockDim.x) {
      double pv = 0.0;
      for (int i = srp[v]; i < srp[v + 1]; ++i) pv += abs2(cvt(a[i]));
      if (ro.p) ro.p[v] = pv;
      acc += pv;
      if (marked(smark, v)) pm += pv;
    }
    double tot = block_sum(acc, red);
    double ptot = block_sum(pm, red);
    if (threadIdx.x == 0) {
      if (ro.norm) *ro.norm = tot;
      if (ro.pmarked) *ro.pmarked = ptot;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_coined_small(GraphView g, T *psi, int hadamard,
                                                       int64_t steps, Readout ro) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[16];
  coined_small_walk<T>(g, psi, hadamard, steps, ro, smem, red);
}

// ---- coined: general CSR, one LDS tile of whole vertex blocks per workgroup --
// Tile t covers vertices [tiles[t], tiles[t+1]); its arcs fit kTileArcs unless
// the tile is a single vertex of larger degree.  Loads are coalesced in arc
// order; the flip-flop shift scatters phi_a to out[rev[a]].
template <typename T>
__global__ __launch_bounds__(kTileThreads) void k_coined_tile(GraphView g, const T *__restrict__ in,
                                                              T *__restrict__ out, int hadamard) {
  __shared__ T s[kTileArcs];
  __shared__ double red[16];
  const int t = blockIdx.x;
  const int vb = g.tiles[t], ve = g.tiles[t + 1];
  const int ab = g.rp[vb], ae = g.rp[ve];
  const int na = ae - ab;
  if (na <= kTileArcs) {
    for (int i = threadIdx.x; i < na; i += blockDim.x) s[i] = in[ab + i];
    __syncthreads();
    for (int v = vb + threadIdx.x; v < ve; v += blockDim.x) {
      const int lo = g.rp[v] - ab, hi = g.rp[v + 1] - ab, d = hi - lo;
      if (d == 0) continue;
      if (marked(g.markbits, v)) {
        for (int i = lo; i < hi; ++i) s[i] = pack<T>(scale(cvt(s[i]), -1.0));
      } else if (hadamard) {
        double2 x0 = cvt(s[lo]), x1 = cvt(s[lo + 1]);
        s[lo] = pack<T>(scale(add(x0, x1), kInvSqrt2));
        s[lo + 1] = pack<T>(scale(sub(x0, x1), kInvSqrt2));
      } else if (g.sqrtp) {
        const double *wt = g.sqrtp + ab;  // Szegedy: 2 w_a <w, x> - x_a
        double2 sum = make_double2(0.0, 0.0);
        for (int i = lo; i < hi; ++i) sum = add(sum, scale(cvt(s[i]), wt[i]));
        for (int i = lo; i < hi; ++i) s[i] = pack<T>(sub(scale(sum, 2.0 * wt[i]), cvt(s[i])));
      } else {
        double2 sum = make_double2(0.0, 0.0);
        for (int i = lo; i < hi; ++i) sum = add(sum, cvt(s[i]));
        double2 m = grover_mean(sum, d);
        for (int i = lo; i < hi; ++i) s[i] = pack<T>(sub(add(m, m), cvt(s[i])));
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < na; i += blockDim.x) out[g.rev[ab + i]] = s[i];
  } else {
    // one vertex of degree > kTileArcs (Hadamard is never here: d = 2)
    const int v = vb;
    const bool mk = marked(g.markbits, v);
    double2 m = make_double2(0.0, 0.0);
    if (!mk) {
      double sx = 0.0, sy = 0.0;
      for (int i = ab + threadIdx.x; i < ae; i += blockDim.x) {
        double2 x = ld(in, i);
        const double wt = g.sqrtp ? g.sqrtp[i] : 1.0;
        sx += wt * x.x;
        sy += wt * x.y;
      }
      sx = block_sum(sx, red);
      sy = block_sum(sy, red);
      m = g.sqrtp ? make_double2(sx, sy) : grover_mean(make_double2(sx, sy), na);
    }
    for (int i = ab + threadIdx.x; i < ae; i += blockDim.x) {
      double2 x = ld(in, i);
      double2 phi = mk ? scale(x, -1.0)
                       : (g.sqrtp ? sub(scale(m, 2.0 * g.sqrtp[i]), x) : sub(add(m, m), x));
      st(out, g.rev[i], phi);
    }
  }
}

// ---- coined: index-free structured layouts ------------------------------------
// Internal state is slot-major: element (slot j, vertex v) at j*n + v.
//   CYCLE:     slot 0 -> v+1, slot 1 -> v-1; reverse slot 1-j.
//   TORUS:     v = r*l2 + c; slots c+1, c-1, r+1, r-1; reverse slot j^1.
//   HYPERCUBE: slot j -> v xor 2^j; reverse slot j.
// One thread per vertex: the d loads and the d stores are each coalesced
// across the wavefront.
template <int KIND>
__device__ __forceinline__ int head_of(int v, int j, int n, int l2) {
  if (KIND == kCycle) {
    return j == 0 ? (v + 1 == n ? 0 : v + 1) : (v == 0 ? n - 1 : v - 1);
  } else if (KIND == kTorus) {
    const int r = v / l2, c = v - r * l2;
    switch (j) {
      case 0: return r * l2 + (c + 1 == l2 ? 0 : c + 1);
      case 1: return r * l2 + (c == 0 ? l2 - 1 : c - 1);
      case 2: return (r + 1 == n / l2 ? 0 : r + 1) * l2 + c;
      default: return (r == 0 ? n / l2 - 1 : r - 1) * l2 + c;
    }
  } else {
    return v ^ (1 << j);
  }
}
template <int KIND> __device__ __forceinline__ int rev_slot(int j) {
  return KIND == kCycle ? 1 - j : (KIND == kTorus ? (j ^ 1) : j);
}

template <typename T, int KIND, int D>
__global__ __launch_bounds__(kBlock) void k_coined_struct(GraphView g, const T *__restrict__ in,
                                                          T *__restrict__ out, int dim,
                                                          int hadamard) {
  const int n = g.n;
  const int v = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int d = (KIND == kHypercube) ? dim : D;
  const int l2 = g.dims[1];
  T x[D];
#pragma unroll
  for (int j = 0; j < D; ++j)
    if (j < d) x[j] = in[static_cast<int64_t>(j) * n + v];
  const bool mk = marked(g.markbits, v);
  if (mk) {
#pragma unroll
    for (int j = 0; j < D; ++j)
      if (j < d) x[j] = pack<T>(scale(cvt(x[j]), -1.0));
  } else if (KIND == kCycle && hadamard) {
    double2 x0 = cvt(x[0]), x1 = cvt(x[1]);
    x[0] = pack<T>(scale(add(x0, x1), kInvSqrt2));
    x[1] = pack<T>(scale(sub(x0, x1), kInvSqrt2));
  } else if (KIND != kHypercube && g.coin) {
    // d x d coin on the slots, which are the rows' (direction) order here:
    // phi_j = sum_k C[j][k] x_k, FP64, with the entries read uniformly
    double2 xin[D];
#pragma unroll
    for (int k = 0; k < D; ++k) xin[k] = cvt(x[k]);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const double cr = g.coin[2 * (j * D + k)], ci = g.coin[2 * (j * D + k) + 1];
        re += cr * xin[k].x - ci * xin[k].y;
        im += cr * xin[k].y + ci * xin[k].x;
      }
      x[j] = pack<T>(make_double2(re, im));
    }
  } else {
    double2 sum = make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < D; ++j)
      if (j < d) sum = add(sum, cvt(x[j]));
    double2 m = grover_mean(sum, d);
#pragma unroll
    for (int j = 0; j < D; ++j)
      if (j < d) x[j] = pack<T>(sub(add(m, m), cvt(x[j])));
  }
  // flip-flop: the amplitude moves to the reverse arc's slot at the head;
  // persistent (lattices): it keeps its direction slot
  const bool keep = KIND != kHypercube && g.persistent;
#pragma unroll
  for (int j = 0; j < D; ++j)
    if (j < d) out[static_cast<int64_t>(keep ? j : rev_slot<KIND>(j)) * n + head_of<KIND>(v, j, n, l2)] = x[j];
}

// internal[i] = psi[perm[i]]
template <typename T>
__global__ __launch_bounds__(kBlock) void k_perm_in(const T *__restrict__ psi, T *__restrict__ internal,
                                                    const int32_t *__restrict__ perm, int na) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < na) internal[i] = psi[perm[i]];
}

// psi[perm[j*n+v]] = internal[j*n+v], one thread per vertex, with the vertex
// probability fused: p_v = sum_j |internal[j*n+v]|^2.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_perm_out(const T *__restrict__ internal, T *__restrict__ psi,
                                                     const int32_t *__restrict__ perm, int n, int d,
                                                     double *p, double *partials) {
  __shared__ double red[16];
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  double pv = 0.0;
  if (v < n) {
    for (int j = 0; j < d; ++j) {
      const int64_t i = static_cast<int64_t>(j) * n + v;
      T x = internal[i];
      psi[perm[i]] = x;
      pv += abs2(cvt(x));
    }
    if (p) p[v] = pv;
  }
  if (partials) {
    double tot = block_sum(pv, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy(const T *__restrict__ in, T *__restrict__ out, int64_t len) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < len) out[i] = in[i];
}

// Coined readout on the CSR arc order: p_v = sum over row v of |psi_a|^2.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prob_csr(GraphView g, const T *__restrict__ psi, double *p,
                                                     double *partials) {
  // The workgroup's vertices own one contiguous run of arcs: it is staged
  // through LDS in chunks with coalesced loads, and each thread adds its
  // vertex's |psi_a|^2 from there in arc order (a vertex block of d arcs read
  // by one thread straight from memory would touch d cache lines per step of
  // the wavefront).
  constexpr int kChunk = 2048;
  __shared__ T cs[kChunk];
  __shared__ double red[16];
  const int n = g.n;
  const int v0 = blockIdx.x * blockDim.x;
  const int v = v0 + threadIdx.x;
  const int v1 = v0 + static_cast<int>(blockDim.x) < n ? v0 + static_cast<int>(blockDim.x) : n;
  const int ab = g.rp[v0], ae = g.rp[v1];
  const int lo = v < n ? g.rp[v] : 0, hi = v < n ? g.rp[v + 1] : 0;
  double pv = 0.0;
  for (int c0 = ab; c0 < ae; c0 += kChunk) {
    const int c1 = c0 + kChunk < ae ? c0 + kChunk : ae;
    __syncthreads();  // the previous chunk is no longer read
    for (int i = threadIdx.x; i < c1 - c0; i += blockDim.x) cs[i] = psi[c0 + i];
    __syncthreads();
    const int a0 = lo > c0 ? lo : c0, a1 = hi < c1 ? hi : c1;
    for (int a = a0; a < a1; ++a) pv += abs2(cvt(cs[a - c0]));
  }
  if (v < n) p[v] = pv;
  double tot = block_sum(pv, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// CTQW readout: p_v = |psi_v|^2.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prob_vertex(const T *__restrict__ psi, int n, double *p,
                                                        double *partials) {
  __shared__ double red[16];
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  double pv = 0.0;
  if (v < n) {
    pv = abs2(ld(psi, v));
    p[v] = pv;
  }
  double tot = block_sum(pv, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// Sum of y over a row's neighbours, in arc order a = lo..hi-1.  A row of up to
// 8 arcs issues all its index loads, then all its gathers, before the first
// add, so a lane keeps up to 8 independent loads in flight instead of a chain
// of dependent ones; longer rows go 4 arcs at a time.  The summation order is
// the same in every branch, so results do not depend on which one runs.
template <typename T>
__device__ __forceinline__ double2 gather_sum(const T *__restrict__ y, const int32_t *__restrict__ col, int lo,
                                              int hi) {
  const int d = hi - lo;
  double2 s = make_double2(0.0, 0.0);
  if (d <= 8) {
    int c[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j < d) c[j] = col[lo + j];
    T x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j < d) x[j] = y[c[j]];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j < d) s = add(s, cvt(x[j]));
  } else {
    int a = lo;
    for (; a + 4 <= hi; a += 4) {
      const int c0 = col[a], c1 = col[a + 1], c2 = col[a + 2], c3 = col[a + 3];
      const T x0 = y[c0], x1 = y[c1], x2 = y[c2], x3 = y[c3];
      s = add(s, cvt(x0));
      s = add(s, cvt(x1));
      s = add(s, cvt(x2));
      s = add(s, cvt(x3));
    }
    for (; a < hi; ++a) s = add(s, cvt(y[col[a]]));
  }
  return s;
}

// Same sum for the column-major neighbour table of a d-regular graph:
// neighbour j of v at colT[j*n + v], so the index loads of a wavefront are
// contiguous and no row pointer is read.  Order j = 0..d-1 is row order.
template <typename T>
__device__ __forceinline__ double2 ell_gather_sum(const T *__restrict__ y, const int32_t *__restrict__ colT,
                                                  int n, int d, int v) {
  double2 s = make_double2(0.0, 0.0);
  if (d <= 8) {
    int c[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j < d) c[j] = colT[static_cast<int64_t>(j) * n + v];
    T x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j < d) x[j] = y[c[j]];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j < d) s = add(s, cvt(x[j]));
  } else {
    int j = 0;
    for (; j + 4 <= d; j += 4) {
      const int64_t b = static_cast<int64_t>(j) * n + v;
      const int c0 = colT[b], c1 = colT[b + n], c2 = colT[b + 2 * static_cast<int64_t>(n)],
                c3 = colT[b + 3 * static_cast<int64_t>(n)];
      const T x0 = y[c0], x1 = y[c1], x2 = y[c2], x3 = y[c3];
      s = add(s, cvt(x0));
      s = add(s, cvt(x1));
      s = add(s, cvt(x2));
      s = add(s, cvt(x3));
    }
    for (; j < d; ++j) s = add(s, cvt(y[colT[static_cast<int64_t>(j) * n + v]]));
  }
  return s;
}

// ---- CTQW: one Horner stage ---------------------------------------------------
// y_out = psi + i (alpha sum_{u~v} y_u + beta [v in M] y_v)
// psi + i (alpha nsum + beta [marked] yv).  The unmarked part is one fused
// multiply-add per component and the marked term a second one, so an
// unmarked cell gets the same bits whether or not the code path allows a
// marked term (overlapping grid strips of the two kinds store equal values).
__device__ __forceinline__ double2 horner_out(double2 psi, double2 nsum, double2 yv, bool mk,
                                              double alpha, double beta) {
  double re = __fma_rn(-alpha, nsum.y, psi.x);
  double im = __fma_rn(alpha, nsum.x, psi.y);
  if (mk) {
    re = __fma_rn(-beta, yv.y, re);
    im = __fma_rn(beta, yv.x, im);
  }
  return make_double2(re, im);
}

// General CSR, G lanes per row (G in 1..64, power of two), lane sums strided
// by G then a butterfly across the G lanes.  PROB fuses the readout.
template <typename T, int G, bool PROB>
__global__ __launch_bounds__(kBlock) void k_ctqw_csr(GraphView g, const T *__restrict__ y,
                                                     const T *psi, T *out, double alpha, double beta,
                                                     double *p, double *partials) {
  __shared__ double red[16];
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int row = gid / G, lane = gid % G;
  double sx = 0.0, sy = 0.0;
  if (row < g.n) {
    const int lo = g.rp[row], hi = g.rp[row + 1];
    if (G == 1) {
      const double2 t = gather_sum(y, g.col, lo, hi);
      sx = t.x;
      sy = t.y;
    } else {
      for (int a = lo + lane; a < hi; a += G) {
        double2 x = ld(y, g.col[a]);
        sx += x.x;
        sy += x.y;
      }
    }
  }
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) {
    sx += __shfl_xor(sx, off, 64);
    sy += __shfl_xor(sy, off, 64);
  }
  double pv = 0.0;
  if (row < g.n && lane == 0) {
    const bool mk = marked(g.markbits, row);
    double2 yv = mk ? ld(y, row) : make_double2(0.0, 0.0);
    double2 r = horner_out(ld(psi, row), make_double2(sx, sy), yv, mk, alpha, beta);
    st(out, row, r);
    if (PROB) {
      T stored = pack<T>(r);
      pv = abs2(cvt(stored));
      p[row] = pv;
    }
  }
  if (PROB) {
    double tot = block_sum(pv, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
  }
}

// Out-of-core stage: rows [r0, r1) of a CSR graph whose neighbour indices were
// copied into a device slot (slot[a - arc0] = col[a]); one thread per row,
// neighbours summed in arc order.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_ctqw_csr_slot(const int32_t *__restrict__ rp,
                                                          const int32_t *__restrict__ slot, int64_t arc0,
                                                          int r0, int r1, const uint32_t *markbits,
                                                          const T *__restrict__ y, const T *psi, T *out,
                                                          double alpha, double beta) {
  const int r = r0 + static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
  if (r >= r1) return;
  const int lo = static_cast<int>(rp[r] - arc0), hi = static_cast<int>(rp[r + 1] - arc0);
  const double2 sum = gather_sum(y, slot, lo, hi);
  const bool mk = marked(markbits, r);
  const double2 yv = mk ? ld(y, r) : make_double2(0.0, 0.0);
  st(out, r, horner_out(ld(psi, r), sum, yv, mk, alpha, beta));
}

// Direct out-of-core stage.  The neighbour indices of most arcs sit in pinned
// host memory and are read across the host link by the kernel itself: a
// workgroup stages its tile's indices into LDS with 16-byte loads (a
// contiguous run of arcs, so every load instruction of a wavefront reads 1 KiB
// of consecutive host memory), then each thread sums its row from LDS in arc
// order, as the other CSR stages do.  A row with more arcs than the LDS holds
// is its own tile, staged chunk by chunk and summed by one thread.
__device__ __forceinline__ void dir_stage(int32_t *cs, const int32_t *dcol, const int32_t *hcol, int64_t split,
                                          int64_t a0, int64_t a1) {
  // cs[a - (a0 & ~3)] = col[a] for a in [a0 & ~3, (a1 + 3) & ~3): whole 16-byte groups,
  // each from one side of `split`
  const int64_t q0 = a0 >> 2, q1 = (a1 + 3) >> 2;
  const int4 *d4 = reinterpret_cast<const int4 *>(dcol);
  const int4 *h4 = reinterpret_cast<const int4 *>(hcol);
  int4 *c4 = reinterpret_cast<int4 *>(cs);
  for (int64_t q = q0 + threadIdx.x; q < q1; q += blockDim.x) c4[q - q0] = (q << 2) < split ? d4[q] : h4[q];
}

template <typename T>
__device__ __forceinline__ double2 gather_fold(double2 s, const T *__restrict__ y, const int32_t *col, int lo,
                                               int hi) {
  for (int a = lo; a < hi; ++a) s = add(s, cvt(y[col[a]]));
  return s;
}

template <typename T>
__global__ __launch_bounds__(kDirRows) void k_ctqw_csr_direct(const int32_t *__restrict__ rp,
                                                            const int32_t *__restrict__ wg_row,
                                                            const int32_t *dcol, const int32_t *hcol,
                                                            int64_t split, const uint32_t *markbits,
                                                            const T *__restrict__ y, const T *psi, T *out,
                                                            double alpha, double beta) {
  __shared__ __align__(16) int32_t cs[kDirArcs + 8];
  const int rb = wg_row[blockIdx.x], re = wg_row[blockIdx.x + 1];
  const int64_t ab = rp[rb], ae = rp[re];
  if (ae - ab <= kDirArcs) {
    dir_stage(cs, dcol, hcol, split, ab, ae);
    __syncthreads();
    const int r = rb + static_cast<int>(threadIdx.x);
    if (r >= re) return;
    const int base = static_cast<int>(ab & 3) - static_cast<int>(ab);  // cs index of arc a: a + base
    const double2 sum = gather_sum(y, static_cast<const int32_t *>(cs), rp[r] + base, rp[r + 1] + base);
    const bool mk = marked(markbits, r);
    const double2 yv = mk ? ld(y, r) : make_double2(0.0, 0.0);
    st(out, r, horner_out(ld(psi, r), sum, yv, mk, alpha, beta));
    return;
  }
  // one row (re = rb + 1) longer than a tile: its arcs in chunks of kDirArcs, folded in order
  double2 sum = make_double2(0.0, 0.0);
  for (int64_t c0 = ab; c0 < ae; c0 += kDirArcs) {
    const int64_t c1 = c0 + kDirArcs < ae ? c0 + kDirArcs : ae;
    __syncthreads();  // the previous chunk is no longer read
    dir_stage(cs, dcol, hcol, split, c0, c1);
    __syncthreads();
    if (threadIdx.x == 0) {
      const int lo = static_cast<int>(c0 & 3);
      sum = gather_fold(sum, y, static_cast<const int32_t *>(cs), lo, lo + static_cast<int>(c1 - c0));
    }
  }
  if (threadIdx.x == 0) {
    const bool mk = marked(markbits, rb);
    const double2 yv = mk ? ld(y, rb) : make_double2(0.0, 0.0);
    st(out, rb, horner_out(ld(psi, rb), sum, yv, mk, alpha, beta));
  }
}

// Regular graphs: ELL stage, one thread per row, column-major neighbour table.
template <typename T, bool PROB>
__global__ __launch_bounds__(kBlock) void k_ctqw_ell(GraphView g, const T *__restrict__ y, const T *psi,
                                                     T *out, double alpha, double beta, double *p,
                                                     double *partials) {
  __shared__ double red[16];
  const int n = g.n;
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  double pv = 0.0;
  if (v < n) {
    const double2 s = ell_gather_sum(y, g.col, n, g.ell_d, v);
    const bool mk = marked(g.markbits, v);
    const double2 yv = mk ? ld(y, v) : make_double2(0.0, 0.0);
    const double2 r = horner_out(ld(psi, v), s, yv, mk, alpha, beta);
    st(out, v, r);
    if (PROB) {
      pv = abs2(cvt(pack<T>(r)));
      p[v] = pv;
    }
  }
  if (PROB) {
    double tot = block_sum(pv, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
  }
}

// Regular graphs whose vector is several times an XCD's L2 (above
// kEllSliceFrom bytes): the same ELL stage, column-sliced.  A thread takes RPT
// rows of a row group and loads their neighbour indices once; then, for each
// slice of kEllSliceEntries entries of the input vector in turn, it gathers
// only the neighbours inside that slice.  The grid is what the GPU holds at
// once (groups taken grid-stride), so its workgroups walk the slices together
// and an XCD's L2 holds the slice being gathered instead of a random part of
// the whole vector.  Rows are sorted by neighbour, so adding slice after slice
// adds each row's neighbours in row order: the result is bitwise that of
// k_ctqw_ell.
template <typename T, int RPT>
__global__ __launch_bounds__(kBlock) void k_ctqw_ell_sliced(GraphView g, const T *__restrict__ y, const T *psi,
                                                            T *out, double alpha, double beta, int slice) {
  const int n = g.n, d = g.ell_d;
  const int n_groups = (n + kBlock * RPT - 1) / (kBlock * RPT);
  for (int grp = blockIdx.x; grp < n_groups; grp += gridDim.x) {
    const int r0 = grp * (kBlock * RPT) + static_cast<int>(threadIdx.x);
    int c[RPT][8];  // neighbour indices; -1 (never inside a slice as unsigned) pads
    double2 acc[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = r0 + i * kBlock;
      const int rc = r < n ? r : n - 1;
#pragma unroll
      for (int j = 0; j < 8; ++j) c[i][j] = g.col[static_cast<int64_t>(j < d ? j : d - 1) * n + rc];
#pragma unroll
      for (int j = 0; j < 8; ++j) c[i][j] = (r < n && j < d) ? c[i][j] : -1;
      acc[i] = make_double2(0.0, 0.0);
    }
    for (int s0 = 0; s0 < n; s0 += slice) {
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        T x[8];
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (static_cast<unsigned>(c[i][j] - s0) < static_cast<unsigned>(slice)) x[j] = y[c[i][j]];
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (static_cast<unsigned>(c[i][j] - s0) < static_cast<unsigned>(slice)) acc[i] = add(acc[i], cvt(x[j]));
      }
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = r0 + i * kBlock;
      if (r >= n) continue;
      const bool mk = marked(g.markbits, r);
      const double2 yv = mk ? ld(y, r) : make_double2(0.0, 0.0);
      st(out, r, horner_out(ld(psi, r), acc[i], yv, mk, alpha, beta));
    }
  }
}

// The same slicing on the CSR layout (rows sorted by neighbour), G lanes per
// row as in k_ctqw_csr<G>: lane l of a row takes its arcs lo + l + G m, the
// first eight of them held in registers, the rest (rows longer than 8 G) read
// from memory behind a cursor.  In each slice's pass a lane adds its arcs that
// fall inside the slice in increasing m, so each lane's sum, and the butterfly
// across the row's lanes, are those of k_ctqw_csr<G>: the same bits.
template <typename T, int G>
__global__ __launch_bounds__(kBlock) void k_ctqw_csr_sliced(GraphView g, const T *__restrict__ y, const T *psi,
                                                            T *out, double alpha, double beta, int slice) {
  constexpr int RPW = kBlock / G;  // rows per workgroup
  const int n = g.n;
  const int n_groups = (n + RPW - 1) / RPW;
  const int lane = static_cast<int>(threadIdx.x) % G;
  for (int grp = blockIdx.x; grp < n_groups; grp += gridDim.x) {
    const int row = grp * RPW + static_cast<int>(threadIdx.x) / G;
    const int lo = row < n ? g.rp[row] : 0, hi = row < n ? g.rp[row + 1] : 0;
    unsigned c[8];  // 0xffffffff (never inside a slice) pads
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int a = lo + lane + G * m;
      c[m] = a < hi ? static_cast<unsigned>(g.col[a]) : 0xffffffffu;
    }
    int cur = lo + lane + 8 * G;  // next arc of this lane beyond the registers
    double2 acc = make_double2(0.0, 0.0);
    for (int s0 = 0; s0 < n; s0 += slice) {
      const unsigned b0 = static_cast<unsigned>(s0), b1 = b0 + static_cast<unsigned>(slice);
      T x[8];
#pragma unroll
      for (int m = 0; m < 8; ++m)
        if (c[m] - b0 < b1 - b0) x[m] = y[c[m]];
#pragma unroll
      for (int m = 0; m < 8; ++m)
        if (c[m] - b0 < b1 - b0) acc = add(acc, cvt(x[m]));
      while (cur < hi) {  // rows longer than 8 G: the lane's later arcs, in order
        const unsigned cc = static_cast<unsigned>(g.col[cur]);
        if (cc >= b1) break;
        acc = add(acc, cvt(y[cc]));
        cur += G;
      }
    }
    double sx = acc.x, sy = acc.y;
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
      sx += __shfl_xor(sx, off, 64);
      sy += __shfl_xor(sy, off, 64);
    }
    if (row < n && lane == 0) {
      const bool mk = marked(g.markbits, row);
      const double2 yv = mk ? ld(y, row) : make_double2(0.0, 0.0);
      st(out, row, horner_out(ld(psi, row), make_double2(sx, sy), yv, mk, alpha, beta));
    }
  }
}

// workgroups of `kernel` (kBlock threads) the current device holds at once
template <typename K> int resident_groups(K kernel) {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 1024;
  if (cached[dev] > 0) return cached[dev];
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess || per_cu <= 0 ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
    (void)hipGetLastError();
    return 1024;
  }
  cached[dev] = per_cu * cus;
  return cached[dev];
}

// Structured stencils (no index arrays): neighbours computed from v.
template <typename T, int KIND, bool PROB>
__global__ __launch_bounds__(kBlock) void k_ctqw_struct(GraphView g, const T *__restrict__ y,
                                                        const T *psi, T *out, double alpha,
                                                        double beta, double *p, double *partials) {
  __shared__ double red[16];
  const int n = g.n;
  const int v = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  double pv = 0.0;
  if (v < n) {
    double2 s = make_double2(0.0, 0.0);
    if (KIND == kHypercube) {
      const int dim = g.dims[0];
      for (int j = 0; j < dim; ++j) s = add(s, ld(y, v ^ (1 << j)));
    } else if (KIND == kCycle) {
      s = add(ld(y, head_of<kCycle>(v, 0, n, 0)), ld(y, head_of<kCycle>(v, 1, n, 0)));
    } else {
      const int l2 = g.dims[1];
#pragma unroll
      for (int j = 0; j < 4; ++j) s = add(s, ld(y, head_of<kTorus>(v, j, n, l2)));
    }
    const bool mk = marked(g.markbits, v);
    double2 yv = mk ? ld(y, v) : make_double2(0.0, 0.0);
    double2 r = horner_out(ld(psi, v), s, yv, mk, alpha, beta);
    st(out, v, r);
    if (PROB) {
      pv = abs2(cvt(pack<T>(r)));
      p[v] = pv;
    }
  }
  if (PROB) {
    double tot = block_sum(pv, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
  }
}

struct Coefs {
  double alpha[64];
  double beta[64];
};
// The same coefficients for FP32 arithmetic, each split into a float head and
// the float rounding of its remainder (alpha = hi + lo to about 2^-48
// relative), so that no coefficient of the propagator carries an FP32 rounding
// error from step to step: only the arithmetic rounds.
struct CoefsF32 {
  float ahi[64], alo[64];
  float bhi[64], blo[64];
};

// ---- one-lane wavefront shifts ---------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ double lane_shift(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
template <int CTRL>
__device__ __forceinline__ float lane_shift(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double2 lane_shift(double2 v) {
  return make_double2(lane_shift<CTRL>(v.x), lane_shift<CTRL>(v.y));
}
template <int CTRL>
__device__ __forceinline__ float2 lane_shift(float2 v) {
  return make_float2(lane_shift<CTRL>(v.x), lane_shift<CTRL>(v.y));
}

// ---- grid CTQW, streaming temporal blocking ----------------------------------------
// One wavefront sweeps a strip of the l1 x l2 torus from top to bottom: 64
// columns (core 64 - 2S) by R core rows plus S halo rows above and below.  At
// sweep position t the window row t arrives (y and psi, fetched one body of
// kSweepRing rows ahead), and stage s = 1 .. S computes its value of window
// row t - s from stage s-1's rows t-s-1, t-s, t-s+1: each stage keeps only its
// last three rows, so the registers hold O(S) rows however tall the strip is,
// and the loads stream in while earlier rows compute.  Row neighbours beside a
// cell come from the adjacent lanes through one-lane wavefront shifts; the
// outermost lanes read zeros, so the valid columns shrink by one per stage and
// the core 64 - 2S lanes are exact after S stages.  Stage s starts at t = 2s,
// where its rows become exact, and the last stage stores each core row as soon
// as it is computed.  The sweep computes in its storage type: complex128 in
// FP64, complex64 in FP32 with split coefficients (CoefsF32), which halves the
// lane shifts (one DPP move per float instead of two per double) and needs no
// conversions; the neighbours are summed in the one-stage kernel's order.
// Strips at the grid's right and bottom edges are clamped and overlap their
// neighbour; duplicate stores write equal values.
constexpr int kSweepRing = 6;  // rows per unrolled body; holds psi for S <= 5 stages

__device__ __forceinline__ constexpr int pmod(int a, int m) { return ((a % m) + m) % m; }

template <typename T> struct SweepCoefs;
template <> struct SweepCoefs<double2> { using type = Coefs; };
template <> struct SweepCoefs<float2> { using type = CoefsF32; };

__device__ __forceinline__ float2 sweep_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 sweep_add(double2 a, double2 b) { return add(a, b); }
__device__ __forceinline__ float2 sweep_zero(float2) { return make_float2(0.0f, 0.0f); }
__device__ __forceinline__ double2 sweep_zero(double2) { return make_double2(0.0, 0.0); }

// psi + i (alpha nsum + beta [marked] y) at stage k (index k - 1)
__device__ __forceinline__ double2 sweep_out(double2 psi, double2 nsum, double2 yv, bool mk, const Coefs &c,
                                             int ki) {
  return horner_out(psi, nsum, yv, mk, c.alpha[ki], c.beta[ki]);
}
__device__ __forceinline__ float2 sweep_out(float2 psi, float2 nsum, float2 yv, bool mk, const CoefsF32 &c,
                                            int ki) {
  float re = __fmaf_rn(-c.ahi[ki], nsum.y, psi.x);
  float im = __fmaf_rn(c.ahi[ki], nsum.x, psi.y);
  re = __fmaf_rn(-c.alo[ki], nsum.y, re);
  im = __fmaf_rn(c.alo[ki], nsum.x, im);
  if (mk) {
    re = __fmaf_rn(-c.bhi[ki], yv.y, re);
    im = __fmaf_rn(c.bhi[ki], yv.x, im);
    re = __fmaf_rn(-c.blo[ki], yv.y, re);
    im = __fmaf_rn(c.blo[ki], yv.x, im);
  }
  return make_float2(re, im);
}

template <typename T, int S, bool YP, bool MARK>
__device__ __forceinline__ void sweep_strip(const GraphView &g, const T *__restrict__ P, const T *__restrict__ Yin,
                                            T *__restrict__ Out, int kfirst, const typename SweepCoefs<T>::type &c,
                                            int R, int rb, int lane, int gcol, unsigned boff) {
  constexpr int RING = kSweepRing, W = 64;
  static_assert(S >= 2 && S < RING, "psi ring holds rows t-S .. t");
  const int l1 = g.dims[0], l2 = g.dims[1];
  const int n_in = R + 2 * S;
  auto row_off = [&](int t) -> size_t {
    const int gr = rb + t;  // < 2 l1 since n_in <= l1
    return static_cast<size_t>(gr >= l1 ? gr - l1 : gr) * l2;
  };
  auto at = [](const T *row, unsigned off) -> T {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(row) + off);
  };
  // rows of the next body, fetched while the current one computes (rows past
  // the strip's end re-read its last row and are never used)
  T ny[RING], np[RING];
  uint32_t nmw[RING], nms[RING];  // marked-set word and bit position of each row's cell
  auto fetch = [&](int t0) {
#pragma unroll
    for (int i = 0; i < RING; ++i) {
      const size_t o = row_off(min(t0 + i, n_in - 1));
      np[i] = at(P + o, boff);
      ny[i] = YP ? np[i] : at(Yin + o, boff);
      if (MARK) {
        const int v = static_cast<int>(o) + gcol;
        nmw[i] = g.markbits[v >> 5];
        nms[i] = static_cast<uint32_t>(v & 31);
      }
    }
  };
  T yv[S][3];        // stage s-1 (s = 1 .. S) rows, slot = window row mod 3
  T pr[RING];        // psi, slot = window row mod RING
  uint32_t mr = 0;   // bit k: window row t - k is marked
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int j = 0; j < 3; ++j) yv[s][j] = sweep_zero(T{});
#pragma unroll
  for (int j = 0; j < RING; ++j) pr[j] = sweep_zero(T{});

  // one body: window rows t0 .. t0 + RING - 1.  FULL: every row exists and
  // every stage is past its warm-up, so the body has no branches.
  auto body = [&](int t0, auto full_tag) {
    constexpr bool FULL = decltype(full_tag)::value;
    T cy[RING], cp[RING];
    uint32_t cmw[RING], cms[RING];
#pragma unroll
    for (int i = 0; i < RING; ++i) {
      cy[i] = ny[i];
      cp[i] = np[i];
      if (MARK) {
        cmw[i] = nmw[i];
        cms[i] = nms[i];
      }
    }
    if (t0 + RING < n_in) fetch(t0 + RING);
#pragma unroll
    for (int i = 0; i < RING; ++i) {
      const int t = t0 + i;  // t0 is a multiple of RING, so every ring slot below is static
      if (!FULL && t >= n_in) break;
      yv[0][i % 3] = cy[i];
      pr[i] = cp[i];
      if (MARK) mr = (mr << 1) | ((cmw[i] >> cms[i]) & 1u);
#pragma unroll
      for (int st = 1; st <= S; ++st) {
        if (!FULL && t < 2 * st) break;  // window rows above stage st's exact region
        const T up = yv[st - 1][pmod(i - st - 1, 3)];
        const T self = yv[st - 1][pmod(i - st, 3)];
        const T dn = yv[st - 1][pmod(i - st + 1, 3)];
        const T left = lane_shift<kFromLower>(self), right = lane_shift<kFromUpper>(self);
        // the one-stage kernel's order: right, left, below, above
        T sum = sweep_add(right, left);
        sum = sweep_add(sum, dn);
        sum = sweep_add(sum, up);
        const bool m = MARK && ((mr >> st) & 1u);
        const T val = sweep_out(pr[pmod(i - st, RING)], sum, self, m, c, kfirst - st);
        if (st < S) {
          yv[st][pmod(i - st, 3)] = val;
        } else if (lane >= S && lane < W - S) {
          *reinterpret_cast<T *>(reinterpret_cast<char *>(Out + row_off(t - S)) + boff) = val;
        }
      }
    }
  };
  fetch(0);
  int t0 = 0;
  for (; t0 < 2 * S; t0 += RING) body(t0, std::false_type{});
  for (; t0 + RING <= n_in; t0 += RING) body(t0, std::true_type{});
  if (t0 < n_in) body(t0, std::false_type{});
}

template <typename T, int S, bool YP>
__global__ __launch_bounds__(64 * kStripWaves) void k_ctqw_torus_sweep(GraphView g, const T *__restrict__ P,
                                                                       const T *__restrict__ Yin,
                                                                       T *__restrict__ Out, int kfirst,
                                                                       typename SweepCoefs<T>::type c) {
  constexpr int CORE = 64 - 2 * S;
  const int l1 = g.dims[0], l2 = g.dims[1], R = g.strip_rows;
  const int tiles_c = (l2 + CORE - 1) / CORE, tiles_r = (l1 + R - 1) / R;
  const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int tile = xcd_remap(blockIdx.x, gridDim.x) * kStripWaves + wv;
  if (tile >= tiles_r * tiles_c) return;  // whole wavefront
  const int lane = threadIdx.x & 63;
  const int tr = tile / tiles_c, tc = tile - tr * tiles_c;
  int rb = min(tr * R, l1 - R) - S, cb = min(tc * CORE, l2 - CORE) - S;
  rb += rb < 0 ? l1 : 0;
  cb += cb < 0 ? l2 : 0;
  int gcol = cb + lane;  // < 2 l2 since 64 <= l2
  gcol -= gcol >= l2 ? l2 : 0;
  const unsigned boff = static_cast<unsigned>(gcol) * static_cast<unsigned>(sizeof(T));
  if (g.tmark[tile])
    sweep_strip<T, S, YP, true>(g, P, Yin, Out, kfirst, c, R, rb, lane, gcol, boff);
  else
    sweep_strip<T, S, YP, false>(g, P, Yin, Out, kfirst, c, R, rb, lane, gcol, boff);
}

// CTQW small graphs: every stage of every step in one workgroup, vectors in LDS.
template <typename T>
__device__ void ctqw_small_walk(const GraphView &g, T *psi, const double *alpha, const double *beta, int K,
                                int64_t steps, const Readout &ro, unsigned char *smem, double *red) {
  const int n = g.n, na = g.n_arcs;
  T *ps = reinterpret_cast<T *>(smem);
  T *ya = ps + n;
  T *yb = ya + n;
  int32_t *srp = reinterpret_cast<int32_t *>(yb + n);
  int32_t *scol = srp + n + 1;
  uint32_t *smark = reinterpret_cast<uint32_t *>(scol + na);  // the marked bitmap, read every stage
  for (int i = threadIdx.x; i < n; i += blockDim.x) ps[i] = psi[i];
  for (int i = threadIdx.x; i <= n; i += blockDim.x) srp[i] = g.rp[i];
  for (int i = threadIdx.x; i < na; i += blockDim.x) scol[i] = g.col[i];
  for (int i = threadIdx.x; i < (n + 31) / 32; i += blockDim.x) smark[i] = g.markbits[i];
  __syncthreads();
  for (int64_t s = 0; s < steps; ++s) {
    const T *yin = ps;
    for (int k = K; k >= 1; --k) {
      T *yout = (k == 1) ? ((K == 1) ? ya : ps) : (((K - k) & 1) ? yb : ya);
      // k == 1 with K >= 2 writes psi in place: each thread reads psi[v] before
      // writing it and the gathers read yin != ps.
      for (int v = threadIdx.x; v < n; v += blockDim.x) {
        double2 sum = make_double2(0.0, 0.0);
        for (int a = srp[v]; a < srp[v + 1]; ++a) sum = add(sum, cvt(yin[scol[a]]));
        const bool mk = marked(smark, v);
        double2 yv = mk ? cvt(yin[v]) : make_double2(0.0, 0.0);
        double2 r = horner_out(cvt(ps[v]), sum, yv, mk, alpha[k - 1], beta[k - 1]);
        yout[v] = pack<T>(r);
      }
      __syncthreads();
      yin = yout;
    }
    if (K == 1) {
      for (int v = threadIdx.x; v < n; v += blockDim.x) ps[v] = ya[v];
      __syncthreads();
    }
  }
  for (int v = threadIdx.x; v < n; v += blockDim.x) psi[v] = ps[v];
  if (ro.p || ro.norm || ro.pmarked) {
    double *pout = ro.p ? ro.p : ro.pscratch;
    double acc = 0.0;
    for (int v = threadIdx.x; v < n; v += blockDim.x) {
      double pv = abs2(cvt(ps[v]));
      pout[v] = pv;
      acc += pv;
    }
    double tot = block_sum(acc, red);
    __syncthreads();
    double pm = 0.0;
    for (int i = threadIdx.x; i < g.n_marked; i += blockDim.x) pm += abs2(cvt(ps[g.marklist[i]]));
    double ptot = block_sum(pm, red);
    if (threadIdx.x == 0) {
      if (ro.norm) *ro.norm = tot;
      if (ro.pmarked) *ro.pmarked = ptot;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_ctqw_small(GraphView g, T *psi, Coefs c, int K,
                                                     int64_t steps, Readout ro) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[16];
  ctqw_small_walk<T>(g, psi, c.alpha, c.beta, K, steps, ro, smem, red);
}

// ---- staggered walk -----------------------------------------------------------
// One tessellation U = c0 I + c1 (2P - I), P = sum_alpha |alpha><alpha| over
// the tessellation's polygons: for each polygon, inner = sum_v a_v psi_v in
// position order, then psi_v <- c0 psi_v + c1 (2 a_v inner - psi_v).  The
// polygons partition the vertices, so every update is in place and touches
// only its own polygon.  On the first tessellation of a step the marked
// vertices' phase flip is applied to the values as they are read.

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double2 stag_update(const StagTess &t, double2 x, double a, double2 inner) {
  const double2 r = sub(scale(inner, 2.0 * a), x);
  return add(cmul(make_double2(t.c0[0], t.c0[1]), x), cmul(make_double2(t.c1[0], t.c1[1]), r));
}

template <typename X> __device__ __forceinline__ const X *at_off(const unsigned char *base, int64_t off) {
  return off >= 0 ? reinterpret_cast<const X *>(base + off) : nullptr;
}

// Thread path: thread p owns polygon p (at most MAXS vertices).  ELL: the
// polygons share one size and the vertex table is column-major, so lane p's
// j-th load sits next to lane p+1's.
template <typename T, int MAXS, bool ELL>
__global__ __launch_bounds__(kBlock) void k_stag_poly(const unsigned char *__restrict__ base, StagTess t,
                                                     T *psi, const uint32_t *__restrict__ markbits, int mark) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= t.n_small) return;
  const int32_t *vert = at_off<int32_t>(base, t.off_vert);
  const double *amp = at_off<double>(base, t.off_amp);
  int lo, sz, stride;
  if (ELL) {
    lo = p;
    sz = t.small_size;
    stride = t.n_small;
  } else {
    const int32_t *ptr = at_off<int32_t>(base, t.off_ptr);
    lo = ptr[p];
    sz = ptr[p + 1] - lo;
    stride = 1;
  }
  const double uni = 1.0 / sqrt(static_cast<double>(sz));
  int v[MAXS];
  double2 x[MAXS];
  double a[MAXS];
  double2 inner = make_double2(0.0, 0.0);
#pragma unroll
  for (int j = 0; j < MAXS; ++j) {
    if (j < sz) {
      const int pos = lo + j * stride;
      v[j] = vert[pos];
      double2 xv = ld(psi, v[j]);
      if (mark && marked(markbits, v[j])) xv = scale(xv, -1.0);
      x[j] = xv;
      a[j] = amp ? amp[pos] : uni;
      inner = add(inner, scale(xv, a[j]));
    }
  }
#pragma unroll
  for (int j = 0; j < MAXS; ++j)
    if (j < sz) st(psi, v[j], stag_update(t, x[j], a[j], inner));
}

// Big polygons, pass 1: workgroup c sums a_v psi_v over chunk c.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_stag_big_partial(const unsigned char *__restrict__ base, StagTess t,
                                                            const T *__restrict__ psi,
                                                            const uint32_t *__restrict__ markbits, int mark,
                                                            double2 *__restrict__ partials) {
  __shared__ double red[16];
  const StagChunk ch = at_off<StagChunk>(base, t.off_chunk)[blockIdx.x];
  const int32_t *vert = at_off<int32_t>(base, t.off_bvert);
  const double *amp = at_off<double>(base, t.off_bamp);
  const double uni = 1.0 / sqrt(static_cast<double>(ch.size));
  double2 acc = make_double2(0.0, 0.0);
  for (int i = ch.begin + threadIdx.x; i < ch.end; i += kBlock) {
    const int v = vert[i];
    double2 xv = ld(psi, v);
    if (mark && marked(markbits, v)) xv = scale(xv, -1.0);
    acc = add(acc, scale(xv, amp ? amp[i] : uni));
  }
  const double re = block_sum(acc.x, red);
  const double im = block_sum(acc.y, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = make_double2(re, im);
}

// Big polygons, pass 2: workgroup c sums its polygon's partials (the same
// order in every chunk of the polygon) and updates chunk c.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_stag_big_apply(const unsigned char *__restrict__ base, StagTess t,
                                                          T *psi, const uint32_t *__restrict__ markbits, int mark,
                                                          const double2 *__restrict__ partials) {
  __shared__ double red[16];
  const StagChunk ch = at_off<StagChunk>(base, t.off_chunk)[blockIdx.x];
  const int32_t *vert = at_off<int32_t>(base, t.off_bvert);
  const double *amp = at_off<double>(base, t.off_bamp);
  const double uni = 1.0 / sqrt(static_cast<double>(ch.size));
  double2 acc = make_double2(0.0, 0.0);
  for (int i = threadIdx.x; i < ch.count; i += kBlock) acc = add(acc, partials[ch.first + i]);
  const double2 inner = make_double2(block_sum(acc.x, red), block_sum(acc.y, red));
  for (int i = ch.begin + threadIdx.x; i < ch.end; i += kBlock) {
    const int v = vert[i];
    double2 xv = ld(psi, v);
    if (mark && marked(markbits, v)) xv = scale(xv, -1.0);
    st(psi, v, stag_update(t, xv, amp ? amp[i] : uni, inner));
  }
}

// One-workgroup path: every step in LDS.  Thread-path polygons one per
// thread, big polygons one per wavefront.
template <typename T>
__device__ void stag_small_walk(const GraphView &g, T *psi, int64_t steps, const Readout &ro, unsigned char *smem,
                                double *red) {
  const int n = g.n;
  T *a = reinterpret_cast<T *>(smem);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  for (int i = threadIdx.x; i < n; i += blockDim.x) a[i] = psi[i];
  __syncthreads();
  for (int64_t s = 0; s < steps; ++s) {
    for (int i = threadIdx.x; i < g.n_marked; i += blockDim.x) {
      const int m = g.marklist[i];
      a[m] = pack<T>(scale(cvt(a[m]), -1.0));
    }
    __syncthreads();
    for (int k = 0; k < g.n_tess; ++k) {
      const StagTess &t = g.stag[k];
      const int32_t *vert = at_off<int32_t>(g.base, t.off_vert);
      const double *amp = at_off<double>(g.base, t.off_amp);
      const int32_t *ptr = at_off<int32_t>(g.base, t.off_ptr);
      for (int p = threadIdx.x; p < t.n_small; p += blockDim.x) {
        int lo, sz, stride;
        if (t.small_size > 0) {
          lo = p;
          sz = t.small_size;
          stride = t.n_small;
        } else {
          lo = ptr[p];
          sz = ptr[p + 1] - lo;
          stride = 1;
        }
        const double uni = 1.0 / sqrt(static_cast<double>(sz));
        double2 inner = make_double2(0.0, 0.0);
        for (int j = 0; j < sz; ++j) {
          const int pos = lo + j * stride;
          inner = add(inner, scale(cvt(a[vert[pos]]), amp ? amp[pos] : uni));
        }
        for (int j = 0; j < sz; ++j) {
          const int pos = lo + j * stride;
          const int v = vert[pos];
          a[v] = pack<T>(stag_update(t, cvt(a[v]), amp ? amp[pos] : uni, inner));
        }
      }
      const int32_t *bptr = at_off<int32_t>(g.base, t.off_bptr);
      const int32_t *bvert = at_off<int32_t>(g.base, t.off_bvert);
      const double *bamp = at_off<double>(g.base, t.off_bamp);
      for (int q = wave; q < t.n_big; q += nwaves) {
        const int lo = bptr[q], hi = bptr[q + 1];
        const double uni = 1.0 / sqrt(static_cast<double>(hi - lo));
        double2 acc = make_double2(0.0, 0.0);
        for (int i = lo + lane; i < hi; i += 64) acc = add(acc, scale(cvt(a[bvert[i]]), bamp ? bamp[i] : uni));
        const double2 inner = make_double2(wave_sum(acc.x), wave_sum(acc.y));
        for (int i = lo + lane; i < hi; i += 64) {
          const int v = bvert[i];
          a[v] = pack<T>(stag_update(t, cvt(a[v]), bamp ? bamp[i] : uni, inner));
        }
      }
      __syncthreads();
    }
  }
  for (int v = threadIdx.x; v < n; v += blockDim.x) psi[v] = a[v];
  if (ro.p || ro.norm || ro.pmarked) {
    double *pout = ro.p ? ro.p : ro.pscratch;
    double acc = 0.0;
    for (int v = threadIdx.x; v < n; v += blockDim.x) {
      const double pv = abs2(cvt(a[v]));
      pout[v] = pv;
      acc += pv;
    }
    const double tot = block_sum(acc, red);
    __syncthreads();
    double pm = 0.0;
    for (int i = threadIdx.x; i < g.n_marked; i += blockDim.x) pm += abs2(cvt(a[g.marklist[i]]));
    const double ptot = block_sum(pm, red);
    if (threadIdx.x == 0) {
      if (ro.norm) *ro.norm = tot;
      if (ro.pmarked) *ro.pmarked = ptot;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_stag_small(GraphView g, T *psi, int64_t steps, Readout ro) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[16];
  stag_small_walk<T>(g, psi, steps, ro, smem, red);
}

// Staggered walk on the periodic l1 x l2 square lattice (l1, l2 even):
// tessellation a holds the 2 x 2 squares with top-left corner at even
// coordinates, tessellation b those at odd coordinates, amplitudes 1/2.  A
// workgroup owns a tile of kLatRows x kLatCols vertices (top-left corner at
// even coordinates) and stages it with a halo of two cells on every side
// (periodic) in LDS in the storage type (each tessellation computes in FP64
// and rounds once, as the per-tessellation kernels do): the marked flip as
// it loads, tessellation a on
// every whole a-square of the staged region, then tessellation b on the
// b-squares that cover the tile (their corners lie at most one cell outside
// it, where the halo's a-squares have been applied).  Each vertex of the tile
// is a corner of exactly one b-square, whose update is stored once.
constexpr int kLatRows = 16, kLatCols = 64;
constexpr int kLatR = kLatRows + 4, kLatC = kLatCols + 4;  // staged region

// One square: inner = <alpha|x> with alpha = (1, 1, 1, 1)/2, and
// x_v <- c0 x_v + c1 (2 (1/2) inner - x_v), which for the reflection form
// (c0, c1) = (0, 1) is inner - x_v.
template <bool REFL>
__device__ __forceinline__ void lat_square(double2 &x0, double2 &x1, double2 &x2, double2 &x3, double2 c0,
                                           double2 c1) {
  const double2 inner = scale(add(add(x0, x1), add(x2, x3)), 0.5);
  if (REFL) {
    x0 = sub(inner, x0);
    x1 = sub(inner, x1);
    x2 = sub(inner, x2);
    x3 = sub(inner, x3);
  } else {
    x0 = add(cmul(c0, x0), cmul(c1, sub(inner, x0)));
    x1 = add(cmul(c0, x1), cmul(c1, sub(inner, x1)));
    x2 = add(cmul(c0, x2), cmul(c1, sub(inner, x2)));
    x3 = add(cmul(c0, x3), cmul(c1, sub(inner, x3)));
  }
}

template <typename T, bool REFL>
__global__ __launch_bounds__(256) void k_stag_lattice(GraphView g, const T *__restrict__ in, T *__restrict__ out,
                                                      double2 c0a, double2 c1a, double2 c0b, double2 c1b) {
  __shared__ T sv[kLatR][kLatC];
  const int l1 = g.dims[0], l2 = g.dims[1];
  const int tiles_c = (l2 + kLatCols - 1) / kLatCols;
  // consecutive tiles (a row of tiles, then the next) on one XCD, so the halo
  // rows a tile shares with the tile row above come from that XCD's L2
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int tr = tile / tiles_c, tc = tile - tr * tiles_c;
  const int r0 = tr * kLatRows, c0 = tc * kLatCols;  // even: kLatRows, kLatCols are even
  const bool mark = g.n_marked > 0;
  for (int e = threadIdx.x; e < kLatR * kLatC; e += blockDim.x) {
    const int i = e / kLatC, j = e - i * kLatC;
    // periodic: on lattices smaller than the staged region a vertex is staged
    // more than once, and every copy goes through the same updates
    int gr = r0 - 2 + i, gc = c0 - 2 + j;
    gr += gr < 0 ? l1 : 0;
    gc += gc < 0 ? l2 : 0;
    while (gr >= l1) gr -= l1;
    while (gc >= l2) gc -= l2;
    const int v = gr * l2 + gc;
    T x = in[v];
    if (mark && marked(g.markbits, v)) x = pack<T>(scale(cvt(x), -1.0));
    sv[i][j] = x;
  }
  __syncthreads();
  // tessellation a: squares at region rows/cols (2p, 2q), p < kLatR/2, q < kLatC/2
  for (int e = threadIdx.x; e < (kLatR / 2) * (kLatC / 2); e += blockDim.x) {
    const int p = e / (kLatC / 2), q = e - p * (kLatC / 2);
    const int i = 2 * p, j = 2 * q;
    double2 x0 = cvt(sv[i][j]), x1 = cvt(sv[i][j + 1]), x2 = cvt(sv[i + 1][j]), x3 = cvt(sv[i + 1][j + 1]);
    lat_square<REFL>(x0, x1, x2, x3, c0a, c1a);
    sv[i][j] = pack<T>(x0);
    sv[i][j + 1] = pack<T>(x1);
    sv[i + 1][j] = pack<T>(x2);
    sv[i + 1][j + 1] = pack<T>(x3);
  }
  __syncthreads();
  // tessellation b: squares at region rows/cols (2p+1, 2q+1) covering the tile
  for (int e = threadIdx.x; e < (kLatRows / 2 + 1) * (kLatCols / 2 + 1); e += blockDim.x) {
    const int p = e / (kLatCols / 2 + 1), q = e - p * (kLatCols / 2 + 1);
    const int i = 2 * p + 1, j = 2 * q + 1;
    double2 x[4] = {cvt(sv[i][j]), cvt(sv[i][j + 1]), cvt(sv[i + 1][j]), cvt(sv[i + 1][j + 1])};
    lat_square<REFL>(x[0], x[1], x[2], x[3], c0b, c1b);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int li = i + (k >> 1), lj = j + (k & 1);  // region cell of corner k
      const int gr = r0 - 2 + li, gc = c0 - 2 + lj;
      if (li >= 2 && li < 2 + kLatRows && lj >= 2 && lj < 2 + kLatCols && gr < l1 && gc < l2)
        st(out, gr * l2 + gc, x[k]);
    }
  }
}

// P steps per launch (temporal blocking): the tile is staged with a halo of
// 2P cells; every step applies the marked flip, tessellation a on every
// a-square of the staged region and tessellation b on every b-square inside
// it, writing back to LDS.  The cells whose values are still exact shrink by
// two per side and step (one for the b-squares at the border, one for the
// a-squares' alignment), so after P steps the tile is exact and is stored row
// by row.  Two steps per launch measured fastest on 4096^2 (c64 50.0, c128
// 77.1 us per step; three: 46.6 / 84.6; four: 49.4 / 96.1).
template <typename T, bool REFL, int P>
__global__ __launch_bounds__(256) void k_stag_lattice_p(GraphView g, const T *__restrict__ in, T *__restrict__ out,
                                                        double2 c0a, double2 c1a, double2 c0b, double2 c1b) {
  constexpr int H = 2 * P, R = kLatRows + 2 * H, C = kLatCols + 2 * H;
  __shared__ T sv[R][C];
  __shared__ uint8_t mk[R][C];  // marked cells, flipped again at every later step
  const int l1 = g.dims[0], l2 = g.dims[1];
  const int tiles_c = (l2 + kLatCols - 1) / kLatCols;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int tr = tile / tiles_c, tc = tile - tr * tiles_c;
  const int r0 = tr * kLatRows, c0 = tc * kLatCols;
  const bool mark = g.n_marked > 0;
  for (int e = threadIdx.x; e < R * C; e += blockDim.x) {
    const int i = e / C, j = e - i * C;
    int gr = r0 - H + i, gc = c0 - H + j;  // periodic, also on lattices smaller than the region
    while (gr < 0) gr += l1;
    while (gc < 0) gc += l2;
    while (gr >= l1) gr -= l1;
    while (gc >= l2) gc -= l2;
    const int v = gr * l2 + gc;
    T x = in[v];
    const bool m = mark && marked(g.markbits, v);
    if (m) x = pack<T>(scale(cvt(x), -1.0));
    sv[i][j] = x;
    mk[i][j] = m ? 1 : 0;
  }
  __syncthreads();
#pragma unroll 1
  for (int s = 0; s < P; ++s) {
    if (s > 0 && mark) {
      for (int e = threadIdx.x; e < R * C; e += blockDim.x) {
        const int i = e / C, j = e - i * C;
        if (mk[i][j]) sv[i][j] = pack<T>(scale(cvt(sv[i][j]), -1.0));
      }
      __syncthreads();
    }
    for (int e = threadIdx.x; e < (R / 2) * (C / 2); e += blockDim.x) {
      const int p = e / (C / 2), q = e - p * (C / 2);
      const int i = 2 * p, j = 2 * q;
      double2 x0 = cvt(sv[i][j]), x1 = cvt(sv[i][j + 1]), x2 = cvt(sv[i + 1][j]), x3 = cvt(sv[i + 1][j + 1]);
      lat_square<REFL>(x0, x1, x2, x3, c0a, c1a);
      sv[i][j] = pack<T>(x0);
      sv[i][j + 1] = pack<T>(x1);
      sv[i + 1][j] = pack<T>(x2);
      sv[i + 1][j + 1] = pack<T>(x3);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ((R - 2) / 2) * ((C - 2) / 2); e += blockDim.x) {
      const int p = e / ((C - 2) / 2), q = e - p * ((C - 2) / 2);
      const int i = 2 * p + 1, j = 2 * q + 1;
      double2 x0 = cvt(sv[i][j]), x1 = cvt(sv[i][j + 1]), x2 = cvt(sv[i + 1][j]), x3 = cvt(sv[i + 1][j + 1]);
      lat_square<REFL>(x0, x1, x2, x3, c0b, c1b);
      sv[i][j] = pack<T>(x0);
      sv[i][j + 1] = pack<T>(x1);
      sv[i + 1][j] = pack<T>(x2);
      sv[i + 1][j + 1] = pack<T>(x3);
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < kLatRows * kLatCols; e += blockDim.x) {
    const int i = e / kLatCols, j = e - i * kLatCols;
    const int gr = r0 + i, gc = c0 + j;
    if (gr < l1 && gc < l2) out[gr * l2 + gc] = sv[H + i][H + j];
  }
}

// Many independent small walks in one launch: workgroup b runs walk b whole,
// its vectors in LDS, exactly as the one-walk kernels above do.
template <typename T>
__global__ __launch_bounds__(1024) void k_small_many(const SmallWalk *__restrict__ walks) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[16];
  const SmallWalk &w = walks[blockIdx.x];
  const Readout none;
  if (w.staggered)
    stag_small_walk<T>(w.g, static_cast<T *>(w.psi), w.steps, none, smem, red);
  else if (w.coined)
    coined_small_walk<T>(w.g, static_cast<T *>(w.psi), w.hadamard, w.steps, none, smem, red);
  else
    ctqw_small_walk<T>(w.g, static_cast<T *>(w.psi), w.alpha, w.beta, w.K, w.steps, none, smem, red);
}

// ---- batched launch over many walks -------------------------------------------
// One launch advances every active walk of a batch by one unit: a Horner
// stage (CTQW) or a whole step (coined).  Workgroups grid-stride over a tile
// table; the host places each walk's tiles on indices of one residue mod 8, so
// with a grid that is a multiple of 8 all of a walk's tiles run on the same
// XCD (workgroups are dispatched round-robin over the 8 XCDs) and its gathers
// stay in that XCD's L2.
template <typename T>
__device__ void batch_ctqw_tile(const WalkSlot &w, const TileEntry &te, int64_t u) {
  const int K = w.K;
  const int64_t step = u / K;
  const int k = K - static_cast<int>(u % K);
  const T *psi = static_cast<const T *>(w.psi);
  const T *yin = (k == K) ? psi : static_cast<const T *>(((K - k - 1) & 1) ? w.w1 : w.w0);
  T *yout = (k == 1) ? static_cast<T *>(w.psi) : static_cast<T *>(((K - k) & 1) ? w.w1 : w.w0);
  const double alpha = w.alpha[k - 1], beta = w.beta[k - 1];
  if (w.ell_d > 0 && w.ell_d <= 8) {
    // regular graph: two rows per lane, every index load and then every gather
    // of both rows issued before the first add (row r1 clamped to a valid row
    // when it is past the tile; its result is then discarded).  Memory is
    // reached through global views of the slot's pointers (global, not flat,
    // instructions).
    const int d = w.ell_d, n = w.n;
    const gptr<int32_t> col = as_global(w.col);
    const gptr<uint32_t> bits = as_global(w.markbits);
    const gptr<T> gpsi = as_global(psi), gyin = as_global(yin);
    const gmut<T> gyout = as_global_mut(yout);
    for (int r0 = te.begin + threadIdx.x; r0 < te.end; r0 += 2 * blockDim.x) {
      const int r1raw = r0 + blockDim.x;
      const bool h1 = r1raw < te.end;
      const int r1 = h1 ? r1raw : r0;
      int c0[8], c1[8];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (j < d) {
          c0[j] = col[static_cast<int64_t>(j) * n + r0];
          c1[j] = col[static_cast<int64_t>(j) * n + r1];
        }
      const T p0 = gld(gpsi, r0), p1 = gld(gpsi, r1);
      const T s0v = gld(gyin, r0), s1v = gld(gyin, r1);
      const uint32_t mw0 = bits[r0 >> 5], mw1 = bits[r1 >> 5];
      T x0[8], x1[8];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (j < d) {
          x0[j] = gld(gyin, c0[j]);
          x1[j] = gld(gyin, c1[j]);
        }
      double2 s0 = make_double2(0.0, 0.0), s1 = make_double2(0.0, 0.0);
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (j < d) {
          s0 = add(s0, cvt(x0[j]));
          s1 = add(s1, cvt(x1[j]));
        }
      const bool m0 = (mw0 >> (r0 & 31)) & 1u, m1 = (mw1 >> (r1 & 31)) & 1u;
      const double2 yv0 = m0 ? cvt(s0v) : make_double2(0.0, 0.0);
      const double2 yv1 = m1 ? cvt(s1v) : make_double2(0.0, 0.0);
      const T o0 = pack<T>(horner_out(cvt(p0), s0, yv0, m0, alpha, beta));
      const T o1 = pack<T>(horner_out(cvt(p1), s1, yv1, m1, alpha, beta));
      gst(gyout, r0, o0);
      if (h1) gst(gyout, r1, o1);
      if (k == 1 && w.hist) {
        if (m0) atomicAdd(&w.hist[step], abs2(cvt(o0)));
        if (h1 && m1) atomicAdd(&w.hist[step], abs2(cvt(o1)));
      }
    }
    return;
  }
  for (int row = te.begin + threadIdx.x; row < te.end; row += blockDim.x) {
    const double2 sum = w.ell_d > 0 ? ell_gather_sum(yin, w.col, w.n, w.ell_d, row)
                                    : gather_sum(yin, w.col, w.rp[row], w.rp[row + 1]);
    const bool mk = marked(w.markbits, row);
    const double2 yv = mk ? ld(yin, row) : make_double2(0.0, 0.0);
    const double2 r = horner_out(ld(psi, row), sum, yv, mk, alpha, beta);
    const T stored = pack<T>(r);
    yout[row] = stored;
    if (k == 1 && mk && w.hist) atomicAdd(&w.hist[step], abs2(cvt(stored)));
  }
}

template <typename T>
__device__ void batch_coined_tile(const WalkSlot &w, const TileEntry &te, int64_t u, T *s) {
  const T *in = static_cast<const T *>((u & 1) ? w.w0 : w.psi);
  T *out = static_cast<T *>((u & 1) ? w.psi : w.w0);
  const int vb = te.begin, ve = te.end;
  const int ab = w.rp[vb], ae = w.rp[ve];
  const int na = ae - ab;
  // tiles of batched coined walks always fit the LDS tile (built from the
  // plan's tiles; single-vertex tiles above kTileArcs are refused on the host)
  for (int i = threadIdx.x; i < na; i += blockDim.x) s[i] = in[ab + i];
  __syncthreads();
  for (int v = vb + threadIdx.x; v < ve; v += blockDim.x) {
    const int lo = w.rp[v] - ab, hi = w.rp[v + 1] - ab, d = hi - lo;
    if (d == 0) continue;
    if (marked(w.markbits, v)) {
      for (int i = lo; i < hi; ++i) s[i] = pack<T>(scale(cvt(s[i]), -1.0));
    } else if (w.hadamard) {
      double2 x0 = cvt(s[lo]), x1 = cvt(s[lo + 1]);
      s[lo] = pack<T>(scale(add(x0, x1), kInvSqrt2));
      s[lo + 1] = pack<T>(scale(sub(x0, x1), kInvSqrt2));
    } else {
      double2 sum = make_double2(0.0, 0.0);
      for (int i = lo; i < hi; ++i) sum = add(sum, cvt(s[i]));
      double2 m = grover_mean(sum, d);
      for (int i = lo; i < hi; ++i) s[i] = pack<T>(sub(add(m, m), cvt(s[i])));
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < na; i += blockDim.x) out[w.rev[ab + i]] = s[i];
}

// Structured coined walks of a batch: slot-major state ping-ponging between
// w0 (even units) and w1; one thread per vertex of the tile, the same
// arithmetic as k_coined_struct.
template <typename T, int KIND, int D>
__device__ __forceinline__ void batch_struct_vertices(const WalkSlot &w, const TileEntry &te, int64_t u) {
  const T *in = static_cast<const T *>((u & 1) ? w.w1 : w.w0);
  T *out = static_cast<T *>((u & 1) ? w.w0 : w.w1);
  const int n = w.n, l2 = w.sdims[1];
  const int d = (KIND == kHypercube) ? w.sdims[0] : D;
  for (int v = te.begin + threadIdx.x; v < te.end; v += blockDim.x) {
    T x[D];
#pragma unroll
    for (int j = 0; j < D; ++j)
      if (j < d) x[j] = in[static_cast<int64_t>(j) * n + v];
    if (marked(w.markbits, v)) {
#pragma unroll
      for (int j = 0; j < D; ++j)
        if (j < d) x[j] = pack<T>(scale(cvt(x[j]), -1.0));
    } else if (KIND == kCycle && w.hadamard) {
      const double2 x0 = cvt(x[0]), x1 = cvt(x[1]);
      x[0] = pack<T>(scale(add(x0, x1), kInvSqrt2));
      x[1] = pack<T>(scale(sub(x0, x1), kInvSqrt2));
    } else {
      double2 sum = make_double2(0.0, 0.0);
#pragma unroll
      for (int j = 0; j < D; ++j)
        if (j < d) sum = add(sum, cvt(x[j]));
      const double2 m = grover_mean(sum, d);
#pragma unroll
      for (int j = 0; j < D; ++j)
        if (j < d) x[j] = pack<T>(sub(add(m, m), cvt(x[j])));
    }
#pragma unroll
    for (int j = 0; j < D; ++j)
      if (j < d) out[static_cast<int64_t>(rev_slot<KIND>(j)) * n + head_of<KIND>(v, j, n, l2)] = x[j];
  }
}

template <typename T>
__global__ __launch_bounds__(kTileThreads) void k_batch_struct(const BatchCtl *ctl, const WalkSlot *slots,
                                                               const TileEntry *tiles, const int32_t *n_tiles) {
  const int64_t L = static_cast<int64_t>(ctl->L);
  const int nt = *n_tiles;
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    const TileEntry te = tiles[t];
    if (te.slot < 0) continue;
    const WalkSlot &w = slots[te.slot];
    if (w.kind != 0 || w.structure == kGeneral) continue;
    const int64_t u = L - w.L0;
    if (u < 0 || u >= w.units) continue;
    switch (w.structure) {
      case kCycle: batch_struct_vertices<T, kCycle, 2>(w, te, u); break;
      case kTorus: batch_struct_vertices<T, kTorus, 4>(w, te, u); break;
      default:
        if (w.sdims[0] <= 16) batch_struct_vertices<T, kHypercube, 16>(w, te, u);
        else batch_struct_vertices<T, kHypercube, 32>(w, te, u);
        break;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kTileThreads) void k_batch_stage(BatchCtl *ctl, const WalkSlot *slots,
                                                              const TileEntry *tiles,
                                                              const int32_t *n_tiles, int advance) {
  __shared__ T s[kTileArcs];
  const int64_t L = static_cast<int64_t>(ctl->L);
  const bool probe = ctl->probe != 0;
  const int nt = *n_tiles;
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    const TileEntry te = tiles[t];
    if (te.slot < 0) continue;
    const WalkSlot &w = slots[te.slot];
    if (w.kind < 0) continue;
    const int64_t u = probe ? 0 : L - w.L0;
    if (u < 0 || u >= w.units) continue;
    if (w.kind == 1) {
      batch_ctqw_tile<T>(w, te, u);
    } else if (w.structure == kGeneral) {
      batch_coined_tile<T>(w, te, u, s);
    } else {
      continue;  // structured coined tiles belong to k_batch_struct
    }
    __syncthreads();
  }
  if (probe || !advance) return;
  // Launch ticket: the last workgroup to finish advances L.  Only atomicity
  // is needed -- every workgroup read L before taking its ticket, and the next
  // launch reads it after the kernel boundary -- so no fence is issued (an
  // agent-scope fence would write back the L2 once per workgroup).
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned int prev = atomicAdd(&ctl->done, 1u);
    if (prev == gridDim.x - 1) {
      atomicExch(&ctl->done, 0u);
      atomicAdd(&ctl->L, 1ull);
    }
  }
}

// LDS-staged Horner stage for the batch's CTQW walks on regular graphs of
// degree <= 8 (ELL layout).  A workgroup owns NT * RPL consecutive rows of one
// walk (a tile) and makes one pass over the walk's input vector y in blocks of
// BLK entries held in LDS, so every neighbour value is read from LDS in the
// block that holds it and the random gathers never reach L2; the vector (at
// most a few MB) stays in the XCD's L2 while the walk's tiles read it.  Rows
// keep their neighbour indices in registers.  The plan stores each row's
// neighbours in increasing order, so adding, block after block, the
// neighbours each block holds adds them in row order: the sums are bitwise
// those of the gather kernels.  Blocks are staged by LDS-direct loads
// (global_load_lds_dwordx4: each lane's 16 bytes land at the wave's LDS base
// plus 16 * lane, 1 KiB per wave instruction), which need no registers and no
// LDS write instructions; the registers that a prefetch would hold carry more
// rows per thread (complex64: 9 of 768 threads; complex128: 6 of 1024; the
// register-prefetching form fitted 4), so a walk has fewer tiles to pass over
// its vector.  Every lane visits all 8 neighbour slots of its rows in
// every block (branch-free; a slot outside the block adds -0), so the sum loop
// costs 8 LDS reads per row and block: the kernel pays for walks whose vector
// spans many blocks.  Memory is reached through global-address-space views of
// the slot table's pointers, and every load is unconditional (indices clamped
// into range, unused values dropped by a select).  Tiles are taken
// grid-stride (the host lays out the table by XCD); the last workgroup of the
// launch advances the launch counter when `advance` is set.  The host sends
// only walks whose state holds at least 16 bytes and whose psi and work
// buffers are 16-byte aligned.
template <typename T, int NT, int RPL, int BLK>
__global__ __launch_bounds__(NT) void k_batch_ell_lds(BatchCtl *ctl, const WalkSlot *slots,
                                                      const TileEntry *tiles, const int32_t *n_tiles,
                                                      int advance) {
  constexpr int kWaves = NT / 64;
  constexpr int EPL = 16 / static_cast<int>(sizeof(T));  // entries per lane of one direct load
  constexpr int EPW = 64 * EPL;                           // entries per wave load (1 KiB)
  static_assert(NT % 64 == 0 && BLK % (kWaves * EPW) == 0, "a block is whole rounds of wave loads");
  constexpr int LPW = BLK / (kWaves * EPW);  // direct loads per wave and block
  constexpr unsigned kPadByte = static_cast<unsigned>(BLK) * static_cast<unsigned>(sizeof(T));
  // xs[BLK] is a pad entry holding (-0, -0): a neighbour outside the current
  // block reads it, and adding -0 leaves every value (either zero included)
  // bit for bit unchanged, so the sum loop has no branch
  __shared__ __attribute__((aligned(16))) T xs[BLK + 1];
  if (threadIdx.x == 0) {
    xs[BLK].x = -0.0;
    xs[BLK].y = -0.0;
  }
  const int64_t L = static_cast<int64_t>(ctl->L);
  const bool probe = ctl->probe != 0;
  const int nt = *n_tiles;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    const TileEntry te = tiles[t];
    if (te.slot < 0) continue;
    const WalkSlot &w = slots[te.slot];
    if (w.kind != 1 || w.ell_d <= 0 || w.ell_d > 8 || w.n < EPL) continue;
    const int64_t u = probe ? 0 : L - w.L0;
    if (u < 0 || u >= w.units) continue;
    const int K = w.K;
    const int64_t step = u / K;
    const int k = K - static_cast<int>(u % K);
    const T *yin_p = (k == K) ? static_cast<const T *>(w.psi) : static_cast<const T *>(((K - k - 1) & 1) ? w.w1 : w.w0);
    const gptr<T> psi = as_global(static_cast<const T *>(w.psi));
    const gptr<T> yin = as_global(yin_p);
    const gmut<T> yout = as_global_mut(static_cast<T *>((k == 1) ? w.psi : (((K - k) & 1) ? w.w1 : w.w0)));
    const gptr<int32_t> col = as_global(w.col);
    const gptr<uint32_t> bits = as_global(w.markbits);
    const double alpha = as_global(w.alpha)[k - 1], beta = as_global(w.beta)[k - 1];
    const int n = w.n, d = w.ell_d;
    // the last whole group of EPL entries: a lane whose group runs past the
    // vector loads it instead (those LDS entries are never read, but for n-1
    // when n is odd in complex64, written in place below)
    const int last_group = (n - EPL) / EPL * EPL;
    // neighbour indices of this lane's rows; missing neighbours and rows past the
    // tile (their loads read a valid entry) become the pad offset below.
    int c[RPL][8];
    double2 acc[RPL];
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int r = te.begin + tid + i * NT;
      const int rc = r < te.end ? r : te.end - 1;
#pragma unroll
      for (int j = 0; j < 8; ++j) c[i][j] = col[static_cast<int64_t>(j < d ? j : d - 1) * n + rc];
      acc[i] = make_double2(0.0, 0.0);
    }
    // held as byte offsets into the vector (the host keeps n * sizeof(T) below 2^31);
    // a pad is 0xffffffff, whose offset from any block start (below 2^31) is at
    // least 2^31 and so always clamps to the pad entry
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const bool ok = te.begin + tid + i * NT < te.end;
#pragma unroll
      for (int j = 0; j < 8; ++j) c[i][j] = (ok && j < d) ? c[i][j] * static_cast<int>(sizeof(T)) : -1;
    }
    for (int base = 0; base < n; base += BLK) {
      __syncthreads();  // the previous block (or tile) is no longer read
#pragma unroll
      for (int e = 0; e < LPW; ++e) {
        const int lbase = (e * kWaves + wave) * EPW;  // first entry of this wave load
        const int idx = base + lbase + EPL * lane;
        const int src = idx + EPL <= n ? idx : last_group;
        __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1))) *)(yin_p + src),
                                         (void __attribute__((address_space(3))) *)(xs + lbase), 16, 0, 0);
      }
      __syncthreads();  // the direct loads have landed (the barrier waits for them)
      if constexpr (EPL == 2) {
        // odd n: entry n-1 sits in a group that runs past the vector
        if ((n & 1) && n - 1 >= base && n - 1 < base + BLK) {
          if (tid == 0) xs[n - 1 - base] = gld(yin, n - 1);
          __syncthreads();
        }
      }
      // four LDS reads in flight per group, then their adds in neighbour order;
      // a byte offset outside the block (below it, it wraps) clamps to the pad
      const unsigned base_b = static_cast<unsigned>(base) * static_cast<unsigned>(sizeof(T));
      const char *xs_b = reinterpret_cast<const char *>(xs);
#pragma unroll
      for (int i = 0; i < RPL; ++i)
#pragma unroll
        for (int h = 0; h < 8; h += 4) {
          T xv[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const unsigned off = min(static_cast<unsigned>(c[i][h + j]) - base_b, kPadByte);
            xv[j] = *reinterpret_cast<const T *>(xs_b + off);
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i] = add(acc[i], cvt(xv[j]));
        }
    }
    T pv[RPL], yv[RPL];
    uint32_t mw[RPL];
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int r = te.begin + tid + i * NT;
      const int rc = r < te.end ? r : te.end - 1;
      pv[i] = gld(psi, rc);
      yv[i] = gld(yin, rc);
      mw[i] = bits[rc >> 5];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int r = te.begin + tid + i * NT;
      const int rc = r < te.end ? r : te.end - 1;
      const bool mk = (mw[i] >> (rc & 31)) & 1u;
      const double2 y_self = mk ? cvt(yv[i]) : make_double2(0.0, 0.0);
      const T o = pack<T>(horner_out(cvt(pv[i]), acc[i], y_self, mk, alpha, beta));
      if (r < te.end) {
        gst(yout, r, o);
        if (k == 1 && mk && w.hist) atomicAdd(&w.hist[step], abs2(cvt(o)));
      }
    }
  }
  if (probe || !advance) return;
  // launch ticket, as in k_batch_stage
  __syncthreads();
  if (tid == 0) {
    const unsigned int prev = atomicAdd(&ctl->done, 1u);
    if (prev == gridDim.x - 1) {
      atomicExch(&ctl->done, 0u);
      atomicAdd(&ctl->L, 1ull);
    }
  }
}

// ---- snapshots: device memory straight into pinned host memory ------------------
// A grid-stride copy whose stores cross the link as the kernel issues them
// (no copy engine): 16-byte vector loads from device memory, non-temporal
// 16-byte stores to the device view of a pinned host buffer, then the last
// bytes % 16 bytes one by one.  Both pointers are 16-byte aligned.
__global__ __launch_bounds__(256) void k_copy_link(const i32x4 *__restrict__ src, i32x4 *__restrict__ dst,
                                                   int64_t n16, const unsigned char *__restrict__ src_tail,
                                                   unsigned char *__restrict__ dst_tail, int tail) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t first = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  for (int64_t i = first; i < n16; i += stride) __builtin_nontemporal_store(src[i], &dst[i]);
  if (first < tail) dst_tail[first] = src_tail[first];
}

// ---- dense H on the matrix cores -------------------------------------------------
// H (n x n real, rows padded to kDenseRows, leading dimension ld) times the
// real view of the state block Y (n x 2C: each complex column b is the real
// columns 2b, 2b+1).  Workgroup = 4 wavefronts, 64 rows of H; each wave owns
// 16 rows and all NT*16 real columns as NT accumulator tiles of the
// 16x16x4 MFMA.  H and Y chunks of KC values of k (16 or 32) are staged in
// LDS.
// Epilogue: with z = (H y)_v = a + i b, y_out = psi + c (b - i a): real
// column 2b takes +c * (its odd partner), column 2b+1 takes -c * (its even
// partner); partners sit in neighbouring lanes.
typedef float mf4 __attribute__((ext_vector_type(4)));
typedef double md4 __attribute__((ext_vector_type(4)));

template <typename R> struct Mfma;
// Result layout of the 16x16x4 forms (lane l, register r, column l % 16):
// the FP64 form holds row l/16 + 4r, the FP32 form row 4(l/16) + r.
template <> struct Mfma<double> {
  using acc = md4;
  static __device__ __forceinline__ int row(int l, int r) { return (l >> 4) + 4 * r; }
  static __device__ __forceinline__ acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<float> {
  using acc = mf4;
  static __device__ __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
  static __device__ __forceinline__ acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

template <typename R, int NT, int KC>
__global__ __launch_bounds__(256) void k_dense_stage(const R *__restrict__ H, int ld, int n, int c2,
                                                     const R *__restrict__ yin, const R *psi, R *out,
                                                     double c, int ksplit, double *partial) {
  using M = Mfma<R>;
  constexpr int NC = NT * 16;
  static_assert(kDenseK % KC == 0 && 256 % KC == 0, "chunks tile the split ranges and the FP32 fold");
  constexpr int HPT = kDenseRows * KC / 256;  // H values each thread stages per chunk
  constexpr int XPT = KC * NC / 256;          // Y values each thread stages per chunk
  constexpr int FOLD = 256 / KC;              // FP32 products fold into FP64 every 256 k
  // double-buffered LDS: chunk c is read from buffer c & 1 while the global
  // loads of chunk c+1 are in flight in registers
  __shared__ R hs[2][kDenseRows][KC + 1];
  __shared__ R xs[2][KC][NC];
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int rblocks = (n + kDenseRows - 1) / kDenseRows;
  const int split = blockIdx.x / rblocks;            // k range of this workgroup
  const int row0 = (blockIdx.x - split * rblocks) * kDenseRows;
  const int kbeg = split * ksplit, kend = min(n, kbeg + ksplit);
  typename M::acc acc[NT];
  double wide[NT][4];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    acc[t] = M::zero();
#pragma unroll
    for (int r = 0; r < 4; ++r) wide[t][r] = 0.0;
  }
  // H is fetched in 16-byte pieces: V consecutive k of one row per load
  constexpr int V = 16 / static_cast<int>(sizeof(R)), PR = KC / V;  // pieces per row of a chunk
  static_assert(HPT % V == 0 && KC % V == 0, "whole 16-byte pieces");
  R hreg[HPT], xreg[XPT];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < HPT / V; ++q) {
      const int e = threadIdx.x + q * 256, i = e / PR, j = (e % PR) * V;
      // rows padded, k0 + j + V <= ld, and ld and k0 multiples of KC keep the piece aligned
      *reinterpret_cast<uint4 *>(hreg + q * V) =
          *reinterpret_cast<const uint4 *>(H + static_cast<int64_t>(row0 + i) * ld + k0 + j);
    }
#pragma unroll
    for (int q = 0; q < XPT; ++q) {
      const int e = threadIdx.x + q * 256, i = e / NC, j = e % NC;
      xreg[q] = (k0 + i < kend && j < c2) ? yin[static_cast<int64_t>(k0 + i) * c2 + j] : R(0);
    }
  };
  if (kbeg < kend) fetch(kbeg);
  int chunk = 0;
  for (int k0 = kbeg; k0 < kend; k0 += KC, ++chunk) {
    const int buf = chunk & 1;
#pragma unroll
    for (int q = 0; q < HPT / V; ++q) {
      const int e = threadIdx.x + q * 256, i = e / PR, j = (e % PR) * V;
#pragma unroll
      for (int t = 0; t < V; ++t) hs[buf][i][j + t] = hreg[q * V + t];
    }
#pragma unroll
    for (int q = 0; q < XPT; ++q) {
      const int e = threadIdx.x + q * 256;
      xs[buf][e / NC][e % NC] = xreg[q];
    }
    // one barrier per chunk: a wave passing it has finished its MMAs of chunk-1, so the
    // buffer written next iteration (chunk+1 & 1 = chunk-1 & 1) is free
    __syncthreads();
    if (k0 + KC < kend) fetch(k0 + KC);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const R a = hs[buf][wave * 16 + (l & 15)][kk + (l >> 4)];
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = M::mma(a, xs[buf][kk + (l >> 4)][t * 16 + (l & 15)], acc[t]);
    }
    if (sizeof(R) == 4 && chunk % FOLD == FOLD - 1) {  // FP32 products: fold into FP64 every 256 k
#pragma unroll
      for (int t = 0; t < NT; ++t) {
#pragma unroll
        for (int r = 0; r < 4; ++r) wide[t][r] += static_cast<double>(acc[t][r]);
        acc[t] = M::zero();
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double z = wide[t][r] + static_cast<double>(acc[t][r]);
      const double zp = __shfl_xor(z, 1, 64);
      const int row = row0 + wave * 16 + M::row(l, r);
      const int col = t * 16 + (l & 15);
      if (partial) {  // split k: hand the raw product to the reduction kernel
        if (row < n && col < c2) partial[(static_cast<int64_t>(split) * n + row) * c2 + col] = z;
        continue;
      }
      if (row < n && col < c2) {
        const int64_t idx = static_cast<int64_t>(row) * c2 + col;
        const double ps = static_cast<double>(psi[idx]);
        out[idx] = static_cast<R>((col & 1) ? ps - c * zp : ps + c * zp);
      }
    }
  }
}

// One walk with FP32 H: H y is bound by streaming H once, so it runs on the
// vector units with FP64 accumulation and no matrix cores (for FP64 H the
// LDS-staged matrix-core kernel streams H slightly faster).  A wavefront owns
// RW rows; lane l reads 16 contiguous bytes of each row per chunk (VEC =
// 16 / sizeof(R) columns; a wavefront's loads of one row are one contiguous
// 1 KiB) and the matching VEC rows of the states (2 B VEC contiguous reals),
// and accumulates z = a + ib per row and walk in a fixed order (chunks in
// sequence, then a butterfly over the lanes).  Then y_out = psi + c (b - i a).
template <typename R, int NB, int RW>
__global__ __launch_bounds__(256) void k_dense_gemv(const R *__restrict__ H, int ld, int n, const R *__restrict__ yin,
                                                    const R *psi, R *out, double c) {
  constexpr int VEC = 16 / static_cast<int>(sizeof(R));
  constexpr int CH = 64 * VEC;      // columns per wavefront chunk
  constexpr int YV = 2 * NB * VEC;  // state reals per lane per chunk
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int row0 = (blockIdx.x * 4 + wave) * RW;
  if (row0 >= n) return;  // whole wavefront
  double za[RW][NB], zb[RW][NB];
  const R *hr[RW];
#pragma unroll
  for (int r = 0; r < RW; ++r) {
#pragma unroll
    for (int b = 0; b < NB; ++b) za[r][b] = zb[r][b] = 0.0;
    hr[r] = H + static_cast<int64_t>(min(row0 + r, n - 1)) * ld;  // rows past n re-read row n-1, unused
  }
  auto chunk = [&](int k, auto guarded_tag) {
    constexpr bool GUARDED = decltype(guarded_tag)::value;
    R yv[YV];  // state rows k .. k+VEC-1: (re, im) of walk b of row k+j at 2 (j NB + b)
    const R *ys = yin + 2 * static_cast<int64_t>(k) * NB;
    if (!GUARDED || k + VEC <= n) {
#pragma unroll
      for (int q = 0; q < YV / VEC; ++q)
        *reinterpret_cast<uint4 *>(yv + q * VEC) = *reinterpret_cast<const uint4 *>(ys + q * VEC);
    } else {  // the lane straddles n: H is zero past n, the states have n rows
#pragma unroll
      for (int j = 0; j < YV; ++j) yv[j] = k + j / (2 * NB) < n ? ys[j] : R(0);
    }
    R h[RW][VEC];
#pragma unroll
    for (int r = 0; r < RW; ++r) *reinterpret_cast<uint4 *>(h[r]) = *reinterpret_cast<const uint4 *>(hr[r] + k);
#pragma unroll
    for (int r = 0; r < RW; ++r) {
#pragma unroll
      for (int j = 0; j < VEC; ++j) {
        const double hv = static_cast<double>(h[r][j]);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          za[r][b] = __fma_rn(hv, static_cast<double>(yv[2 * (j * NB + b)]), za[r][b]);
          zb[r][b] = __fma_rn(hv, static_cast<double>(yv[2 * (j * NB + b) + 1]), zb[r][b]);
        }
      }
    }
  };
  // chunks whose columns all lie below n need no guard; the rest (at most
  // one or two) check each lane against ld and n
  const int kmain = n / CH * CH;
  int k0 = 0;
#pragma unroll 2
  for (; k0 < kmain; k0 += CH) chunk(k0 + l * VEC, std::false_type{});
  for (; k0 < ld; k0 += CH)
    if (k0 + l * VEC < ld) chunk(k0 + l * VEC, std::true_type{});
#pragma unroll
  for (int r = 0; r < RW; ++r)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      za[r][b] = wave_sum(za[r][b]);
      zb[r][b] = wave_sum(zb[r][b]);
    }
  // lane r NB + b writes walk b of row row0 + r
  if (l < RW * NB && row0 + l / NB < n) {
    double a = 0.0, bb = 0.0;
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (l == r * NB + b) {
          a = za[r][b];
          bb = zb[r][b];
        }
    const int64_t e = static_cast<int64_t>(row0) * NB + l;  // complex index (row, walk)
    const double pr = static_cast<double>(psi[2 * e]), pi = static_cast<double>(psi[2 * e + 1]);
    out[2 * e] = static_cast<R>(pr + c * bb);
    out[2 * e + 1] = static_cast<R>(pi - c * a);
  }
}

// Split-k epilogue: z = sum of the partial products in split order (fixed),
// then y_out = psi + c (b - i a) for z = a + i b.  One thread per complex entry.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_dense_reduce(const double *__restrict__ partial, int splits, int n,
                                                         int c2, const R *psi, R *out, double c) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;  // complex index
  const int64_t total = static_cast<int64_t>(n) * (c2 / 2);
  if (e >= total) return;
  double a = 0.0, b = 0.0;
  for (int sp = 0; sp < splits; ++sp) {
    const double *ps = partial + static_cast<int64_t>(sp) * n * c2 + 2 * e;
    a += ps[0];
    b += ps[1];
  }
  const double pr = static_cast<double>(psi[2 * e]), pi = static_cast<double>(psi[2 * e + 1]);
  out[2 * e] = static_cast<R>(pr + c * b);
  out[2 * e + 1] = static_cast<R>(pi - c * a);
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_dense_zero(R *H, int64_t total) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    H[i] = R(0);
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_dense_scatter(GraphView g, R *H, double gamma) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= g.n) return;
  R *row = H + static_cast<int64_t>(v) * g.ld;
  for (int a = g.rp[v]; a < g.rp[v + 1]; ++a) row[g.col[a]] = static_cast<R>(-gamma);
  if (marked(g.markbits, v)) row[v] = R(-1);
}

template <typename R, int NT>
void launch_dense(const GraphView &g, const void *y, const void *psi, void *out, double c, hipStream_t s) {
  const int rblocks = (g.n + kDenseRows - 1) / kDenseRows;
  const int splits = dense_splits(g);
  const int ksplit = ((g.n + splits - 1) / splits + kDenseK - 1) / kDenseK * kDenseK;
  const int used = (g.n + ksplit - 1) / ksplit;  // splits that own at least one k
  const dim3 grid(rblocks * used);
  double *partial = used > 1 ? g.dense_partial : nullptr;
  // 32-k chunks halve the barriers per byte of H where the stage streams H
  // (one 16-column tile) and for FP32 from 64 columns; the FP64 tiles of 32
  // and more columns measured faster with 16 (and with 256 columns 32 would
  // not fit LDS twice)
  constexpr int KC = (NT == 1 || (sizeof(R) == 4 && (NT == 4 || NT == 16))) ? 32 : 16;
  hipLaunchKernelGGL((k_dense_stage<R, NT, KC>), grid, dim3(256), 0, s, static_cast<const R *>(g.dense), g.ld, g.n,
                     2 * g.columns, static_cast<const R *>(y), static_cast<const R *>(psi), static_cast<R *>(out),
                     c, ksplit, partial);
  if (partial) {
    const int64_t total = static_cast<int64_t>(g.n) * g.columns;
    hipLaunchKernelGGL(k_dense_reduce<R>, dim3(blocks_for(total, kBlock)), dim3(kBlock), 0, s, partial, used,
                       g.n, 2 * g.columns, static_cast<const R *>(psi), static_cast<R *>(out), c);
  }
}

template <typename R, int NB, int RW>
void launch_gemv(const GraphView &g, const void *y, const void *psi, void *out, double c, hipStream_t s) {
  const dim3 grid((g.n + 4 * RW - 1) / (4 * RW));
  hipLaunchKernelGGL((k_dense_gemv<R, NB, RW>), grid, dim3(256), 0, s, static_cast<const R *>(g.dense), g.ld, g.n,
                     static_cast<const R *>(y), static_cast<const R *>(psi), static_cast<R *>(out), c);
}

template <typename R>
void launch_dense_nt(const GraphView &g, const void *y, const void *psi, void *out, double c, hipStream_t s) {
  const int c2 = 2 * g.columns;
  // the vector kernel reads 2 B state reals per H element from cache; the
  // LDS-staged matrix-core kernel streams H at a rate that does not depend on
  // B up to 8 walks: for FP64 H it is ahead from B = 1, for FP32 H from B = 2
  if (sizeof(R) == 4 && g.columns == 1) return launch_gemv<R, 1, 4>(g, y, psi, out, c, s);
  if (c2 <= 16) launch_dense<R, 1>(g, y, psi, out, c, s);
  else if (c2 <= 32) launch_dense<R, 2>(g, y, psi, out, c, s);
  else if (c2 <= 64) launch_dense<R, 4>(g, y, psi, out, c, s);
  else if (c2 <= 128) launch_dense<R, 8>(g, y, psi, out, c, s);
  else launch_dense<R, 16>(g, y, psi, out, c, s);
}


// A kernel launched with more than 64 KiB of dynamic LDS must be allowed it
// first (on the current device).
template <typename F> hipError_t allow_lds(F *kernel, size_t lds) {
  if (lds <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             static_cast<int>(kSmallLdsBytes));
}

template <typename T> hipError_t launch_coined_small(const GraphView &g, void *psi, int hadamard,
                                                     int64_t steps, const Readout &ro, hipStream_t s) {
  size_t lds = coined_small_lds(sizeof(T) == 16, g.n, g.n_arcs);
  if (hipError_t e = allow_lds(&k_coined_small<T>, lds); e != hipSuccess) return e;
  int threads = 64;
  while (threads < 1024 && threads < g.n_arcs) threads *= 2;
  hipLaunchKernelGGL(k_coined_small<T>, dim3(1), dim3(threads), lds, s, g, static_cast<T *>(psi),
                     hadamard, steps, ro);
  return hipGetLastError();
}

template <typename T> hipError_t launch_ctqw_small(const GraphView &g, void *psi, const double *alpha,
                                                   const double *beta, int K, int64_t steps,
                                                   const Readout &ro, hipStream_t s) {
  Coefs c;
  for (int k = 0; k < 64; ++k) {
    c.alpha[k] = k < K ? alpha[k] : 0.0;
    c.beta[k] = k < K ? beta[k] : 0.0;
  }
  size_t lds = ctqw_small_lds(sizeof(T) == 16, g.n, g.n_arcs);
  if (hipError_t e = allow_lds(&k_ctqw_small<T>, lds); e != hipSuccess) return e;
  int threads = 64;
  while (threads < 1024 && threads < g.n) threads *= 2;
  hipLaunchKernelGGL(k_ctqw_small<T>, dim3(1), dim3(threads), lds, s, g, static_cast<T *>(psi), c, K,
                     steps, ro);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_small_many(const SmallWalk *d_walks, int count, size_t lds, int threads, hipStream_t s) {
  if (hipError_t e = allow_lds(&k_small_many<T>, lds); e != hipSuccess) return e;
  hipLaunchKernelGGL(k_small_many<T>, dim3(count), dim3(threads), lds, s, d_walks);
  return hipGetLastError();
}

template <typename T, int KIND, int D>
void launch_struct(const GraphView &g, const void *in, void *out, int dim, int hadamard, hipStream_t s) {
  hipLaunchKernelGGL((k_coined_struct<T, KIND, D>), dim3(blocks_for(g.n, kBlock)), dim3(kBlock), 0, s, g,
                     static_cast<const T *>(in), static_cast<T *>(out), dim, hadamard);
}

template <typename T>
hipError_t launch_coined_struct(const GraphView &g, const void *in, void *out, int hadamard, hipStream_t s) {
  switch (g.structure) {
    case kCycle: launch_struct<T, kCycle, 2>(g, in, out, 2, hadamard, s); break;
    case kTorus: launch_struct<T, kTorus, 4>(g, in, out, 4, 0, s); break;
    case kHypercube: {
      const int dim = g.dims[0];
      if (dim <= 8) launch_struct<T, kHypercube, 8>(g, in, out, dim, 0, s);
      else if (dim <= 16) launch_struct<T, kHypercube, 16>(g, in, out, dim, 0, s);
      else if (dim <= 24) launch_struct<T, kHypercube, 24>(g, in, out, dim, 0, s);
      else launch_struct<T, kHypercube, 32>(g, in, out, dim, 0, s);
      break;
    }
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int G, bool PROB>
void launch_csr_g(const GraphView &g, const T *y, const T *psi, T *out, StageCoef c, double *p,
                  double *partials, hipStream_t s) {
  if (!PROB && g.sorted_rows && G <= 16 &&
      static_cast<int64_t>(g.n) * static_cast<int64_t>(sizeof(T)) > kEllSliceFrom) {
    constexpr int GS = G <= 16 ? G : 16;
    const int groups = static_cast<int>(blocks_for(g.n, kBlock / GS));
    const dim3 sgrid(std::min(groups, resident_groups(k_ctqw_csr_sliced<T, GS>)));
    hipLaunchKernelGGL((k_ctqw_csr_sliced<T, GS>), sgrid, dim3(kBlock), 0, s, g, y, psi, out, c.alpha, c.beta,
                       kEllSliceEntries);
    return;
  }
  const int64_t threads = static_cast<int64_t>(g.n) * G;
  hipLaunchKernelGGL((k_ctqw_csr<T, G, PROB>), dim3(blocks_for(threads, kBlock)), dim3(kBlock), 0, s, g, y,
                     psi, out, c.alpha, c.beta, p, partials);
}

template <typename T, bool PROB>
hipError_t launch_ctqw_stage(const GraphView &g, const T *y, const T *psi, T *out, StageCoef c, double *p,
                             double *partials, hipStream_t s) {
  if (g.structure == kGeneral) {
    switch (g.group) {
      case 1: launch_csr_g<T, 1, PROB>(g, y, psi, out, c, p, partials, s); break;
      case 2: launch_csr_g<T, 2, PROB>(g, y, psi, out, c, p, partials, s); break;
      case 4: launch_csr_g<T, 4, PROB>(g, y, psi, out, c, p, partials, s); break;
      case 8: launch_csr_g<T, 8, PROB>(g, y, psi, out, c, p, partials, s); break;
      case 16: launch_csr_g<T, 16, PROB>(g, y, psi, out, c, p, partials, s); break;
      case 32: launch_csr_g<T, 32, PROB>(g, y, psi, out, c, p, partials, s); break;
      default: launch_csr_g<T, 64, PROB>(g, y, psi, out, c, p, partials, s); break;
    }
  } else {
    const dim3 grid(blocks_for(g.n, kBlock));
    switch (g.structure) {
      case kCycle:
        hipLaunchKernelGGL((k_ctqw_struct<T, kCycle, PROB>), grid, dim3(kBlock), 0, s, g, y, psi, out,
                           c.alpha, c.beta, p, partials);
        break;
      case kTorus:
        hipLaunchKernelGGL((k_ctqw_struct<T, kTorus, PROB>), grid, dim3(kBlock), 0, s, g, y, psi, out,
                           c.alpha, c.beta, p, partials);
        break;
      case kHypercube:
        hipLaunchKernelGGL((k_ctqw_struct<T, kHypercube, PROB>), grid, dim3(kBlock), 0, s, g, y, psi,
                           out, c.alpha, c.beta, p, partials);
        break;
      case kEll:
        if (!PROB && g.ell_d <= 8 && static_cast<int64_t>(g.n) * static_cast<int64_t>(sizeof(T)) > kEllSliceFrom) {
          constexpr int RPT = kEllSliceRows;
          const int groups = static_cast<int>(blocks_for(g.n, kBlock * RPT));
          const dim3 sgrid(std::min(groups, resident_groups(k_ctqw_ell_sliced<T, RPT>)));
          hipLaunchKernelGGL((k_ctqw_ell_sliced<T, RPT>), sgrid, dim3(kBlock), 0, s, g, y, psi, out, c.alpha, c.beta,
                             kEllSliceEntries);
        } else {
          hipLaunchKernelGGL((k_ctqw_ell<T, PROB>), grid, dim3(kBlock), 0, s, g, y, psi, out, c.alpha, c.beta, p,
                             partials);
        }
        break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

template <typename T> hipError_t launch_stag_small(const GraphView &g, void *psi, int64_t steps, const Readout &ro,
                                                   hipStream_t s) {
  const size_t lds = stag_small_lds(sizeof(T) == 16, g.n);
  if (hipError_t e = allow_lds(&k_stag_small<T>, lds); e != hipSuccess) return e;
  int threads = 64;
  while (threads < 1024 && threads < g.n) threads *= 2;
  hipLaunchKernelGGL(k_stag_small<T>, dim3(1), dim3(threads), lds, s, g, static_cast<T *>(psi), steps, ro);
  return hipGetLastError();
}

template <typename T, int MAXS>
void launch_stag_poly(const GraphView &g, const StagTess &t, T *psi, int mark, hipStream_t s) {
  const dim3 grid(blocks_for(t.n_small, kBlock));
  if (t.small_size > 0)
    hipLaunchKernelGGL((k_stag_poly<T, MAXS, true>), grid, dim3(kBlock), 0, s, g.base, t, psi, g.markbits, mark);
  else
    hipLaunchKernelGGL((k_stag_poly<T, MAXS, false>), grid, dim3(kBlock), 0, s, g.base, t, psi, g.markbits, mark);
}

template <typename T>
hipError_t launch_stag_tess(const GraphView &g, const StagTess &t, void *psi_v, bool mark, double *partials,
                            hipStream_t s) {
  T *psi = static_cast<T *>(psi_v);
  const int mk = mark ? 1 : 0;
  if (t.n_small > 0) {
    if (t.max_small <= 2) launch_stag_poly<T, 2>(g, t, psi, mk, s);
    else if (t.max_small <= 4) launch_stag_poly<T, 4>(g, t, psi, mk, s);
    else if (t.max_small <= 8) launch_stag_poly<T, 8>(g, t, psi, mk, s);
    else launch_stag_poly<T, kStagThreadMax>(g, t, psi, mk, s);
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  }
  if (t.n_chunks > 0) {
    auto *part = reinterpret_cast<double2 *>(partials);
    hipLaunchKernelGGL(k_stag_big_partial<T>, dim3(t.n_chunks), dim3(kBlock), 0, s, g.base, t,
                       static_cast<const T *>(psi), g.markbits, mk, part);
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
    hipLaunchKernelGGL(k_stag_big_apply<T>, dim3(t.n_chunks), dim3(kBlock), 0, s, g.base, t, psi, g.markbits, mk,
                       static_cast<const double2 *>(part));
  }
  return hipGetLastError();
}

}  // namespace

// ============================ launchers ======================================

// LDS of the one-workgroup kernels: vectors, row pointers, reverse arcs or
// columns, and the marked bitmap.
size_t coined_small_lds(bool c128, int n, int n_arcs) {
  const size_t es = c128 ? 16 : 8;
  return 2 * es * static_cast<size_t>(n_arcs) + 4 * (static_cast<size_t>(n) + 1 + n_arcs) +
         4 * ((static_cast<size_t>(n) + 31) / 32);
}

size_t ctqw_small_lds(bool c128, int n, int n_arcs) {
  const size_t es = c128 ? 16 : 8;
  return 3 * es * static_cast<size_t>(n) + 4 * (static_cast<size_t>(n) + 1 + n_arcs) +
         4 * ((static_cast<size_t>(n) + 31) / 32);
}

template <typename T, bool REFL>
void launch_stag_lattice(const GraphView &g, int steps, dim3 grid, const void *in, void *out, double2 c0a,
                         double2 c1a, double2 c0b, double2 c1b, hipStream_t s) {
  const T *x = static_cast<const T *>(in);
  T *y = static_cast<T *>(out);
  if (steps == 2)
    hipLaunchKernelGGL((k_stag_lattice_p<T, REFL, 2>), grid, dim3(256), 0, s, g, x, y, c0a, c1a, c0b, c1b);
  else
    hipLaunchKernelGGL((k_stag_lattice<T, REFL>), grid, dim3(256), 0, s, g, x, y, c0a, c1a, c0b, c1b);
}

hipError_t stag_lattice_step(bool c128, const GraphView &g, const StagTess &ta, const StagTess &tb, int steps,
                             const void *in, void *out, hipStream_t s) {
  if (steps != 1 && steps != 2) return hipErrorInvalidValue;
  const int l1 = g.dims[0], l2 = g.dims[1];
  const dim3 grid(static_cast<unsigned>(((l1 + kLatRows - 1) / kLatRows) * ((l2 + kLatCols - 1) / kLatCols)));
  const double2 c0a = make_double2(ta.c0[0], ta.c0[1]), c1a = make_double2(ta.c1[0], ta.c1[1]);
  const double2 c0b = make_double2(tb.c0[0], tb.c0[1]), c1b = make_double2(tb.c1[0], tb.c1[1]);
  const bool refl = ta.c0[0] == 0.0 && ta.c0[1] == 0.0 && ta.c1[0] == 1.0 && ta.c1[1] == 0.0 && tb.c0[0] == 0.0 &&
                    tb.c0[1] == 0.0 && tb.c1[0] == 1.0 && tb.c1[1] == 0.0;
  if (c128 && refl) launch_stag_lattice<double2, true>(g, steps, grid, in, out, c0a, c1a, c0b, c1b, s);
  else if (c128) launch_stag_lattice<double2, false>(g, steps, grid, in, out, c0a, c1a, c0b, c1b, s);
  else if (refl) launch_stag_lattice<float2, true>(g, steps, grid, in, out, c0a, c1a, c0b, c1b, s);
  else launch_stag_lattice<float2, false>(g, steps, grid, in, out, c0a, c1a, c0b, c1b, s);
  return hipGetLastError();
}

size_t stag_small_lds(bool c128, int n) { return (c128 ? 16 : 8) * static_cast<size_t>(n); }

hipError_t stag_small(bool c128, const GraphView &g, void *psi, int64_t steps, const Readout &ro, hipStream_t s) {
  return c128 ? launch_stag_small<double2>(g, psi, steps, ro, s) : launch_stag_small<float2>(g, psi, steps, ro, s);
}

hipError_t stag_tess(bool c128, const GraphView &g, const StagTess &t, void *psi, bool mark, double *partials,
                     hipStream_t s) {
  return c128 ? launch_stag_tess<double2>(g, t, psi, mark, partials, s)
              : launch_stag_tess<float2>(g, t, psi, mark, partials, s);
}

hipError_t small_many(bool c128, const SmallWalk *d_walks, int count, size_t lds, int threads, hipStream_t s) {
  if (count == 0) return hipSuccess;
  return c128 ? launch_small_many<double2>(d_walks, count, lds, threads, s)
              : launch_small_many<float2>(d_walks, count, lds, threads, s);
}

hipError_t coined_small(bool c128, const GraphView &g, void *psi, int hadamard, int64_t steps,
                        const Readout &ro, hipStream_t s) {
  return c128 ? launch_coined_small<double2>(g, psi, hadamard, steps, ro, s)
              : launch_coined_small<float2>(g, psi, hadamard, steps, ro, s);
}

hipError_t coined_tile_step(bool c128, const GraphView &g, const void *in, void *out, int hadamard,
                            hipStream_t s) {
  if (g.n_tiles == 0) return hipSuccess;
  if (c128)
    hipLaunchKernelGGL(k_coined_tile<double2>, dim3(g.n_tiles), dim3(kTileThreads), 0, s, g,
                       static_cast<const double2 *>(in), static_cast<double2 *>(out), hadamard);
  else
    hipLaunchKernelGGL(k_coined_tile<float2>, dim3(g.n_tiles), dim3(kTileThreads), 0, s, g,
                       static_cast<const float2 *>(in), static_cast<float2 *>(out), hadamard);
  return hipGetLastError();
}

hipError_t coined_struct_step(bool c128, const GraphView &g, const void *in, void *out, int hadamard,
                              hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  return c128 ? launch_coined_struct<double2>(g, in, out, hadamard, s)
              : launch_coined_struct<float2>(g, in, out, hadamard, s);
}

hipError_t coined_perm_in(bool c128, const GraphView &g, const void *psi, void *internal, hipStream_t s) {
  if (g.n_arcs == 0) return hipSuccess;
  const dim3 grid(blocks_for(g.n_arcs, kBlock));
  if (c128)
    hipLaunchKernelGGL(k_perm_in<double2>, grid, dim3(kBlock), 0, s, static_cast<const double2 *>(psi),
                       static_cast<double2 *>(internal), g.perm, g.n_arcs);
  else
    hipLaunchKernelGGL(k_perm_in<float2>, grid, dim3(kBlock), 0, s, static_cast<const float2 *>(psi),
                       static_cast<float2 *>(internal), g.perm, g.n_arcs);
  return hipGetLastError();
}

hipError_t coined_perm_out(bool c128, const GraphView &g, const void *internal, void *psi,
                           const Readout &ro, hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  const int d = g.n > 0 ? g.n_arcs / g.n : 0;
  const dim3 grid(blocks_for(g.n, kBlock));
  double *p = ro.any() ? ro.p_out() : nullptr;
  double *partials = ro.any() ? ro.partials : nullptr;
  if (c128)
    hipLaunchKernelGGL(k_perm_out<double2>, grid, dim3(kBlock), 0, s,
                       static_cast<const double2 *>(internal), static_cast<double2 *>(psi), g.perm, g.n, d,
                       p, partials);
  else
    hipLaunchKernelGGL(k_perm_out<float2>, grid, dim3(kBlock), 0, s, static_cast<const float2 *>(internal),
                       static_cast<float2 *>(psi), g.perm, g.n, d, p, partials);
  return hipGetLastError();
}

hipError_t copy_state(bool c128, int64_t len, const void *in, void *out, hipStream_t s) {
  if (len == 0) return hipSuccess;
  const dim3 grid(blocks_for(len, kBlock));
  if (c128)
    hipLaunchKernelGGL(k_copy<double2>, grid, dim3(kBlock), 0, s, static_cast<const double2 *>(in),
                       static_cast<double2 *>(out), len);
  else
    hipLaunchKernelGGL(k_copy<float2>, grid, dim3(kBlock), 0, s, static_cast<const float2 *>(in),
                       static_cast<float2 *>(out), len);
  return hipGetLastError();
}

int readout_partials(const GraphView &g) {
  return blocks_for(g.structure == kDense ? static_cast<int64_t>(g.n) * g.columns : g.n, kBlock);
}

int ctqw_stage_partials(const GraphView &g) {
  const int64_t lanes = g.structure == kGeneral ? static_cast<int64_t>(g.n) * g.group : g.n;
  return blocks_for(lanes, kBlock);
}

hipError_t coined_prob_csr(bool c128, const GraphView &g, const void *psi, const Readout &ro,
                           hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  const dim3 grid(blocks_for(g.n, kBlock));
  if (c128)
    hipLaunchKernelGGL(k_prob_csr<double2>, grid, dim3(kBlock), 0, s, g, static_cast<const double2 *>(psi),
                       ro.p_out(), ro.partials);
  else
    hipLaunchKernelGGL(k_prob_csr<float2>, grid, dim3(kBlock), 0, s, g, static_cast<const float2 *>(psi),
                       ro.p_out(), ro.partials);
  return hipGetLastError();
}

hipError_t ctqw_small(bool c128, const GraphView &g, void *psi, const double *alpha, const double *beta,
                      int K, int64_t steps, const Readout &ro, hipStream_t s) {
  return c128 ? launch_ctqw_small<double2>(g, psi, alpha, beta, K, steps, ro, s)
              : launch_ctqw_small<float2>(g, psi, alpha, beta, K, steps, ro, s);
}

hipError_t ctqw_stage(bool c128, const GraphView &g, const void *y, const void *psi, void *out, StageCoef c,
                      const Readout *fused, hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  if (c128) {
    auto *yy = static_cast<const double2 *>(y);
    auto *pp = static_cast<const double2 *>(psi);
    auto *oo = static_cast<double2 *>(out);
    return fused ? launch_ctqw_stage<double2, true>(g, yy, pp, oo, c, fused->p_out(), fused->partials, s)
                 : launch_ctqw_stage<double2, false>(g, yy, pp, oo, c, nullptr, nullptr, s);
  }
  auto *yy = static_cast<const float2 *>(y);
  auto *pp = static_cast<const float2 *>(psi);
  auto *oo = static_cast<float2 *>(out);
  return fused ? launch_ctqw_stage<float2, true>(g, yy, pp, oo, c, fused->p_out(), fused->partials, s)
               : launch_ctqw_stage<float2, false>(g, yy, pp, oo, c, nullptr, nullptr, s);
}

hipError_t vertex_prob(bool c128, const GraphView &g, const void *psi, const Readout &ro, hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  const int len = g.structure == kDense ? g.n * g.columns : g.n;
  const dim3 grid(blocks_for(len, kBlock));
  if (c128)
    hipLaunchKernelGGL(k_prob_vertex<double2>, grid, dim3(kBlock), 0, s, static_cast<const double2 *>(psi),
                       len, ro.p_out(), ro.partials);
  else
    hipLaunchKernelGGL(k_prob_vertex<float2>, grid, dim3(kBlock), 0, s, static_cast<const float2 *>(psi),
                       len, ro.p_out(), ro.partials);
  return hipGetLastError();
}

hipError_t batch_stage(bool c128, BatchCtl *ctl, const WalkSlot *slots, const TileEntry *tiles,
                       const int32_t *n_tiles, int grid, int advance, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (c128)
    hipLaunchKernelGGL(k_batch_stage<double2>, dim3(grid), dim3(kTileThreads), 0, s, ctl, slots, tiles, n_tiles,
                       advance);
  else
    hipLaunchKernelGGL(k_batch_stage<float2>, dim3(grid), dim3(kTileThreads), 0, s, ctl, slots, tiles, n_tiles,
                       advance);
  return hipGetLastError();
}

hipError_t ctqw_slot_stage(bool c128, const GraphView &g, const int32_t *slot, int64_t arc0, int r0, int r1,
                           const void *y, const void *psi, void *out, double alpha, double beta, hipStream_t s) {
  if (r1 <= r0) return hipSuccess;
  const dim3 grid(blocks_for(r1 - r0, kBlock));
  if (c128)
    hipLaunchKernelGGL(k_ctqw_csr_slot<double2>, grid, dim3(kBlock), 0, s, g.rp, slot, arc0, r0, r1, g.markbits,
                       static_cast<const double2 *>(y), static_cast<const double2 *>(psi),
                       static_cast<double2 *>(out), alpha, beta);
  else
    hipLaunchKernelGGL(k_ctqw_csr_slot<float2>, grid, dim3(kBlock), 0, s, g.rp, slot, arc0, r0, r1, g.markbits,
                       static_cast<const float2 *>(y), static_cast<const float2 *>(psi),
                       static_cast<float2 *>(out), alpha, beta);
  return hipGetLastError();
}

hipError_t copy_link(void *dst, const void *src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  const int64_t n16 = static_cast<int64_t>(bytes / 16);
  const int tail = static_cast<int>(bytes % 16);
  const int grid = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(kLinkCopyGroups, (n16 + 255) / 256)));
  hipLaunchKernelGGL(k_copy_link, dim3(grid), dim3(256), 0, s, static_cast<const i32x4 *>(src),
                     static_cast<i32x4 *>(dst), n16, static_cast<const unsigned char *>(src) + 16 * n16,
                     static_cast<unsigned char *>(dst) + 16 * n16, tail);
  return hipGetLastError();
}

hipError_t ctqw_direct_stage(bool c128, const GraphView &g, const int32_t *wg_row, int64_t n_wg, const int32_t *dcol,
                             const int32_t *hcol, int64_t split, const void *y, const void *psi, void *out,
                             double alpha, double beta, hipStream_t s) {
  if (n_wg <= 0) return hipSuccess;
  const dim3 grid(static_cast<unsigned>(n_wg));
  if (c128)
    hipLaunchKernelGGL(k_ctqw_csr_direct<double2>, grid, dim3(kDirRows), 0, s, g.rp, wg_row, dcol, hcol, split,
                       g.markbits, static_cast<const double2 *>(y), static_cast<const double2 *>(psi),
                       static_cast<double2 *>(out), alpha, beta);
  else
    hipLaunchKernelGGL(k_ctqw_csr_direct<float2>, grid, dim3(kDirRows), 0, s, g.rp, wg_row, dcol, hcol, split,
                       g.markbits, static_cast<const float2 *>(y), static_cast<const float2 *>(psi),
                       static_cast<float2 *>(out), alpha, beta);
  return hipGetLastError();
}

hipError_t batch_ell_lds(bool c128, BatchCtl *ctl, const WalkSlot *slots, const TileEntry *tiles,
                         const int32_t *n_tiles, int grid, int advance, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  static_assert(kLdsTileRows64 % kLdsTileThreads64 == 0 && kLdsTileRows128 % kLdsTileThreads128 == 0,
                "whole rows per thread");
  if (c128)
    hipLaunchKernelGGL((k_batch_ell_lds<double2, kLdsTileThreads128, kLdsTileRows128 / kLdsTileThreads128,
                                        kLdsBlockBytes128 / 16>),
                       dim3(grid), dim3(kLdsTileThreads128), 0, s, ctl, slots, tiles, n_tiles, advance);
  else
    hipLaunchKernelGGL((k_batch_ell_lds<float2, kLdsTileThreads64, kLdsTileRows64 / kLdsTileThreads64,
                                        kLdsBlockBytes64 / 8>),
                       dim3(grid), dim3(kLdsTileThreads64), 0, s, ctl, slots, tiles, n_tiles, advance);
  return hipGetLastError();
}

int dense_splits(const GraphView &g) {
  const int rblocks = (g.n + kDenseRows - 1) / kDenseRows;
  int sp = (512 + rblocks - 1) / rblocks;
  sp = std::min(sp, kMaxDenseSplits);
  sp = std::min(sp, std::max(1, g.n / (4 * kDenseK)));
  return std::max(sp, 1);
}

hipError_t dense_fill(bool c128, const GraphView &g, double gamma, size_t rows_pad, hipStream_t s) {
  const int64_t total = static_cast<int64_t>(rows_pad) * g.ld;
  const dim3 zgrid(static_cast<unsigned>(std::min<int64_t>((total + kBlock - 1) / kBlock, 8192)));
  const dim3 sgrid(blocks_for(g.n, kBlock));
  if (c128) {
    hipLaunchKernelGGL(k_dense_zero<double>, zgrid, dim3(kBlock), 0, s, static_cast<double *>(g.dense), total);
    if (g.n) hipLaunchKernelGGL(k_dense_scatter<double>, sgrid, dim3(kBlock), 0, s, g, static_cast<double *>(g.dense), gamma);
  } else {
    hipLaunchKernelGGL(k_dense_zero<float>, zgrid, dim3(kBlock), 0, s, static_cast<float *>(g.dense), total);
    if (g.n) hipLaunchKernelGGL(k_dense_scatter<float>, sgrid, dim3(kBlock), 0, s, g, static_cast<float *>(g.dense), gamma);
  }
  return hipGetLastError();
}

hipError_t dense_stage(bool c128, const GraphView &g, const void *y, const void *psi, void *out, double c,
                       hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  if (c128) launch_dense_nt<double>(g, y, psi, out, c, s);
  else launch_dense_nt<float>(g, y, psi, out, c, s);
  return hipGetLastError();
}

StripGrid torus_strips(bool c128, int l1, int l2, int S) {
  StripGrid sg;
  if (S < 2 || S >= kSweepRing || l2 < 64) return StripGrid{};
  sg.width = 64;
  sg.core = 64 - 2 * S;
  sg.halo = S;
  sg.tiles_c = (l2 + sg.core - 1) / sg.core;
  // strips as tall as possible while every SIMD still gets its wavefronts.
  // complex64: two per SIMD as long as the strips stay at least 2S rows tall;
  // the second wavefront hides the latency of the first's dependent stages
  // and loads, which measured worth more than the extra halo rows (S = 5:
  // 1024^2 4% and 2048^2 18% faster than one wavefront per SIMD, 4096^2 the
  // same; three per SIMD no better).  complex128: one per SIMD (two measured
  // 2% slower on 2048^2 and 4096^2).  Strips with one wavefront per SIMD keep
  // at least 4S rows, so the halo rows stay a minor share of the work.
  auto rows_for = [&](int waves_per_simd) {
    const int want_r = std::max(1, kSimds * waves_per_simd / sg.tiles_c);
    return (l1 + want_r - 1) / want_r;
  };
  int rows = !c128 && rows_for(2) >= 2 * S ? rows_for(2) : std::max(rows_for(1), kSweepMinRowsPerStage * S);
  rows = std::min(rows, l1 - 2 * S);  // a strip's window rows must be distinct grid rows
  if (rows < 1) return StripGrid{};
  sg.rows = rows;
  sg.tiles_r = (l1 + rows - 1) / rows;
  return sg;
}

int torus_block_depth(bool c128, const GraphView &g, int K) {
  if (g.structure != kTorus) return 1;
  for (int S : {5, 4, 3, 2})
    if (K % S == 0 && torus_strips(c128, g.dims[0], g.dims[1], S).count() > 0) return S;
  return 1;
}

template <typename T, int S>
hipError_t launch_sweep(const GraphView &g, const void *P, const void *Yin, void *Out, int kfirst,
                        const typename SweepCoefs<T>::type &c, hipStream_t s) {
  const StripGrid sg = torus_strips(sizeof(T) == 16, g.dims[0], g.dims[1], S);
  if (sg.count() == 0 || sg.rows != g.strip_rows || !g.tmark) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>((sg.count() + kStripWaves - 1) / kStripWaves)), block(64 * kStripWaves);
  const T *p = static_cast<const T *>(P), *y = static_cast<const T *>(Yin);
  if (Yin == P)
    hipLaunchKernelGGL((k_ctqw_torus_sweep<T, S, true>), grid, block, 0, s, g, p, y, static_cast<T *>(Out), kfirst, c);
  else
    hipLaunchKernelGGL((k_ctqw_torus_sweep<T, S, false>), grid, block, 0, s, g, p, y, static_cast<T *>(Out), kfirst, c);
  return hipGetLastError();
}

hipError_t torus_block_stages(bool c128, const GraphView &g, int S, const void *P, const void *Yin, void *Out,
                              int kfirst, const double *alpha, const double *beta, hipStream_t s) {
  if (c128) {
    Coefs c;
    for (int k = 0; k < 64; ++k) {
      c.alpha[k] = alpha[k];
      c.beta[k] = beta[k];
    }
    switch (S) {
      case 5: return launch_sweep<double2, 5>(g, P, Yin, Out, kfirst, c, s);
      case 4: return launch_sweep<double2, 4>(g, P, Yin, Out, kfirst, c, s);
      case 3: return launch_sweep<double2, 3>(g, P, Yin, Out, kfirst, c, s);
      case 2: return launch_sweep<double2, 2>(g, P, Yin, Out, kfirst, c, s);
      default: return hipErrorInvalidValue;
    }
  }
  CoefsF32 c;
  for (int k = 0; k < 64; ++k) {
    c.ahi[k] = static_cast<float>(alpha[k]);
    c.alo[k] = static_cast<float>(alpha[k] - static_cast<double>(c.ahi[k]));
    c.bhi[k] = static_cast<float>(beta[k]);
    c.blo[k] = static_cast<float>(beta[k] - static_cast<double>(c.bhi[k]));
  }
  switch (S) {
    case 5: return launch_sweep<float2, 5>(g, P, Yin, Out, kfirst, c, s);
    case 4: return launch_sweep<float2, 4>(g, P, Yin, Out, kfirst, c, s);
    case 3: return launch_sweep<float2, 3>(g, P, Yin, Out, kfirst, c, s);
    case 2: return launch_sweep<float2, 2>(g, P, Yin, Out, kfirst, c, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t batch_struct(bool c128, const BatchCtl *ctl, const WalkSlot *slots, const TileEntry *tiles,
                        const int32_t *n_tiles, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (c128)
    hipLaunchKernelGGL(k_batch_struct<double2>, dim3(grid), dim3(kTileThreads), 0, s, ctl, slots, tiles, n_tiles);
  else
    hipLaunchKernelGGL(k_batch_struct<float2>, dim3(grid), dim3(kTileThreads), 0, s, ctl, slots, tiles, n_tiles);
  return hipGetLastError();
}

hipError_t finish_readout(const GraphView &g, int count, const Readout &ro, hipStream_t s) {
  if (!ro.norm && !ro.pmarked) return hipSuccess;
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, ro.partials, count, ro.p_out(), g.marklist,
                     g.n_marked, g.structure == kDense ? g.columns : 1, ro.norm, ro.pmarked);
  return hipGetLastError();
}

}  // namespace qwk
