// Internal declarations shared by the host runtime (qw_host.cpp) and the
// HIP kernels (qw_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace qwk {

// Layout of the coined general path: contiguous vertex ranges whose arcs fit
// one workgroup's LDS tile are processed together.
constexpr int kTileArcs = 2048;
constexpr int kTileThreads = 256;
// The LDS-staged batch stage, per state type: workgroup size, rows per tile
// (a whole number per thread) and the LDS block of the input vector it
// stages (whole rounds of 1 KiB direct loads by every wavefront).  complex64:
// 768 threads x 9 rows, 156 KiB blocks; complex128 (whose sum registers are
// twice as wide): 1024 threads x 6 rows, 144 KiB blocks.
constexpr int kLdsTileThreads64 = 768;
constexpr int kLdsTileRows64 = 6912;
constexpr int kLdsBlockBytes64 = 156 * 1024;
constexpr int kLdsTileThreads128 = 1024;
constexpr int kLdsTileRows128 = 6144;
constexpr int kLdsBlockBytes128 = 144 * 1024;
// single-walk ELL stage: vectors above kEllSliceFrom bytes are gathered in
// slices of kEllSliceEntries entries (measured best on 2^20 vertices for both
// types, against 64Ki and 256Ki: 1 MiB complex64, 2 MiB complex128).  The
// slicing pays from about 8 MiB on (random 6-regular graphs: 9.6 MiB and up
// faster, 4.8 MiB complex64 even, 7.2 MiB complex128 and below slower).
#ifndef QW_ELL_SLICE_FROM
#define QW_ELL_SLICE_FROM (int64_t{15} << 19)
#endif
constexpr int64_t kEllSliceFrom = QW_ELL_SLICE_FROM;
constexpr int kEllSliceEntries = 131072;
#ifndef QW_ELL_SLICE_ROWS
#define QW_ELL_SLICE_ROWS 2
#endif
constexpr int kEllSliceRows = QW_ELL_SLICE_ROWS;  // rows per thread of the sliced stage
constexpr int kDirRows = 256;   // rows per workgroup tile of the direct out-of-core stage (one per thread)
constexpr int kDirArcs = 8192;  // neighbour indices such a tile stages in LDS (32 KiB)
constexpr int kLinkCopyGroups = 16;  // workgroups of the device-to-pinned-host copy (enough for the link)
constexpr int kTileMaxVerts = 1024;
// Threads per workgroup of the elementwise/stencil kernels.
constexpr int kBlock = 256;
// LDS budget of the one-workgroup whole-walk kernels.
constexpr size_t kSmallLdsBytes = 156 * 1024;  // dynamic LDS of the one-workgroup path (of 160 KiB)
// Largest hypercube dimension the structured kernels handle.
constexpr int kMaxHypercubeDim = 30;

enum Structure : int32_t {
  kGeneral = 0, kCycle = 1, kTorus = 2, kHypercube = 3, kSmall = 4, kEll = 5, kDense = 6, kStagLattice = 7
};
// Dense-H GEMM tiles: rows of H per workgroup, k per LDS chunk.
constexpr int kDenseRows = 64;
constexpr int kDenseK = 32;  // H's leading dimension and split-k ranges are multiples of it
constexpr int kMaxDenseColumns = 128;
constexpr int kMaxDenseSplits = 8;
// Largest degree of the ELL (regular-graph) CTQW layout.
constexpr int kMaxEllDegree = 64;

// Grid CTQW strips (streaming temporal blocking): one wavefront sweeps a strip
// of 64 columns; strips are sized so each SIMD gets two of them (complex64,
// strips of at least 2S core rows), else one (at least kSweepMinRowsPerStage
// * S rows).
constexpr int kStripWaves = 4;  // wavefronts (strips) per workgroup
constexpr int kSimds = 256 * 4;  // MI355X: 256 compute units of 4 SIMDs
constexpr int kSweepMinRowsPerStage = 4;

// Strip decomposition of an l1 x l2 grid for S stages per launch.
struct StripGrid {
  int rows = 0;     // core rows per strip
  int width = 0;    // columns a wavefront holds
  int core = 0;     // core columns = width - 2S
  int halo = 0;     // S
  int tiles_r = 0;  // strips along the rows (last one clamped to the grid edge)
  int tiles_c = 0;
  int64_t count() const { return static_cast<int64_t>(tiles_r) * tiles_c; }
};

// Staggered walk: polygons of at most kStagThreadMax vertices are handled one
// per thread; larger ones are cut into chunks of at most kStagChunk positions,
// one workgroup per chunk (partial inner products, then the update).
constexpr int kStagThreadMax = 16;
constexpr int kStagChunk = 2048;
constexpr int kStagMaxTess = 64;

// One tessellation of a staggered walk as the kernels see it.  Offsets are
// bytes from the start of the plan's device buffer (-1: absent).
struct StagTess {
  int32_t n_small = 0;     // polygons on the thread path
  int32_t small_size = 0;  // > 0: all of size small_size, column-major table vert[j*n_small + p]; 0: CSR
  int32_t max_small = 0;   // largest thread-path polygon
  int32_t n_big = 0;       // polygons above kStagThreadMax vertices
  int32_t n_chunks = 0;    // chunks of the big polygons
  int32_t pad = 0;
  int64_t off_ptr = -1;    // thread path, CSR: int32[n_small + 1]
  int64_t off_vert = -1;   // thread path: int32 vertices
  int64_t off_amp = -1;    // thread path: double amplitudes (same layout as vert), -1 = uniform
  int64_t off_bptr = -1;   // big polygons: int32[n_big + 1] into bvert
  int64_t off_bvert = -1;
  int64_t off_bamp = -1;   // -1 = uniform
  int64_t off_chunk = -1;  // StagChunk[n_chunks]
  double c0[2] = {0.0, 0.0};  // U = c0 I + c1 (2P - I): reflection (0, 1), Hamiltonian (cos t, i sin t)
  double c1[2] = {1.0, 0.0};
};

// A chunk of a big polygon: positions [begin, end) of bvert; the polygon's
// chunks are first .. first + count - 1.
struct StagChunk {
  int32_t begin;
  int32_t end;
  int32_t first;
  int32_t count;
  int32_t size;  // vertices of the polygon
  int32_t pad[3];
};

// Device view of a plan's graph tables (pointers into the caller's buffer).
struct GraphView {
  int32_t n = 0;
  int32_t n_arcs = 0;
  int32_t structure = kGeneral;
  int32_t dims[2] = {0, 0};
  int32_t n_marked = 0;
  int32_t n_tiles = 0;
  int32_t group = 1;           // CTQW CSR: lanes per row
  int32_t sorted_rows = 0;     // CTQW CSR: every row's neighbours in increasing order
  const int32_t *rp = nullptr;      // n+1
  const int32_t *col = nullptr;     // n_arcs (CTQW general/small: CSR order; ELL: col[j*n + v])
  int32_t ell_d = 0;                // ELL degree
  int32_t columns = 1;              // dense: walks sharing H
  int32_t ld = 0;                   // dense: leading dimension of H (multiple of kDenseK)
  void *dense = nullptr;            // dense: H, rows padded to kDenseRows, FP64 or FP32
  double *dense_partial = nullptr;  // dense: split-k partial products (workspace)
  const int32_t *rev = nullptr;     // n_arcs (coined general/small)
  const int32_t *tiles = nullptr;   // n_tiles+1 (coined general)
  const int32_t *perm = nullptr;    // n_arcs (coined structured: slot-major -> CSR position)
  const uint32_t *markbits = nullptr;  // ceil(n/32)
  const int32_t *marklist = nullptr;   // n_marked
  const uint8_t *tmark = nullptr;      // grid CTQW strips: 1 if a marked vertex lies in the strip's window
  int32_t strip_rows = 0;              // grid CTQW strips: core rows per strip
  int32_t two_reg = 0;                 // coined, one workgroup: 1 if every vertex has degree 2 and n <= 64
                                       // (amplitudes in one wavefront's registers), 2 if moreover a cycle in
                                       // direction order (rev[2v] = 2(v+1)+1, rev[2v+1] = 2(v-1), mod n)
  int32_t persistent = 0;              // coined on a lattice: persistent shift
  const double *coin = nullptr;        // coined on a lattice: d x d complex coin (row-major), else null
  const double *sqrtp = nullptr;       // Szegedy coin: sqrt(P) per arc, else null
  const unsigned char *base = nullptr; // start of the plan's device buffer
  const StagTess *stag = nullptr;      // staggered: device array of n_tess descriptors
  int32_t n_tess = 0;
};

// One walk of a many-small-walks launch (the whole walk in one workgroup's LDS).
struct SmallWalk {
  GraphView g;
  void *psi = nullptr;
  int32_t coined = 0;
  int32_t hadamard = 0;
  int32_t K = 0;
  int32_t staggered = 0;
  int64_t steps = 0;
  double alpha[64] = {};  // CTQW stage coefficients gamma dt / k, dt / k
  double beta[64] = {};
};

// Readout request: any pointer may be null.  `pscratch` (n doubles) and
// `partials` (enough for the launch) come from the workspace.
struct Readout {
  double *p = nullptr;
  double *norm = nullptr;
  double *pmarked = nullptr;
  double *pscratch = nullptr;
  double *partials = nullptr;
  bool any() const { return p || norm || pmarked; }
  double *p_out() const { return p ? p : pscratch; }
};

// Coefficients of one Horner stage y_out = psi + i*(alpha*sum_nbr y + beta*[marked] y_v),
// alpha = gamma*dt/k, beta = dt/k (FP64; rounded once for complex64).
struct StageCoef {
  double alpha;
  double beta;
};

// ---- launchers (qw_kernels.hip) -------------------------------------------
// All return the hipError_t of the launch (hipGetLastError after it).
hipError_t coined_small(bool c128, const GraphView &g, void *psi, int hadamard, int64_t steps,
                        const Readout &ro, hipStream_t s);
size_t coined_small_lds(bool c128, int n, int n_arcs);

hipError_t coined_tile_step(bool c128, const GraphView &g, const void *in, void *out,
                            int hadamard, hipStream_t s);
hipError_t coined_struct_step(bool c128, const GraphView &g, const void *in, void *out,
                              int hadamard, hipStream_t s);
hipError_t coined_perm_in(bool c128, const GraphView &g, const void *psi, void *internal,
                          hipStream_t s);
hipError_t coined_perm_out(bool c128, const GraphView &g, const void *internal, void *psi,
                           const Readout &ro, hipStream_t s);
hipError_t copy_state(bool c128, int64_t len, const void *in, void *out, hipStream_t s);
hipError_t coined_prob_csr(bool c128, const GraphView &g, const void *psi, const Readout &ro,
                           hipStream_t s);

hipError_t small_many(bool c128, const SmallWalk *d_walks, int count, size_t lds, int threads, hipStream_t s);
hipError_t ctqw_small(bool c128, const GraphView &g, void *psi, const double *alpha,
                      const double *beta, int K, int64_t steps, const Readout &ro, hipStream_t s);
size_t ctqw_small_lds(bool c128, int n, int n_arcs);
hipError_t ctqw_stage(bool c128, const GraphView &g, const void *y, const void *psi, void *out,
                      StageCoef c, const Readout *fused, hipStream_t s);
hipError_t vertex_prob(bool c128, const GraphView &g, const void *psi, const Readout &ro,
                       hipStream_t s);

// Dense H: expand the CSR into H (zero fill then scatter of -gamma and the
// marked diagonal), and one Horner stage y_out = psi + (-i c) H y_in on MFMA.
hipError_t dense_fill(bool c128, const GraphView &g, double gamma, size_t rows_pad, hipStream_t s);
// Number of k ranges the dense stage splits into (1 = no split; partials then unused).
int dense_splits(const GraphView &g);
hipError_t dense_stage(bool c128, const GraphView &g, const void *y, const void *psi, void *out, double c,
                       hipStream_t s);

// Grid CTQW with temporal blocking: depth S (stages per launch, dividing K;
// 1 = not applicable), and S stages k = kfirst..kfirst-S+1 of one time step
// from (P, Yin) to Out (Yin may equal P at the first stage of a step).
// alpha/beta hold 64 entries (stage k at [k-1]).
int torus_block_depth(bool c128, const GraphView &g, int K);
StripGrid torus_strips(bool c128, int l1, int l2, int S);
hipError_t torus_block_stages(bool c128, const GraphView &g, int S, const void *P, const void *Yin, void *Out,
                              int kfirst, const double *alpha, const double *beta, hipStream_t s);

// Staggered walk.  stag_small: every step in one workgroup's LDS (descriptors
// read from g.stag).  stag_tess: one tessellation in place on psi; `mark`
// applies the marked phase flip to what it reads (first tessellation of a
// step); `partials` holds t.n_chunks complex partial sums (workspace).
size_t stag_small_lds(bool c128, int n);
hipError_t stag_small(bool c128, const GraphView &g, void *psi, int64_t steps, const Readout &ro, hipStream_t s);
hipError_t stag_tess(bool c128, const GraphView &g, const StagTess &t, void *psi, bool mark, double *partials,
                     hipStream_t s);
// Staggered walk on the square lattice (structure kStagLattice, dims {l1, l2}):
// `steps` (1 or 2) steps, both tessellations each, in one launch, from `in`
// to `out` (distinct buffers); `ta`, `tb` give the tessellations' (c0, c1).
hipError_t stag_lattice_step(bool c128, const GraphView &g, const StagTess &ta, const StagTess &tb, int steps,
                             const void *in, void *out, hipStream_t s);

// Sum of `count` partials -> *norm; sum over the marked list of p -> *pmarked.
hipError_t finish_readout(const GraphView &g, int count, const Readout &ro, hipStream_t s);

// ---- batched execution ------------------------------------------------------
// Launch counter shared by all workgroups of a batched launch: every
// workgroup reads L at its start; the last one to finish advances it.
struct BatchCtl {
  unsigned long long L;      // launches completed
  unsigned int done;         // workgroups finished in the current launch
  unsigned int probe;        // 1: timing probe (every walk runs its first stage, L frozen)
};

// One walk of a batch (device copy).  kind < 0 marks an empty slot.
struct WalkSlot {
  int32_t kind;      // QW_COINED / QW_CTQW, -1 = empty
  int32_t n;
  int32_t K;         // CTQW Taylor order (>= 2); 1 for coined
  int32_t hadamard;
  int64_t L0;        // global launch index at which the walk starts
  int64_t units;     // launches it needs: steps * K (CTQW) or steps (coined)
  const int32_t *rp;
  const int32_t *col;     // CTQW (CSR order, or column-major when ell_d > 0)
  int32_t ell_d;          // CTQW: regular degree of the ELL layout, 0 = CSR
  int32_t pad0;
  const int32_t *rev;     // coined
  const uint32_t *markbits;
  void *psi;
  void *w0;
  void *w1;
  const double *alpha;    // K entries, stage k at [k-1]
  const double *beta;
  double *hist;           // CTQW: p_marked after each step (caller-zeroed), may be null
  int32_t structure;      // coined: kGeneral (CSR tiles, state in psi/w0) or kCycle/kTorus/
                          // kHypercube (slot-major state in w0/w1, see k_batch_struct)
  int32_t sdims[2];       // structured coined: {n, 0} / {l1, l2} / {dim, 0}
  int32_t pad1;
};

// A unit of work of a batched launch: rows (CTQW) or vertices (coined) [begin, end) of a slot.
struct TileEntry {
  int32_t slot;      // -1 = padding
  int32_t begin;
  int32_t end;
  int32_t pad;
};

// The gather-path stage of a batched launch (CSR and ELL CTQW tiles, general
// coined tiles); the last workgroup advances the launch counter when
// `advance` is nonzero.
hipError_t batch_stage(bool c128, BatchCtl *ctl, const WalkSlot *slots, const TileEntry *tiles,
                       const int32_t *n_tiles, int grid, int advance, hipStream_t s);
// Out-of-core CTQW stage on rows [r0, r1) whose neighbour indices (CSR arcs
// [arc0, ...)) sit in a device slot: slot[a - arc0] = col[a].
hipError_t ctqw_slot_stage(bool c128, const GraphView &g, const int32_t *slot, int64_t arc0, int r0, int r1,
                           const void *y, const void *psi, void *out, double alpha, double beta, hipStream_t s);
// Copy `bytes` bytes of device memory src to dst, the device view of pinned
// host memory, by a kernel on stream s (both 16-byte aligned).
hipError_t copy_link(void *dst, const void *src, size_t bytes, hipStream_t s);
// Direct out-of-core CTQW stage: workgroup tile w holds rows [wg_row[w],
// wg_row[w+1]) (at most kDirRows rows and kDirArcs arcs, or one longer row);
// neighbour indices of arcs below `split` (a multiple of 4) come from the
// device prefix dcol, the others straight from pinned host memory hcol (both
// 16-byte aligned, hcol padded to a multiple of 4 entries).
hipError_t ctqw_direct_stage(bool c128, const GraphView &g, const int32_t *wg_row, int64_t n_wg, const int32_t *dcol,
                             const int32_t *hcol, int64_t split, const void *y, const void *psi, void *out,
                             double alpha, double beta, hipStream_t s);
// The LDS-staged stage of the batch's CTQW walks on the ELL layout (degree
// <= 8): tiles of kLdsTileRows64/128 rows, one workgroup of
// kLdsTileThreads64/128 each, the input vector staged in blocks of
// kLdsBlockBytes64/128.  The last workgroup
// advances the launch counter when `advance` is nonzero.
hipError_t batch_ell_lds(bool c128, BatchCtl *ctl, const WalkSlot *slots, const TileEntry *tiles,
                         const int32_t *n_tiles, int grid, int advance, hipStream_t s);
// The structured coined tiles of a batched launch (run before batch_stage in
// each launch unit; reads the launch counter, does not advance it).
hipError_t batch_struct(bool c128, const BatchCtl *ctl, const WalkSlot *slots, const TileEntry *tiles,
                        const int32_t *n_tiles, int grid, hipStream_t s);

// Number of partial sums the readout kernels (one thread per vertex) write.
int readout_partials(const GraphView &g);
// Number of partial sums a CTQW stage with the readout fused writes.
int ctqw_stage_partials(const GraphView &g);

}  // namespace qwk
