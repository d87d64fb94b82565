/*
 * qwalk.h -- C ABI of the MI355X quantum-walk step engine.
 *
 * The engine applies the time-evolution step of the two walk models of
 * Hiperwalk (arXiv 2406.08186) to a complex state vector held in device
 * memory, and reduces the state to per-vertex probabilities in FP64.
 *
 *   Coined walk (Sec. 3.2): one step is psi <- S C psi, with the flip-flop
 *   shift S|v,w> = |w,v> and the Grover coin
 *   C|v,w> = sum_{v' in N(v)} (2/d(v) - delta_{w,v'}) |v,v'>.  The arc basis is
 *   the paper's: arcs grouped by tail, the group of tail v being row v of the
 *   CSR adjacency.  Two extensions serve the benchmark workloads: the
 *   Hadamard coin (1/sqrt2)[[1,1],[1,-1]] on a degree-2 vertex's two arcs in
 *   row order, and the coin -I at marked vertices (spatial search).
 *   Probability (Sec. 3.2): p_v = sum over arcs with tail v of |psi_a|^2.
 *
 *   Continuous-time walk (Sec. 3.1): H = -gamma A - sum_{v in M} |v><v|,
 *   psi(t) = exp(-iHt) psi(0).  One step of length dt applies the order-K
 *   Taylor polynomial T_K(-iH dt) = sum_{k=0..K} (-iH dt)^k / k!, evaluated
 *   as K sparse products (Horner form).  Probability (Sec. 3.1):
 *   p_v = |psi_v|^2.
 *
 * Conventions
 *   - Every function returns a status (QW_OK or an error code) and never
 *     throws; qw_last_error() gives a thread-local description of the last
 *     failure on the calling thread.
 *   - Host pointers are read during the call only; the library copies what
 *     it keeps.  Device pointers are caller-owned: the library never
 *     allocates, frees or retains device memory beyond what the caller
 *     passes in, and never frees caller memory.
 *   - Complex arrays are interleaved (re, im): float2 for QW_C64, double2
 *     for QW_C128 (the layout of torch.complex64 / torch.complex128).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Device-side calls are asynchronous on it: they enqueue kernels and
 *     copies and return; errors of the kernels themselves surface at the
 *     caller's next synchronising call.  They perform no allocation and no
 *     host synchronisation, so they may be captured into a hipGraph.
 */
#ifndef QWALK_H
#define QWALK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define QW_OK 0
#define QW_EINVAL 1       /* null pointer, bad enum, out-of-range scalar       */
#define QW_EGRAPH 2       /* adjacency not a simple symmetric graph            */
#define QW_EUNSUPPORTED 3 /* valid input outside what the engine implements    */
#define QW_ENOMEM 4       /* caller buffer smaller than the size query / host  */
#define QW_EDEVICE 5      /* a HIP runtime call or kernel launch failed        */
#define QW_ESTATE 6       /* call out of order (e.g. evolve before upload)     */

/* ---- enums ------------------------------------------------------------- */
#define QW_COINED 0
#define QW_CTQW 1
/* Staggered walk (named as future work in Sec. 5; the paper gives no
 * definition, the engine follows the published staggered model of Portugal
 * et al.).  The state lives on the vertices.  Each tessellation k partitions
 * the vertices into polygons alpha (cliques of the graph) with real unit
 * vectors |alpha> = sum_{v in alpha} a_v |v> (uniform a_v = 1/sqrt|alpha|
 * unless given); P_k = sum_alpha |alpha><alpha| and H_k = 2 P_k - I.  One step
 * is psi <- U_T ... U_1 R_M psi: first the phase flip R_M = I - 2 sum_{m in M}
 * |m><m| of the marked vertices, then U_1, ..., U_T in order, with
 * U_k = H_k (QW_REFLECTION) or U_k = exp(i theta_k H_k) = cos(theta_k) I +
 * i sin(theta_k) H_k (QW_HAMILTONIAN).  Probability: p_v = |psi_v|^2. */
#define QW_STAGGERED 2

#define QW_REFLECTION 0
#define QW_HAMILTONIAN 1

/* Coins (Sec. 3.2).  GROVER: (2/d) J - I on each vertex's arcs.  HADAMARD:
 * (1/sqrt 2)[[1, 1], [1, -1]] (degree 2 only).  FOURIER: F[j][k] =
 * exp(2 pi i j k / d) / sqrt(d).  MATRIX: the caller's d x d matrix.
 * SZEGEDY: the reflection 2|alpha_x><alpha_x| - I with alpha_x = sum_y
 * sqrt(P_xy) |x,y>, which with the flip-flop shift is Szegedy's walk for the
 * transition matrix P (the paper's future work, Sec. 5; GROVER is the case
 * P_xy = 1/d_x).  Marked vertices take -I whatever the coin.  HADAMARD,
 * FOURIER and MATRIX act on the coin basis, which is the order of the
 * vertex's row in the CSR. */
#define QW_GROVER 0
#define QW_HADAMARD 1
#define QW_FOURIER 2
#define QW_MATRIX 3
#define QW_SZEGEDY 4

/* Shifts (Sec. 3.2).  FLIPFLOP: S|v,w> = |w,v>.  PERSISTENT (the lattice
 * shift of position-coin notation): the walker keeps its direction, S maps
 * the arc v -> w to the arc w -> u with u = w + (w - v) on a cycle or a
 * periodic 2-D grid. */
#define QW_FLIPFLOP 0
#define QW_PERSISTENT 1

#define QW_C64 0  /* complex64 state, FP64 reductions */
#define QW_C128 1 /* complex128 state                 */

/* Path choice.  AUTO runs a walk small enough for one workgroup's LDS in a
 * single launch, otherwise recognises cycles, periodic 2-D grids and
 * hypercubes in the CSR and uses index-free structured kernels for them
 * (for a CTQW on any other regular graph of degree <= 64, a column-major
 * neighbour table without row pointers), and otherwise the general sparse
 * kernels.  CSR forces the general sparse
 * kernels.  STRUCTURED is AUTO without the one-workgroup path. */
#define QW_LAYOUT_AUTO 0
#define QW_LAYOUT_CSR 1
#define QW_LAYOUT_STRUCTURED 2
/* CTQW only: H stored densely (N x N, FP64 for QW_C128, FP32 for QW_C64) and
 * each Horner stage run as a real-split complex GEMM on the matrix cores, for
 * `columns` walks that share H (state: N x columns complex, vertex-major:
 * element (v, b) at v*columns + b).  For dense graphs and batches of walks
 * (the paper's dense vector-matrix product, Sec. 4.6.1, is the B = 1 case). */
#define QW_LAYOUT_DENSE 3

/* Structure the plan chose (reported by qw_plan_get_info). */
#define QW_STRUCT_GENERAL 0
#define QW_STRUCT_CYCLE 1
#define QW_STRUCT_TORUS 2
#define QW_STRUCT_HYPERCUBE 3
#define QW_STRUCT_SMALL 4 /* whole walk in one launch on one workgroup: resident in its LDS, or, for a
                             coined walk on at most 64 vertices all of degree 2, in one wavefront's
                             registers */
#define QW_STRUCT_ELL 5   /* CTQW on a regular graph: column-major neighbour table */
#define QW_STRUCT_DENSE 6 /* CTQW with a dense H on MFMA (QW_LAYOUT_DENSE)        */
#define QW_STRUCT_STAG_LATTICE 7 /* staggered walk on an even periodic l1 x l2
                                    lattice tessellated by its 2 x 2 squares
                                    (corners at even, then at odd coordinates,
                                    uniform amplitudes): both tessellations of
                                    a step in one index-free launch          */

/* ---- graph ------------------------------------------------------------- */
/* Adjacency pattern of a simple undirected graph (Sec. 3.1 and 3.2 take the
 * graph as its adjacency matrix A).  Host memory, read at plan creation.
 *   n        vertices, 0 <= n < 2^31
 *   row_ptr  int64[n+1], row_ptr[0] = 0, non-decreasing, row_ptr[n] = number
 *            of arcs (= nnz(A) = 2|E|), below 2^31
 *   col      int32[row_ptr[n]]: heads of the arcs whose tail is the row.
 * A must be symmetric with no self-loops and no repeated entries in a row
 * (else QW_EGRAPH).  Rows need not be sorted: the order of row v is the
 * order of v's coin basis (the paper's default is ascending head labels). */
typedef struct qw_csr {
  int64_t n;
  const int64_t *row_ptr;
  const int32_t *col;
} qw_csr;

/* ---- staggered-walk tessellation ----------------------------------------- */
/* One tessellation of a staggered walk (QW_STAGGERED above).  Host memory,
 * read and copied at plan creation.
 *   n_polygons  >= 1 (0 only when the graph has no vertices)
 *   poly_ptr    int64[n_polygons + 1], poly_ptr[0] = 0, strictly increasing,
 *               poly_ptr[n_polygons] = n: polygon p is the vertex list
 *               poly_vert[poly_ptr[p] .. poly_ptr[p+1] - 1]
 *   poly_vert   int32[n], every vertex exactly once (a partition); every
 *               polygon must be a clique of the plan's graph (else QW_EGRAPH)
 *   amp         double[n] aligned with poly_vert (the real amplitude of the
 *               vertex in its polygon's vector; each polygon's squares sum to
 *               1 within 1e-12), or NULL for uniform amplitudes
 *   form        QW_REFLECTION or QW_HAMILTONIAN; theta: the angle of the
 *               Hamiltonian form (finite), ignored by the reflection form */
typedef struct qw_tessellation {
  int64_t n_polygons;
  const int64_t *poly_ptr;
  const int32_t *poly_vert;
  const double *amp;
  int32_t form;
  double theta;
} qw_tessellation;

/* ---- walk description --------------------------------------------------- */
typedef struct qw_walk_desc {
  int32_t kind;         /* QW_COINED, QW_CTQW or QW_STAGGERED                   */
  int32_t coin;         /* coined: QW_GROVER, QW_HADAMARD (degree 2 only),
                           QW_FOURIER, QW_MATRIX or QW_SZEGEDY                 */
  int32_t dtype;        /* QW_C64 or QW_C128                                   */
  int32_t layout;       /* QW_LAYOUT_AUTO or QW_LAYOUT_CSR                     */
  double gamma;         /* CTQW: gamma > 0 (Sec. 3.1)                          */
  double dt;            /* CTQW: step length > 0                               */
  int32_t taylor_order; /* CTQW: K in [1, 64]; 0 = smallest K meeting trunc_tol
                           over horizon_steps steps (qw_taylor_order)          */
  double trunc_tol;     /* CTQW, taylor_order = 0: bound on the accumulated
                           truncation error                                    */
  int64_t horizon_steps;/* CTQW, taylor_order = 0: steps the bound must cover  */
  const int32_t *marked;/* host int32[n_marked], distinct vertices in [0, n):
                           coin -I (coined) / -|v><v| term (CTQW); may be NULL
                           when n_marked = 0                                   */
  int64_t n_marked;
  int32_t columns;      /* QW_LAYOUT_DENSE: walks sharing H, 1..128 (0 = 1);
                           other layouts: must be 0 or 1                      */
  int32_t shift;        /* coined: QW_FLIPFLOP or QW_PERSISTENT                */
  int32_t coin_dim;     /* coined, QW_MATRIX: d, the degree of every vertex    */
  const double *coin_matrix; /* coined, QW_MATRIX: host double[2 d d], row-major
                           interleaved complex C[j][k], copied at creation and
                           used as given (not checked for unitarity)          */
  const double *transition; /* coined, QW_SZEGEDY: host double[n_arcs], P of each
                           arc (tail -> head) in CSR order, >= 0, every row
                           of a vertex with arcs summing to 1 within 1e-12;
                           copied at creation                                 */
  int32_t n_tessellations; /* staggered: T in [1, 64]                         */
  const qw_tessellation *tessellations; /* staggered: host array of T, applied
                           in array order                                     */
} qw_walk_desc;
/* FOURIER and MATRIX coins and the PERSISTENT shift run on the index-free
 * lattice kernels only: the graph must be a cycle (rows ordered v+1, v-1) or
 * a periodic l1 x l2 grid, l1, l2 >= 3, vertex v = r*l2 + c (rows ordered
 * c+1, c-1, r+1, r-1, wrapping), and the layout AUTO or STRUCTURED; a
 * PERSISTENT shift with the GROVER coin accepts the rows in any order.
 * Otherwise QW_EUNSUPPORTED.  Such walks cannot join a batch.  The SZEGEDY
 * coin runs on the one-workgroup and general CSR paths (any graph, flip-flop
 * shift) and cannot join a batch either.  A STAGGERED walk (state length n,
 * marked vertices phase-flipped) runs on the one-workgroup path (AUTO, when
 * the state fits one workgroup's LDS) or on per-tessellation polygon kernels
 * (any layout but DENSE, which it rejects); with layout AUTO or STRUCTURED,
 * two tessellations that are the 2 x 2 squares of a periodic l1 x l2 lattice
 * (vertex r*l2 + c, l1 and l2 even and >= 4; the first with corners at even
 * coordinates, the second at odd ones; uniform amplitudes; either form) run
 * on a fused index-free kernel instead.  It cannot join a batch but can
 * join qw_small_many.  The graph only serves to check that every polygon is
 * a clique: edges that lie in no polygon play no part in the walk. */

typedef struct qw_plan qw_plan;

typedef struct qw_plan_info {
  int64_t n;               /* vertices                                        */
  int64_t n_arcs;          /* arcs (= 2|E|)                                   */
  int64_t state_len;       /* complex elements of the state: n_arcs (coined),
                              n (CTQW, staggered) or n * columns (dense)      */
  int32_t kind, coin, dtype, structure;
  int32_t dims[2];         /* CYCLE: {n,0}; TORUS, STAG_LATTICE: {l1,l2};
                              HYPERCUBE: {dim,0}; ELL: {degree,0}             */
  int32_t max_degree;
  int32_t taylor_order;    /* CTQW: K in use                                  */
  double dt;               /* CTQW: step length                               */
  double h_norm_bound;     /* CTQW: max_v gamma d(v) + [v in M]               */
  double trunc_bound;      /* CTQW: per-step truncation bound at (dt, K)      */
  size_t graph_bytes;      /* device bytes qw_plan_upload needs               */
  size_t state_bytes;      /* bytes of one state vector                       */
  size_t work_bytes;       /* device workspace qw_evolve/qw_probabilities need*/
  int32_t columns;         /* walks per state (dense layout), else 1          */
  int32_t block_depth;     /* CTQW on a torus: Horner stages per launch (> 1
                              when temporal blocking applies), else 1         */
} qw_plan_info;

/* The walk constructors of the paper's user interface: ContinuousTime(graph,
 * gamma, time, marked) (Sec. 3.1) and Coined(graph, shift, coin) (Sec. 3.2).
 * Validate the graph and the walk, precompute the host-side tables (reverse
 * arcs, degree tiles, structure recognition, Taylor order), and return a new
 * plan in *out.  Host only: touches no device.  Errors: QW_EINVAL (null
 * pointers, bad enums, gamma/dt not positive, marked vertex out of range or
 * repeated), QW_EGRAPH (asymmetric, self-loop, repeated arc, malformed
 * row_ptr, head out of range), QW_EUNSUPPORTED (Hadamard at an unmarked
 * vertex of degree other than 0 or 2, arcs >= 2^31, no K <= 64 meets
 * trunc_tol), QW_ENOMEM (host allocation).  On error *out is NULL. */
int qw_plan_create(const qw_csr *graph, const qw_walk_desc *walk, qw_plan **out);

/* Free a plan (host memory only).  NULL is accepted. */
int qw_plan_destroy(qw_plan *plan);

/* Sizes and choices of a plan. */
int qw_plan_get_info(const qw_plan *plan, qw_plan_info *info);

/* The explicit host-to-device move of the paper's library layer (Sec. 4.4:
 * data is moved to the device by an explicit call and stays in the caller's
 * ownership).  Copy the plan's device tables into the caller's device buffer d_graph
 * (at least info.graph_bytes bytes, 256-byte aligned) on `stream`, and bind
 * the plan to that buffer: later calls read it, so it must stay allocated
 * and unmodified while the plan is used.  A plan is bound to one buffer at a
 * time; uploading again rebinds it.  Not thread-safe against concurrent
 * calls on the same plan.  Errors: QW_EINVAL, QW_ENOMEM (buffer too small),
 * QW_EDEVICE. */
int qw_plan_upload(qw_plan *plan, void *d_graph, size_t graph_bytes, void *stream);

/* The time evolution of simulate() (Sec. 3.1: U(t) = exp(-iHt) applied to
 * the state; Sec. 3.2: U = S C applied step after step).
 * Advance the state by `steps` steps in place: psi <- U^steps psi (coined,
 * staggered) or psi <- T_K(-iH dt)^steps psi (CTQW).  d_psi: device state of
 * info.state_len complex elements in the boundary layout (coined: CSR arc
 * order; CTQW and staggered: vertex order), read and written.  d_work: device workspace of
 * at least info.work_bytes bytes, contents undefined on return.  If any of
 * d_p (double[n]), d_norm (double[1]), d_pmarked (double[1]) is non-NULL the
 * readout of qw_probabilities is produced from the final state as part of
 * the same call (fused into the last kernel where the layout permits).
 * steps = 0 leaves psi unchanged.  Errors: QW_EINVAL, QW_ENOMEM (workspace
 * too small), QW_ESTATE (not uploaded), QW_EDEVICE. */
int qw_evolve(const qw_plan *plan, void *d_psi, void *d_work, size_t work_bytes, int64_t steps,
              double *d_p, double *d_norm, double *d_pmarked, void *stream);

/* ---- Out-of-core evolution (Sec. 5: tiling operators larger than device memory)
 * The paper names, as future work, splitting matrices that exceed device
 * memory into tiles.  A CTQW plan on the CSR path (QW_LAYOUT_CSR) can keep its
 * largest table, the neighbour indices (4 bytes per arc), in caller-pinned
 * host memory; the device holds the state, the workspace, the row pointers,
 * the marked set and what the mode below keeps there.  Two modes:
 *
 * QW_STREAM_DIRECT (the default): the device keeps the indices of as many
 * arcs as the budget allows (a prefix of the CSR table) and the stage kernel
 * reads the others from the pinned buffer itself, across the host link, in
 * workgroup tiles staged through LDS: one launch per Horner stage, no copies
 * and no events.  The pinned buffer must be device-mapped (hipHostMalloc,
 * torch pin_memory); others are refused with QW_EINVAL.
 *
 * QW_STREAM_RING: every Horner stage streams the indices in row tiles
 * through a ring of three device slots, the copies (on a stream the plan
 * owns) overlapping the stage kernels of earlier tiles.  Stages visit the
 * tiles in alternating order and skip the copy of a tile the ring still
 * holds, so a stage streams the table minus the ring (nothing after the
 * first stage of a call when the ring holds every tile).
 *
 * Both modes sum every row's neighbours in arc order, so they give the same
 * bits as each other at every budget. */
#define QW_STREAM_DIRECT 0
#define QW_STREAM_RING 1
/* qw_plan_stream_sizes: for a device budget (bytes the walk may use on the
 * device in total: state + info.work_bytes + the streamed graph buffer) and a
 * mode, the pinned host bytes (*host_bytes: the neighbour table, padded to a
 * multiple of 16 bytes), the device graph buffer (*device_bytes,
 * <= budget - state - workspace), the number of row tiles a stage runs
 * (*n_tiles: ring tiles, or direct mode's workgroup tiles) and the arcs whose
 * indices stay on the device (*device_arcs; 0 in ring mode).  Host only.
 * Errors: QW_EUNSUPPORTED (not a CTQW plan on the CSR path), QW_ENOMEM (the
 * budget does not hold state, workspace and resident tables, and in ring
 * mode a slot of the largest row), QW_EINVAL (null plan, unknown mode).
 * NULL outputs are skipped. */
int qw_plan_stream_sizes(const qw_plan *plan, size_t device_budget, int mode, size_t *host_bytes,
                         size_t *device_bytes, int64_t *n_tiles, int64_t *device_arcs);
/* Bind the plan for out-of-core evolution with the same budget and mode:
 * copies the neighbour table into h_pinned (pinned host memory, 16-byte
 * aligned, >= *host_bytes, caller-owned, kept unmodified while bound) and the
 * resident tables into d_buf (device, >= *device_bytes, 256-byte aligned) on
 * `stream`; ring mode also creates the plan's copy stream and ring events.
 * Ends any previous binding; qw_plan_upload ends this one.  qw_evolve and
 * qw_probabilities then work as usual (qw_evolve enqueues the stage kernels,
 * and in ring mode the tile copies; host calls, no host sync); the plan
 * cannot join a batch.  Errors: as qw_plan_stream_sizes, QW_ENOMEM (buffers
 * below the sizes), QW_EINVAL (misaligned buffers, or in direct mode a host
 * buffer the device cannot read), QW_EDEVICE. */
int qw_plan_upload_streamed(qw_plan *plan, size_t device_budget, int mode, void *h_pinned, size_t host_bytes,
                            void *d_buf, size_t device_bytes, void *stream);

/* ---- Allocation-free evolution
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): qw_evolve
 * with its workspace taken from a device array the library holds, of
 * QW_STATIC_SCRATCH_BYTES bytes on each GPU it runs on (held from the
 * library's load until the process ends).  Same arguments and results as
 * qw_evolve(plan, d_psi, <that array>, QW_STATIC_SCRATCH_BYTES, steps, d_p,
 * d_norm, d_pmarked, stream); the caller still owns the state and the
 * readout outputs.  The array is looked up on the stream's device at the
 * first call there.  The call allocates no device memory (no hipMalloc or
 * hipFree, no allocating library routine).  Every call on one GPU shares that GPU's array,
 * which keeps the last call's contents (nothing in it needs to start at
 * zero): calls that overlap on one GPU (two streams, two threads) race and
 * must be serialised by the caller.  Errors: as qw_evolve, and QW_ENOMEM when
 * the plan's info.work_bytes exceeds QW_STATIC_SCRATCH_BYTES. */
#define QW_STATIC_SCRATCH_BYTES (64u * 1024u * 1024u)
int qw_evolve_static(const qw_plan *plan, void *d_psi, int64_t steps, double *d_p, double *d_norm,
                     double *d_pmarked, void *stream);

/* FP64 readout of a state (Sec. 3.1, Sec. 3.2): d_p[v] = probability of
 * vertex v (coined: summed over arcs with tail v; CTQW and
 * staggered: |psi_v|^2; dense
 * layout: d_p has n * columns entries, p of walk b at v*columns + b, and the
 * norm and marked sums run over all walks),
 * *d_norm = sum_v p_v, *d_pmarked = sum over the marked set of p_v.  Each
 * output pointer may be NULL.  Sums run in a fixed order: results are
 * bitwise reproducible for a given plan.  Errors as qw_evolve. */
int qw_probabilities(const qw_plan *plan, const void *d_psi, double *d_p, double *d_norm,
                     double *d_pmarked, void *d_work, size_t work_bytes, void *stream);

/* Snapshot transfer for simulate(range=...) (Sec. 3.1, Sec. 3.2: the state,
 * or its probabilities, at every step of a range, handed back to the caller
 * in host memory).  Copy `bytes` bytes from device memory d_src to h_dst,
 * pinned host memory the device can write (hipHostMalloc, or a framework's
 * pinned allocation built on it), by a kernel on `stream` whose stores cross
 * the host link directly; no copy engine takes part, so the copy is ordered
 * with the stream's kernels like any other launch and does not compete with
 * them for a second queue.  Both pointers 16-byte aligned; d_src lies in one
 * device allocation of at least `bytes` bytes from d_src on; h_dst holds at
 * least `bytes` bytes.  The caller owns both buffers; h_dst may be read once
 * the stream has passed the call.  bytes == 0 is a no-op.  Errors:
 * QW_EINVAL (null or misaligned buffer, source not device memory or shorter
 * than `bytes`, destination not pinned), QW_EDEVICE. */
int qw_copy_to_host(void *h_dst, const void *d_src, size_t bytes, void *stream);

/* ---- many small walks in one launch ------------------------------------- */
/* Advance `count` independent walks by steps[i] steps each (Sec. 3.1 for
 * CTQW, Sec. 3.2 for coined walks, QW_STAGGERED above for staggered walks)
 * in a single launch, one workgroup per
 * walk: each walk runs whole in its workgroup (in LDS, or in one wavefront's
 * registers where QW_STRUCT_SMALL says so), with the arithmetic and order of
 * qw_evolve on the same plan, so results are bitwise those of
 * qw_evolve(plans[i], d_psi[i], ..., steps[i]).  Every plan must be uploaded,
 * share one dtype and have taken the one-workgroup path (info.structure ==
 * QW_STRUCT_SMALL, which QW_LAYOUT_AUTO picks for graphs whose vectors fit in
 * LDS); the walks may differ in kind, graph and step count.  plans, d_psi
 * and steps are host arrays of count entries; d_psi[i] is the device state of
 * walk i, read and written in place; no readout is produced (call
 * qw_probabilities afterwards).  d_desc: caller-owned device buffer of at
 * least qw_small_many_desc_bytes(count) bytes that must stay allocated until
 * the launch has run; the call returns once the walk descriptors are staged
 * for the copy into it, and is otherwise asynchronous on `stream`.  count = 0
 * does nothing.  Errors: QW_EINVAL (null arrays, negative steps or count,
 * mixed dtypes, a plan not on the one-workgroup path), QW_ENOMEM (d_desc too
 * small), QW_ESTATE (a plan not uploaded), QW_EDEVICE. */
size_t qw_small_many_desc_bytes(int32_t count);
int qw_small_many(const qw_plan *const *plans, void *const *d_psi, const int64_t *steps, int32_t count,
                  void *d_desc, size_t desc_bytes, void *stream);

/* ---- batched walks ------------------------------------------------------ */
/* A batch advances many walks (of different graphs, sizes, kinds and step
 * counts) together: each launch moves every active slot one unit forward --
 * a Horner stage of a CTQW step, or one coined step -- so small walks share
 * launches with large ones.  Launch sequences are captured into a hipGraph
 * and replayed.  Slots can be filled and emptied between runs, which is how a
 * serving loop does continuous batching; the per-walk arithmetic and its order
 * do not depend on the other slots, so a walk's result is bitwise the same
 * alone and in any mix.  All slots share one dtype.  Walks need plans on the
 * general CSR path (QW_LAYOUT_CSR); CTQW walks need K >= 2; coined walks need
 * every vertex degree <= 2048.
 *
 * Typical use: qw_batch_create -> qw_batch_device_bytes -> (caller allocates)
 * -> qw_batch_bind -> qw_batch_set_slot... -> qw_batch_commit -> [optional
 * qw_batch_autotune] -> qw_batch_run(launches) -> qw_batch_remaining /
 * qw_batch_readout -> qw_batch_clear_slot / qw_batch_set_slot -> commit ...
 * Host calls on one batch are not thread-safe. */
typedef struct qw_batch qw_batch;

/* capacity: slots (1..2^20); max_tiles: upper bound on the tile table (a tile
 * is up to rows_per_tile CTQW rows or one LDS tile of a coined walk; rounded
 * up to a multiple of 8); dtype: QW_C64 or QW_C128.  Host only. */
int qw_batch_create(int32_t capacity, int32_t max_tiles, int32_t dtype, qw_batch **out);
/* Frees the batch's host state, pinned staging buffer, capture stream and
 * graph.  Does not touch caller device memory.  NULL is accepted. */
int qw_batch_destroy(qw_batch *batch);
/* Device bytes for the batch's tables (control word, slots, coefficients,
 * tiles). */
int qw_batch_device_bytes(const qw_batch *batch, size_t *bytes);
/* Bind the batch to a caller-owned device buffer (>= qw_batch_device_bytes,
 * 256-byte aligned), reset the launch counter and empty every slot (tables
 * uploaded on `stream`). */
int qw_batch_bind(qw_batch *batch, void *d_buf, size_t bytes, void *stream);
/* Stage a walk into `slot` (host side; takes effect at the next commit).  The
 * plan must be uploaded and outlive the slot; d_psi (state, in/out) and
 * d_work (>= the plan's work_bytes) are caller-owned and must not be used by
 * anything else while the walk runs.  `steps` time steps are run starting at
 * the next launch.  d_hist (CTQW only, may be NULL): double[steps], zeroed by
 * the caller, receives p_marked after each step (atomic adds, so with several
 * marked vertices the last bits depend on order). */
int qw_batch_set_slot(qw_batch *batch, int32_t slot, const qw_plan *plan, void *d_psi, void *d_work,
                      size_t work_bytes, int64_t steps, double *d_hist);
/* Empty a slot (host side; takes effect at the next commit). */
int qw_batch_clear_slot(qw_batch *batch, int32_t slot);
/* Rebuild the tile table (each walk's tiles on one XCD when the schedule says
 * so) and upload slots and tiles on `stream`.  QW_ENOMEM if the tiles exceed
 * max_tiles. */
int qw_batch_commit(qw_batch *batch, void *stream);
/* Enqueue `launches` batched launches on `stream` (graph replays plus single
 * launches, as qw_batch_launch_plan states).  Slots whose walks finished are
 * skipped by the kernel. */
int qw_batch_run(qw_batch *batch, int64_t launches, void *stream);
/* Replay mode.  use_graph != 0 (the default): qw_batch_run replays a captured
 * hipGraph of 16 launches and launches the remainder one by one.  use_graph
 * == 0: every launch is a direct kernel launch on the stream (same kernels,
 * same arithmetic and results; meant for profilers and counter collection,
 * which cannot attribute graph-replayed dispatches reliably).  Host only. */
int qw_batch_set_replay(qw_batch *batch, int32_t use_graph);
/* How qw_batch_run(launches) issues its work in the current mode: number of
 * graph replays (16 launches each) and of direct launches per batched unit.
 * Host only; NULL outputs are skipped. */
int qw_batch_launch_plan(const qw_batch *batch, int64_t launches, int64_t *graph_replays,
                         int64_t *direct_launches);
/* Launches still needed by a slot (host mirror; 0 for an empty or finished
 * slot), and launches enqueued since bind. */
int qw_batch_remaining(const qw_batch *batch, int32_t slot, int64_t *remaining);
int qw_batch_launches(const qw_batch *batch, int64_t *launches);
/* Finish a walk: bring its final state into d_psi (coined walks with an odd
 * step count end in the workspace) and produce the FP64 readout of
 * qw_probabilities into the given device pointers (each may be NULL).
 * QW_ESTATE if the slot has launches left. */
int qw_batch_readout(qw_batch *batch, int32_t slot, double *d_p, double *d_norm, double *d_pmarked,
                     void *stream);
/* Schedule knobs: CTQW rows per tile (64..2^20) and XCD-aware placement. */
int qw_batch_set_schedule(qw_batch *batch, int32_t rows_per_tile, int32_t xcd_aware);
/* Kernel for the Horner stages of CTQW walks on regular graphs of degree <= 8
 * (plans on the ELL path; the series of Sec. 3.1's evolution operator).
 * QW_BATCH_LDS (the default): tiles of 6912 rows (complex64) or 6144
 * (complex128), one workgroup each, that
 * pass over the walk's input vector in LDS-staged blocks, so the neighbour
 * gathers read LDS instead of L2 (walks whose state and workspace are 16-byte
 * aligned and whose state holds at least 16 bytes; others, like every other
 * walk, take the gather kernel).  QW_BATCH_GATHER: the gather kernel that
 * runs every other walk (rows_per_tile rows per tile, gathers through L2).
 * Both add a row's neighbours in increasing index order in FP64, so results
 * are bitwise equal.  Takes effect at the next commit.  Host only; QW_EINVAL
 * for another value. */
#define QW_BATCH_GATHER 0
#define QW_BATCH_LDS 1
int qw_batch_set_stage_kernel(qw_batch *batch, int32_t kernel);
/* The current schedule (rows per tile, XCD placement, stage kernel); NULL
 * outputs are skipped.  Host only. */
int qw_batch_get_schedule(const qw_batch *batch, int32_t *rows_per_tile, int32_t *xcd_aware, int32_t *kernel);
/* Autotuner: time each candidate schedule (stage kernel, rows per tile in
 * {256..4096}, XCD placement on/off) with `reps` probe launches in which
 * every active walk computes its first unit without advancing (states
 * unchanged), keep the fastest, and cache it in-process by (dtype, log2 total
 * rows, mean degree).  Synchronises `stream`.  QW_ESTATE unless every active
 * walk is at its first unit.  Outputs may be NULL; *ms_per_launch is -1 on a
 * cache hit. */
int qw_batch_autotune(qw_batch *batch, int32_t reps, void *stream, int32_t *rows_per_tile,
                      int32_t *xcd_aware, double *ms_per_launch);

/* ---- Taylor truncation rule (FP64, host) -------------------------------- */
/* With rho = dt * ||H|| the one-step remainder of the order-K series is at
 * most rho^(K+1)/(K+1)! * (K+2)/(K+2-rho) (valid for rho < K+2).
 * qw_taylor_order: smallest K in [1, 64] with steps * bound <= tol, in *K;
 * QW_EUNSUPPORTED if none.  qw_taylor_plan: for a total time t_total, the
 * smallest step count keeping rho <= rho_max, dt = t_total / steps, and K
 * from qw_taylor_order.  Errors: QW_EINVAL for non-positive or non-finite
 * arguments. */
int qw_taylor_order(double rho, int64_t steps, double tol, int32_t *K);
int qw_taylor_plan(double h_bound, double t_total, double rho_max, double tol, int32_t *K,
                   double *dt, int64_t *steps);
double qw_taylor_tail_bound(double rho, int32_t K);

/* Thread-local description of the last error on this thread ("" if none). */
const char *qw_last_error(void);

/* Library version string. */
const char *qw_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QWALK_H */
