// Host-side plan object shared by the plan and batch halves of the C ABI.
// Not part of the public ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "qw_internal.h"
#include "qwalk.h"

struct qw_plan {
  // walk description
  int32_t kind = QW_COINED, coin = QW_GROVER, dtype = QW_C128, layout = QW_LAYOUT_AUTO;
  int32_t shift = QW_FLIPFLOP;
  std::vector<double> coin_mat;  // Fourier / matrix coin: interleaved complex d x d, row-major
  bool lattice() const { return shift == QW_PERSISTENT || coin == QW_FOURIER || coin == QW_MATRIX; }
  std::vector<double> sqrt_p;  // Szegedy coin: sqrt(P) per arc
  int32_t structure = qwk::kGeneral;
  int64_t n = 0, n_arcs = 0;
  int32_t dims[2] = {0, 0};
  int32_t max_degree = 0;
  double gamma = 0.0, dt = 0.0, h_bound = 0.0, trunc_bound = 0.0;
  int32_t K = 0;
  int32_t n_marked = 0;
  int32_t n_tiles = 0;
  int32_t group = 1;
  int32_t sorted_rows = 0;  // CTQW CSR: every row's neighbours in increasing order
  // dense layout: walks per state, leading dimension and padded rows of H,
  // and where H sits in the device graph buffer (after the uploaded image)
  int32_t columns = 1;
  int32_t ld = 0;
  size_t rows_pad = 0, off_dense = 0, dense_bytes = 0, off_dpartial = 0;
  // host image of the device graph buffer, and section offsets into it
  std::vector<unsigned char> image;
  size_t off_rp = 0, off_col = 0, off_rev = 0, off_tiles = 0, off_perm = 0, off_bits = 0, off_mlist = 0;
  size_t off_tmark = 0;  // grid CTQW strips: marked-window flag per strip
  size_t off_coin = 0;   // Fourier / matrix coin
  bool has_coin = false;
  size_t off_sqrtp = 0;  // Szegedy coin weights
  bool has_sqrtp = false;
  bool has_col = false, has_rev = false, has_tiles = false, has_perm = false, has_tmark = false;
  // device binding
  unsigned char *d_graph = nullptr;
  qwk::GraphView view;
  // workspace layout
  size_t state_bytes = 0, off_w1 = 0, off_w2 = 0, off_pscratch = 0, off_partials = 0, work_bytes = 0;
  // staggered walk: tessellation descriptors (offsets into the device buffer),
  // where their array sits, and the workspace of big-polygon partial sums
  std::vector<qwk::StagTess> stag;
  size_t off_stag = 0, off_stagpart = 0;
  int32_t strip_rows = 0;   // grid CTQW blocked kernel: core rows per strip
  int32_t two_reg = 0;      // one-workgroup coined walk in one wavefront's registers: 0 no, 1 permutes, 2 cycle shifts
  int32_t block_depth = 1;  // grid CTQW: Horner stages per launch (temporal blocking)
  // out-of-core binding (qw_plan_upload_streamed): the CSR neighbour table stays
  // in caller-pinned host memory.  Ring mode streams it, tile by tile, through
  // a ring of device slots on the plan's copy stream while the stage kernels
  // run; direct mode keeps a prefix of it on the device and the stage kernel
  // reads the rest from host memory itself.
  bool streamed = false;
  int32_t st_mode = 0;              // QW_STREAM_DIRECT or QW_STREAM_RING
  const int32_t *h_col = nullptr;   // pinned host copy of col (CSR order)
  const int32_t *h_col_dev = nullptr;  // the same memory as the device addresses it
  int32_t *d_wg_row = nullptr;      // direct: workgroup tiles' first rows (n_wg + 1)
  int64_t st_n_wg = 0;
  int32_t *d_prefix = nullptr;      // direct: col[0, st_split) on the device
  int64_t st_split = 0;
  std::vector<int32_t> st_row;      // tile t holds rows [st_row[t], st_row[t+1])
  std::vector<int64_t> st_arc;      // and arcs [st_arc[t], st_arc[t+1])
  int32_t st_slots = 0;             // device slots in the ring
  int64_t st_slot_arcs = 0;         // neighbour indices per slot
  int32_t *d_ring = nullptr;
  hipStream_t st_copy = nullptr;
  std::vector<hipEvent_t> st_free, st_copied;  // per slot: its kernel finished / its copy landed
  qw_plan() = default;
  qw_plan(const qw_plan &) = delete;
  qw_plan &operator=(const qw_plan &) = delete;
  ~qw_plan();
};

namespace qwk {
// Host helpers shared by the plan and batch entry points (qw_host.cpp).
int set_error(int code, const char *fmt, ...);
int clear_error();
int plan_readout(const qw_plan *p, const void *psi, unsigned char *work, double *d_p, double *d_norm,
                 double *d_pmarked, hipStream_t s);
// Structured coined plans: slot-major `internal` -> boundary-order psi, with the readout fused.
int plan_struct_out(const qw_plan *p, const void *internal, void *psi, unsigned char *work, double *d_p,
                    double *d_norm, double *d_pmarked, hipStream_t s);
// Out-of-core CTQW evolution of a plan bound by qw_plan_upload_streamed (qw_stream.cpp).
int evolve_streamed(const qw_plan *p, void *psi, unsigned char *work, int64_t steps, double *d_p, double *d_norm,
                    double *d_pmarked, hipStream_t s);
// Release the out-of-core binding's copy stream and events.
void release_streamed(qw_plan *p);
}  // namespace qwk
