// Out-of-core evolution of CTQW plans: the qw_plan_stream_sizes /
// qw_plan_upload_streamed half of the C ABI.
//
// The paper names, as future work, splitting matrices larger than device
// memory into tiles (Sec. 5).  Here the operator's largest table, the CSR
// neighbour indices (4 bytes per arc), stays in caller-pinned host memory.
// The device keeps the state, the workspace, the row pointers and the marked
// set, plus a ring of slots that each hold the neighbour indices of one row
// tile.  Every Horner stage streams the tiles through the ring: a copy on the
// plan's copy stream fills a slot once the kernel that last read it has
// finished, and the stage kernel for that tile runs on the caller's stream
// once its copy has landed, so copies of later tiles overlap the kernels of
// earlier ones.  The stages of a step, and the steps, stay in order on the
// caller's stream.  The table does not change between stages, so the ring is
// also a cache: stages visit the tiles in alternating order (forward, then
// backward), each stage starts with the tiles the previous one ended with,
// and a tile already in a slot is not copied again (slots are reused least
// recently used first).  A stage then streams its table minus what the ring
// holds; a ring that holds every tile streams nothing after the first stage.
// The order of the tiles within a stage does not change any row's arithmetic.

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "qw_internal.h"
#include "qw_plan.h"
#include "qwalk.h"

using namespace qwk;

namespace {

constexpr int kSlots = 3;  // ring depth: one slot filling, one being read, one spare

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

struct Schedule {
  std::vector<int32_t> row;  // tile t: rows [row[t], row[t+1])
  std::vector<int64_t> arc;  // arcs [arc[t], arc[t+1])
  int64_t slot_arcs = 0;
  size_t rp_bytes = 0, bits_bytes = 0, mlist_bytes = 0, resident = 0, slot_stride = 0;
  size_t device_bytes = 0, host_bytes = 0;
};

int schedule(const qw_plan *p, size_t budget, Schedule *out) {
  if (!p) return set_error(QW_EINVAL, "null plan");
  if (p->kind != QW_CTQW || p->structure != kGeneral)
    return set_error(QW_EUNSUPPORTED, "out-of-core evolution needs a CTQW plan on the CSR path (QW_LAYOUT_CSR)");
  if (p->n == 0) return set_error(QW_EINVAL, "empty graph");
  Schedule &sc = *out;
  sc.rp_bytes = sizeof(int32_t) * static_cast<size_t>(p->n + 1);
  sc.bits_bytes = sizeof(uint32_t) * static_cast<size_t>((p->n + 31) / 32);
  sc.mlist_bytes = sizeof(int32_t) * static_cast<size_t>(std::max<int32_t>(p->n_marked, 1));
  sc.resident = align256(sc.rp_bytes) + align256(sc.bits_bytes) + align256(sc.mlist_bytes);
  const size_t walk = p->state_bytes + p->work_bytes;
  if (budget < walk + sc.resident + kSlots * 256)
    return set_error(QW_ENOMEM,
                     "device budget of %zu bytes is below the state, workspace and resident tables (%zu bytes)",
                     budget, walk + sc.resident + kSlots * 256);
  const size_t avail = budget - walk - sc.resident;
  int64_t slot_arcs = static_cast<int64_t>((avail / kSlots) & ~static_cast<size_t>(255)) / 4;
  slot_arcs = std::min<int64_t>(slot_arcs, std::max<int64_t>(64, (p->n_arcs + 63) / 64 * 64));
  if (slot_arcs < p->max_degree)
    return set_error(QW_ENOMEM, "device budget of %zu bytes leaves %lld neighbour indices per slot, below the "
                                "maximum degree %d", budget, static_cast<long long>(slot_arcs), p->max_degree);
  sc.slot_arcs = slot_arcs;
  sc.slot_stride = align256(sizeof(int32_t) * static_cast<size_t>(slot_arcs));
  const int32_t *rp = reinterpret_cast<const int32_t *>(p->image.data() + p->off_rp);
  sc.row.clear();
  sc.arc.clear();
  int64_t r = 0;
  while (r < p->n) {
    sc.row.push_back(static_cast<int32_t>(r));
    sc.arc.push_back(rp[r]);
    const int64_t a0 = rp[r];
    while (r < p->n && rp[r + 1] - a0 <= slot_arcs) ++r;
  }
  sc.row.push_back(static_cast<int32_t>(p->n));
  sc.arc.push_back(rp[p->n]);
  sc.device_bytes = sc.resident + kSlots * sc.slot_stride;
  sc.host_bytes = sizeof(int32_t) * static_cast<size_t>(std::max<int64_t>(p->n_arcs, 1));
  return QW_OK;
}

int dev_fail(hipError_t e, const char *what) {
  return set_error(QW_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define QW_TRY(expr, what)                           \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) return dev_fail(e_, what); \
  } while (0)

}  // namespace

qw_plan::~qw_plan() { release_streamed(this); }

namespace qwk {

void release_streamed(qw_plan *p) {
  for (hipEvent_t e : p->st_free) (void)hipEventDestroy(e);
  for (hipEvent_t e : p->st_copied) (void)hipEventDestroy(e);
  p->st_free.clear();
  p->st_copied.clear();
  if (p->st_copy) (void)hipStreamDestroy(p->st_copy);
  p->st_copy = nullptr;
  p->streamed = false;
  p->h_col = nullptr;
  p->d_ring = nullptr;
}

int evolve_streamed(const qw_plan *p, void *psi, unsigned char *work, int64_t steps, double *d_p, double *d_norm,
                    double *d_pmarked, hipStream_t s) {
  const bool c128 = p->dtype == QW_C128;
  const GraphView &g = p->view;
  const int K = p->K;
  if (steps > 0) {
    void *w0 = work, *w1 = work + p->off_w1;
    const int64_t tiles = static_cast<int64_t>(p->st_row.size()) - 1;
    const size_t stride = align256(sizeof(int32_t) * static_cast<size_t>(p->st_slot_arcs));
    // every slot starts free (and empty) once the caller's earlier work on `s` is done
    for (int i = 0; i < p->st_slots; ++i) QW_TRY(hipEventRecord(p->st_free[i], s), "ring event");
    std::vector<int64_t> held(p->st_slots, -1), used(p->st_slots, -1);  // tile in each slot, its last use
    int64_t q = 0, stage = 0;
    for (int64_t i = 0; i < steps; ++i) {
      const void *yin = psi;
      for (int k = K; k >= 1; --k, ++stage) {
        void *yout = (k == 1) ? (K == 1 ? w0 : psi) : (((K - k) & 1) ? w1 : w0);
        const double alpha = p->gamma * p->dt / k, beta = p->dt / k;
        for (int64_t j = 0; j < tiles; ++j, ++q) {
          const int64_t t = (stage & 1) ? tiles - 1 - j : j;
          int slot = -1;
          for (int x = 0; x < p->st_slots; ++x)
            if (held[x] == t) slot = x;
          int32_t *dst;
          if (slot >= 0) {
            // in the ring since an earlier stage: the kernels on `s` that read it
            // already waited for its copy, and no copy can refill the slot before
            // this kernel's free event
            dst = reinterpret_cast<int32_t *>(reinterpret_cast<unsigned char *>(p->d_ring) + slot * stride);
          } else {
            slot = 0;
            for (int x = 1; x < p->st_slots; ++x)
              if (used[x] < used[slot]) slot = x;
            dst = reinterpret_cast<int32_t *>(reinterpret_cast<unsigned char *>(p->d_ring) + slot * stride);
            const int64_t a0 = p->st_arc[t], na = p->st_arc[t + 1] - a0;
            QW_TRY(hipStreamWaitEvent(p->st_copy, p->st_free[slot], 0), "ring wait");
            if (na > 0)
              QW_TRY(hipMemcpyAsync(dst, p->h_col + a0, sizeof(int32_t) * static_cast<size_t>(na),
                                    hipMemcpyHostToDevice, p->st_copy),
                     "neighbour tile copy");
            QW_TRY(hipEventRecord(p->st_copied[slot], p->st_copy), "ring event");
            QW_TRY(hipStreamWaitEvent(s, p->st_copied[slot], 0), "ring wait");
            held[slot] = t;
          }
          used[slot] = q;
          QW_TRY(ctqw_slot_stage(c128, g, dst, p->st_arc[t], p->st_row[t], p->st_row[t + 1], yin, psi, yout, alpha,
                                 beta, s),
                 "out-of-core CTQW stage kernel");
          QW_TRY(hipEventRecord(p->st_free[slot], s), "ring event");
        }
        yin = yout;
      }
      if (K == 1) QW_TRY(copy_state(c128, p->n, w0, psi, s), "state copy kernel");
    }
  }
  if (!d_p && !d_norm && !d_pmarked) return QW_OK;
  return plan_readout(p, psi, work, d_p, d_norm, d_pmarked, s);
}

}  // namespace qwk

extern "C" {

int qw_plan_stream_sizes(const qw_plan *plan, size_t device_budget, size_t *host_bytes, size_t *device_bytes,
                         int64_t *n_tiles) {
  Schedule sc;
  const int st = schedule(plan, device_budget, &sc);
  if (st != QW_OK) return st;
  if (host_bytes) *host_bytes = sc.host_bytes;
  if (device_bytes) *device_bytes = sc.device_bytes;
  if (n_tiles) *n_tiles = static_cast<int64_t>(sc.row.size()) - 1;
  return clear_error();
}

int qw_plan_upload_streamed(qw_plan *p, size_t device_budget, void *h_pinned, size_t host_bytes, void *d_buf,
                            size_t device_bytes, void *stream) {
  if (!p || !h_pinned || !d_buf) return set_error(QW_EINVAL, "null plan or buffer");
  Schedule sc;
  try {
    const int st = schedule(p, device_budget, &sc);
    if (st != QW_OK) return st;
  } catch (const std::bad_alloc &) {
    return set_error(QW_ENOMEM, "host allocation failed");
  }
  if (host_bytes < sc.host_bytes)
    return set_error(QW_ENOMEM, "pinned host buffer of %zu bytes, the neighbour table needs %zu", host_bytes,
                     sc.host_bytes);
  if (device_bytes < sc.device_bytes)
    return set_error(QW_ENOMEM, "device buffer of %zu bytes, the streamed plan needs %zu", device_bytes,
                     sc.device_bytes);
  if (reinterpret_cast<uintptr_t>(d_buf) % 256 != 0) return set_error(QW_EINVAL, "device buffer not 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  release_streamed(p);
  p->d_graph = nullptr;
  auto *base = static_cast<unsigned char *>(d_buf);
  const size_t o_rp = 0, o_bits = align256(sc.rp_bytes), o_ml = o_bits + align256(sc.bits_bytes);
  QW_TRY(hipMemcpyAsync(base + o_rp, p->image.data() + p->off_rp, sc.rp_bytes, hipMemcpyHostToDevice, s),
         "row pointer upload");
  QW_TRY(hipMemcpyAsync(base + o_bits, p->image.data() + p->off_bits, sc.bits_bytes, hipMemcpyHostToDevice, s),
         "marked set upload");
  if (p->n_marked > 0)
    QW_TRY(hipMemcpyAsync(base + o_ml, p->image.data() + p->off_mlist, sizeof(int32_t) * p->n_marked,
                          hipMemcpyHostToDevice, s),
           "marked list upload");
  std::memcpy(h_pinned, p->image.data() + p->off_col, sizeof(int32_t) * static_cast<size_t>(p->n_arcs));
  QW_TRY(hipStreamCreateWithFlags(&p->st_copy, hipStreamNonBlocking), "copy stream");
  p->st_free.assign(kSlots, nullptr);
  p->st_copied.assign(kSlots, nullptr);
  for (int i = 0; i < kSlots; ++i) {
    QW_TRY(hipEventCreateWithFlags(&p->st_free[i], hipEventDisableTiming), "ring event");
    QW_TRY(hipEventCreateWithFlags(&p->st_copied[i], hipEventDisableTiming), "ring event");
  }
  GraphView &g = p->view;
  g = GraphView();
  g.n = static_cast<int32_t>(p->n);
  g.n_arcs = static_cast<int32_t>(p->n_arcs);
  g.structure = p->structure;
  g.n_marked = p->n_marked;
  g.group = p->group;
  g.rp = reinterpret_cast<const int32_t *>(base + o_rp);
  g.markbits = reinterpret_cast<const uint32_t *>(base + o_bits);
  g.marklist = reinterpret_cast<const int32_t *>(base + o_ml);
  g.base = base;
  p->h_col = static_cast<const int32_t *>(h_pinned);
  p->st_row = std::move(sc.row);
  p->st_arc = std::move(sc.arc);
  p->st_slots = kSlots;
  p->st_slot_arcs = sc.slot_arcs;
  p->d_ring = reinterpret_cast<int32_t *>(base + sc.resident);
  p->d_graph = base;
  p->streamed = true;
  return clear_error();
}

}  // extern "C"
